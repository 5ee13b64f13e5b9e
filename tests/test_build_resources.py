"""Register and LDS budget of the stage kernels (compile-time, no GPU).

The FP64 stage kernels are sized for two waves per SIMD without private-
memory spills; the mixed-precision ones for three waves per SIMD, also
without spills.  A change
that silently pushes a kernel past its budget (spills to scratch, or a drop
in occupancy) costs far more than it saves, so the compiler's own resource
report is checked here."""
from __future__ import annotations

import os
import re
import shutil
import subprocess

import pytest

from paper_2508_16387_amd import build as B

HIPCC = B.hipcc()


SOURCES = ("k_stage.hip", "k_stage_eos.hip", "k_stage_eos_nasg.hip", "k_stage_eos_other.hip", "k_stage_opts.hip",
           "k_riemann_eos.hip")


def _parse(stderr):
    out = {}
    name = None
    for line in stderr.splitlines():
        m = re.search(r"Function Name: (\S+)", line)
        if m:
            name = m.group(1)
            out[name] = {}
            continue
        for key, pat in (("vgpr", r"VGPRs: (\d+)"), ("agpr", r"AGPRs: (\d+)"),
                         ("scratch", r"ScratchSize \[bytes/lane\]: (\d+)"),
                         ("occupancy", r"Occupancy \[waves/SIMD\]: (\d+)"),
                         ("lds", r"LDS Size \[bytes/block\]: (\d+)")):
            m = re.search(pat, line)
            if m and name:
                out[name][key] = int(m.group(1))
    return out


@pytest.fixture(scope="module")
def all_resources(tmp_path_factory):
    """The compiler's resource report of the three stage-kernel sources,
    compiled side by side."""
    if not os.path.exists(HIPCC) and not shutil.which("hipcc"):
        pytest.skip("hipcc not available")
    d = tmp_path_factory.mktemp("res")
    procs = {}
    for src in SOURCES:
        procs[src] = subprocess.Popen([HIPCC, *B.flags_for(src), "-c", os.path.join(B.CSRC, src), "-o", str(d / (src + ".o")),
                                       "-Rpass-analysis=kernel-resource-usage"],
                                      stdout=subprocess.DEVNULL, stderr=subprocess.PIPE, text=True)
    out = {}
    for src, p in procs.items():
        err = p.communicate()[1]
        assert p.returncode == 0, err[-2000:]
        out[src] = _parse(err)
    return out


@pytest.fixture(scope="module")
def stage_resources(all_resources):
    return all_resources["k_stage.hip"]


@pytest.fixture(scope="module")
def stage_eos_resources(all_resources):
    out = {}
    for src in ("k_stage_eos.hip", "k_stage_eos_nasg.hip", "k_stage_eos_other.hip"):
        out.update(all_resources[src])
    return out


@pytest.fixture(scope="module")
def stage_opts_resources(all_resources):
    return all_resources["k_stage_opts.hip"]


# the 64x2 tile exists for quasi-1D grids only; its budget is not tuned
TUNED = ("Li16ELi16E", "Li32ELi8E", "Li16ELi15E", "Li32ELi7E")


def test_fp64_stage_kernels_fit_two_waves_without_spills(stage_resources):
    ks = {n: r for n, r in stage_resources.items() if "k_stage" in n and "Ed" in n and any(t in n for t in TUNED)}
    assert len(ks) == 24, sorted(ks)            # 4 stage kinds single-grid + 2 batched, 4 tiles
    for n, r in ks.items():
        assert r["scratch"] == 0, (n, r)
        assert r["agpr"] == 0, (n, r)
        assert r["occupancy"] >= 2, (n, r)
        assert 2 * r["lds"] <= 160 * 1024, (n, r)


def test_mixed_stage_kernels_keep_three_waves_without_spills(stage_resources):
    ks = {n: r for n, r in stage_resources.items() if "k_stage" in n and "Ef" in n and any(t in n for t in TUNED)}
    assert len(ks) == 24, sorted(ks)
    for n, r in ks.items():
        assert r["scratch"] == 0, (n, r)
        assert r["occupancy"] >= 3, (n, r)
        assert r["vgpr"] + r["agpr"] <= 168, (n, r)


def test_general_eos_stage_kernels_fit_two_waves_without_spills(stage_eos_resources):
    """The general-EOS stage kernels on the 16x15 tile (the default scheme
    for each of the six sets of one or two families, and the run-time
    options): no scratch and two waves per SIMD for every stage kind (holding
    W^n across the plane iteration pushed kinds 2 and 3 to one wave)."""
    ks = {n: r for n, r in stage_eos_resources.items() if "k_stage" in n and "Li16ELi15E" in n}
    assert len(ks) == 4 * (6 + 1), sorted(ks)   # 4 stage kinds x (6 family sets + run-time options)
    for n, r in ks.items():
        assert r["scratch"] == 0, (n, r)
        assert r["occupancy"] >= 2, (n, r)


def test_general_eos_point_solvers_per_family_pair(all_resources):
    """The point solver compiled per unordered family pair: no spills but 32
    bytes per lane for Mie-Grueneisen on both sides (the run-time dispatching
    kernel, kept for sets of several family pairs, spills), two waves per
    SIMD without Mie-Grueneisen."""
    ks = {n: r for n, r in all_resources["k_riemann_eos.hip"].items() if "k_riemann_eosILi" in n and "Lin1" not in n}
    assert len(ks) == 6, sorted(ks)
    for n, r in ks.items():
        mg = "Li1E" in n
        assert r["scratch"] <= (32 if mg else 28), (n, r)
        if not mg:
            assert r["occupancy"] >= 2, (n, r)


def test_option_stage_kernels_fit_two_waves_without_spills(stage_opts_resources):
    """The run-time option kernels (limiter, flux, band) in FP64 on the
    16x16 tile: two waves per SIMD without scratch for every stage kind."""
    ks = {n: r for n, r in stage_opts_resources.items() if "k_stage" in n and "Li16ELi16EdLb1" in n}
    assert len(ks) == 4, sorted(ks)
    for n, r in ks.items():
        assert r["scratch"] == 0, (n, r)
        assert r["occupancy"] >= 2, (n, r)
