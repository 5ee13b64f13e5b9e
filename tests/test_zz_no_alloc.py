"""The allocation-free learned-guess solver (m2c_riemann_solve_learned_noalloc)
against the allocating entry point (m2c_riemann_solve_learned), called
through the C ABI on the same problems: two calls in a row, the second with a
smaller input, with the learned guess and with the acoustic one.  Both run
the same kernels, so the star states and Newton counts agree bit for bit."""
import ctypes as C
import os

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def env():
    import torch
    import paper_2508_16387_amd as m2c
    L = m2c.lib()
    net = m2c.Mlp(np.load(os.path.join(ROOT, "paper_2508_16387_amd", "learned_guess.npy")))
    return torch, m2c, L, net


def _problems(torch, seed, n):
    inp, eos = W.riemann_problem_set(seed, n)
    return (torch.tensor(inp.T.copy(), device="cuda"), torch.tensor(eos.T.copy(), device="cuda"))


def _noalloc(torch, L, net, di, de):
    n = di.shape[1]
    out = torch.full((4, n), -1.0, dtype=torch.float64, device="cuda")
    it = torch.full((n,), -7, dtype=torch.int32, device="cuda")
    s = torch.cuda.current_stream().cuda_stream
    rc = L.m2c_riemann_solve_learned_noalloc(None if net is None else net.h, n, di.data_ptr(), de.data_ptr(),
                                              1e-12, 50, out.data_ptr(), it.data_ptr(), s)
    assert rc == 0
    torch.cuda.synchronize()
    return out.cpu().numpy(), it.cpu().numpy()


def _alloc(torch, L, net, di, de):
    n = di.shape[1]
    out = torch.empty((4, n), dtype=torch.float64, device="cuda")
    it = torch.empty((n,), dtype=torch.int32, device="cuda")
    nfb = C.c_int64(0)
    s = torch.cuda.current_stream().cuda_stream
    rc = L.m2c_riemann_solve_learned(None if net is None else net.h, n, di.data_ptr(), de.data_ptr(), 1e-12, 50,
                                     out.data_ptr(), it.data_ptr(), C.byref(nfb), s)
    assert rc in (0, -3)            # -3: some problem without an admissible star pressure
    torch.cuda.synchronize()
    return out.cpu().numpy(), it.cpu().numpy()


@pytest.mark.parametrize("learned", [True, False], ids=["learned", "acoustic"])
def test_noalloc_matches_allocating_entry_point(env, learned):
    torch, m2c, L, net = env
    guess = net if learned else None
    for seed, n in ((2000, 300_000), (2001, 70_001)):          # second call smaller
        di, de = _problems(torch, seed, n)
        o_na, it_na = _noalloc(torch, L, guess, di, de)
        o_a, it_a = _alloc(torch, L, guess, di, de)
        assert np.array_equal(it_na, it_a), (seed, n)
        assert np.array_equal(np.isnan(o_na), np.isnan(o_a))
        ok = ~np.isnan(o_a)
        assert np.array_equal(o_na[ok], o_a[ok]), (seed, n)
        assert (it_a == 0).sum() > 0 and (it_a != 0).sum() > n // 2


def test_noalloc_rejects_oversize(env):
    torch, m2c, L, net = env
    n = m2c.NOALLOC_MAX_PROBLEMS + 1
    s = torch.cuda.current_stream().cuda_stream
    rc = L.m2c_riemann_solve_learned_noalloc(net.h, n, 1, 1, 1e-12, 50, 1, 1, s)   # rejected before any access
    assert rc == m2c.M2C_ERR_ARG
