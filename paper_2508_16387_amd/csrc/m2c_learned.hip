// m2c_learned.hip -- host side of the learned star-pressure guess: the
// network object, feature extraction, inference, gradient, the Adam
// training loop and the learned-guess Riemann solver (include/m2c.h).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/m2c.h"
#include "m2c_internal.h"
#include "m2c_kernels.h"
#include "m2c_mlp.h"

using namespace m2c;

struct m2c_mlp {
    int device = 0;
    MlpDev d{};
};

const MlpDev* m2c_mlp_dev(const m2c_mlp* m) { return m ? &m->d : nullptr; }

// Scratch of the allocation-free solver: one learned guess per problem and
// the two counters the solve kernel updates (no admissible star pressure,
// acoustic starts).  One copy per GPU, held until the process ends; every
// call on a GPU shares its copy, so calls that overlap on one GPU race.
constexpr long long NOALLOC_MAX = M2C_NOALLOC_MAX_PROBLEMS;
static __device__ __align__(256) double scratch[NOALLOC_MAX + 2];

namespace {

constexpr int MAX_DEVICES = 64;
std::mutex scratch_mu;
double* scratch_ptr[MAX_DEVICES] = {};

// Device address of this GPU's scratch (the array's name is only a
// host-side handle).  Looked up once per device, with that device current.
hipError_t scratch_of_current_device(double** out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (!scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        scratch_ptr[dev] = static_cast<double*>(p);
    }
    *out = scratch_ptr[dev];
    return hipSuccess;
}

}  // namespace

namespace {

// Glorot-uniform initial weights from SplitMix64 (Steele, Lea and Flood).
struct SplitMix {
    uint64_t s;
    double uniform()
    {
        s += 0x9E3779B97F4A7C15ull;
        uint64_t z = s;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        z ^= z >> 31;
        return (double)(z >> 11) * (1.0 / 9007199254740992.0);
    }
};

void glorot(std::vector<float>& p, uint64_t seed)
{
    SplitMix r{seed};
    p.assign(MLP_NPARAM, 0.0f);
    auto fill = [&](int off, int n, double lim) {
        for (int i = 0; i < n; ++i) p[off + i] = (float)((2.0 * r.uniform() - 1.0) * lim);
    };
    fill(MLP_OFF_W1, 512, std::sqrt(6.0 / (MLP_H + MLP_IN)));
    fill(MLP_OFF_W2, 4096, std::sqrt(6.0 / (MLP_H + MLP_H)));
    fill(MLP_OFF_W3, 64, std::sqrt(6.0 / (MLP_H + 1)));
}

}  // namespace

extern "C" {

void m2c_train_opts_default(m2c_train_opts* o)
{
    if (!o) return;
    memset(o, 0, sizeof(*o));
    o->struct_size = sizeof(m2c_train_opts);
    o->epochs = 20;
    o->batch = 4096;
    o->lr = 3e-3f;
    o->lr_final = 1e-4f;
    o->beta1 = 0.9f;
    o->beta2 = 0.999f;
    o->eps = 1e-8f;
}

void m2c_mlp_destroy(m2c_mlp* m)
{
    if (!m) return;
    (void)hipSetDevice(m->device);
    (void)hipFree(m->d.master);
    (void)hipFree(m->d.wbf);
    delete m;
}

int m2c_mlp_create(const float* params, uint64_t seed, m2c_mlp** out)
{
    if (!out) return M2C_ERR_ARG;
    *out = nullptr;
    std::vector<float> p;
    if (params) p.assign(params, params + MLP_NPARAM);
    else glorot(p, seed);
    m2c_mlp* m = new (std::nothrow) m2c_mlp();
    if (!m) return M2C_ERR_NOMEM;
    if (hipGetDevice(&m->device) != hipSuccess || hipMalloc((void**)&m->d.master, MLP_NPARAM * sizeof(float)) != hipSuccess ||
        hipMalloc((void**)&m->d.wbf, MLP_NBF * sizeof(uint16_t)) != hipSuccess) {
        m2c_mlp_destroy(m);
        return M2C_ERR_NOMEM;
    }
    if (hipMemcpy(m->d.master, p.data(), MLP_NPARAM * sizeof(float), hipMemcpyHostToDevice) != hipSuccess ||
        launch_mlp_sync(m->d, nullptr) != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
        m2c_mlp_destroy(m);
        return M2C_ERR_DEVICE;
    }
    *out = m;
    return M2C_OK;
}

int m2c_mlp_get_params(const m2c_mlp* m, float* params)
{
    if (!m || !params) return M2C_ERR_ARG;
    if (hipSetDevice(m->device) != hipSuccess ||
        hipMemcpy(params, m->d.master, MLP_NPARAM * sizeof(float), hipMemcpyDeviceToHost) != hipSuccess)
        return M2C_ERR_DEVICE;
    return M2C_OK;
}

int m2c_mlp_features(int64_t n, const double* in, const double* eos, const double* pstar, float* X8, float* target,
                     void* stream)
{
    if (n < 0 || (n > 0 && (!in || !eos || !X8))) return M2C_ERR_ARG;
    if (n == 0) return M2C_OK;
    if (launch_mlp_features(n, in, eos, pstar, X8, target, (hipStream_t)stream) != hipSuccess) return M2C_ERR_DEVICE;
    return M2C_OK;
}

int m2c_mlp_forward(const m2c_mlp* m, int64_t n, const float* X8, float* y, void* stream)
{
    if (!m || n < 0 || (n > 0 && (!X8 || !y))) return M2C_ERR_ARG;
    if (n == 0) return M2C_OK;
    if (launch_mlp_forward(n, X8, m->d, y, (hipStream_t)stream) != hipSuccess) return M2C_ERR_DEVICE;
    return M2C_OK;
}

int m2c_mlp_grad(const m2c_mlp* m, int64_t n, const float* X8, const float* t, float* grad, float* loss, void* stream)
{
    if (!m || n < 1 || !X8 || !t || !grad) return M2C_ERR_ARG;
    hipStream_t s = (hipStream_t)stream;
    float* dg = nullptr;
    if (hipMalloc((void**)&dg, (MLP_NPARAM + 1) * sizeof(float)) != hipSuccess) return M2C_ERR_NOMEM;
    int rc = M2C_OK;
    float sse = 0.0f;
    if (launch_fill_f32(dg, MLP_NPARAM + 1, 0.0f, s) != hipSuccess ||
        launch_mlp_grad(0, n, n, 1.0f / (float)n, X8, t, m->d, dg, dg + MLP_NPARAM, s) != hipSuccess ||
        hipMemcpyAsync(grad, dg, MLP_NPARAM * sizeof(float), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(&sse, dg + MLP_NPARAM, sizeof(float), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        rc = M2C_ERR_DEVICE;
    (void)hipFree(dg);
    if (loss) *loss = sse / (float)n;
    return rc;
}

int m2c_mlp_train(m2c_mlp* m, int64_t n, const float* X8, const float* t, const m2c_train_opts* o,
                  float* loss_per_epoch, void* stream)
{
    if (!m || n < 1 || !X8 || !t || !o || o->struct_size != sizeof(m2c_train_opts)) return M2C_ERR_ARG;
    if (o->epochs < 1 || o->batch < 16 || !(o->lr > 0.0f) || !(o->lr_final > 0.0f)) return M2C_ERR_ARG;
    hipStream_t s = (hipStream_t)stream;
    float* buf = nullptr;                       // grad | m | v | sse
    const size_t nb = 3 * (size_t)MLP_NPARAM + 1;
    if (hipSetDevice(m->device) != hipSuccess) return M2C_ERR_DEVICE;
    if (hipMalloc((void**)&buf, nb * sizeof(float)) != hipSuccess) return M2C_ERR_NOMEM;
    float* grad = buf;
    float* mo = buf + MLP_NPARAM;
    float* ve = buf + 2 * MLP_NPARAM;
    float* sse = buf + 3 * MLP_NPARAM;
    int rc = launch_fill_f32(buf, (long long)nb, 0.0f, s) == hipSuccess ? M2C_OK : M2C_ERR_DEVICE;
    const long long B = o->batch;
    const long long nbatch = (n + B - 1) / B;
    const long long total = nbatch * o->epochs;
    long long step = 0;
    for (int ep = 0; ep < o->epochs && rc == M2C_OK; ++ep) {
        for (long long bi = 0; bi < nbatch && rc == M2C_OK; ++bi) {
            const long long i0 = bi * B, cnt = (i0 + B <= n) ? B : n - i0;
            ++step;
            const float lr = o->lr * std::pow(o->lr_final / o->lr, (float)(step - 1) / (float)(total > 1 ? total - 1 : 1));
            if (launch_mlp_grad(i0, cnt, n, 1.0f / (float)cnt, X8, t, m->d, grad, sse, s) != hipSuccess ||
                launch_adam(m->d, mo, ve, grad, lr, o->beta1, o->beta2, o->eps, (int)step, s) != hipSuccess)
                rc = M2C_ERR_DEVICE;
        }
        if (rc == M2C_OK && loss_per_epoch) {
            float h = 0.0f;
            if (hipMemcpyAsync(&h, sse, sizeof(float), hipMemcpyDeviceToHost, s) != hipSuccess ||
                hipStreamSynchronize(s) != hipSuccess || launch_fill_f32(sse, 1, 0.0f, s) != hipSuccess)
                rc = M2C_ERR_DEVICE;
            loss_per_epoch[ep] = h / (float)n;
        }
    }
    if (rc == M2C_OK && hipStreamSynchronize(s) != hipSuccess) rc = M2C_ERR_DEVICE;
    (void)hipFree(buf);
    return rc;
}

int m2c_riemann_solve_learned(const m2c_mlp* m, int64_t n, const double* in, const double* eos, double rtol,
                              int32_t maxit, double* out, int32_t* iters, int64_t* n_fallback, void* stream)
{
    if (n < 0 || (n > 0 && (!in || !eos || !out))) return M2C_ERR_ARG;
    if (!(rtol > 0.0) || maxit < 1) return M2C_ERR_ARG;
    if (n == 0) return M2C_OK;
    hipStream_t s = (hipStream_t)stream;
    double* g = nullptr;
    if (hipMalloc((void**)&g, n * sizeof(double) + 16) != hipSuccess) return M2C_ERR_NOMEM;
    int32_t* dvac = (int32_t*)(g + n);
    unsigned long long* dfb = (unsigned long long*)((char*)(g + n) + 8);
    int32_t hv = 0;
    unsigned long long hfb = 0;
    int rc = M2C_OK;
    if (hipMemsetAsync(dvac, 0, 16, s) != hipSuccess ||
        (m && launch_points_guess(n, in, eos, m->d, g, s) != hipSuccess) ||
        launch_riemann_points(n, in, eos, m ? g : nullptr, rtol, maxit, out, iters, dvac, dfb, s) != hipSuccess ||
        hipMemcpyAsync(&hv, dvac, sizeof(int32_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(&hfb, dfb, sizeof(hfb), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        rc = M2C_ERR_DEVICE;
    (void)hipFree(g);
    if (n_fallback) *n_fallback = (int64_t)hfb;
    if (rc == M2C_OK && hv > 0) rc = M2C_ERR_RIEMANN;
    return rc;
}

int m2c_riemann_solve_learned_noalloc(const m2c_mlp* m, int64_t n, const double* in, const double* eos, double rtol,
                                      int32_t maxit, double* out, int32_t* iters, void* stream)
{
    if (n < 0 || n > NOALLOC_MAX || (n > 0 && (!in || !eos || !out))) return M2C_ERR_ARG;
    if (!(rtol > 0.0) || maxit < 1) return M2C_ERR_ARG;
    if (n == 0) return M2C_OK;
    hipStream_t s = (hipStream_t)stream;
    double* ws = nullptr;
    if (scratch_of_current_device(&ws) != hipSuccess) return M2C_ERR_DEVICE;
    // guesses in ws[0, n); the counters after the largest guess array are
    // written by the solve kernel and read by no one, so they need no clearing
    int32_t* dvac = reinterpret_cast<int32_t*>(ws + NOALLOC_MAX);
    unsigned long long* dfb = reinterpret_cast<unsigned long long*>(ws + NOALLOC_MAX + 1);
    if ((m && launch_points_guess(n, in, eos, m->d, ws, s) != hipSuccess) ||
        launch_riemann_points(n, in, eos, m ? ws : nullptr, rtol, maxit, out, iters, dvac, dfb, s) != hipSuccess)
        return M2C_ERR_DEVICE;
    return M2C_OK;
}

}  // extern "C"
