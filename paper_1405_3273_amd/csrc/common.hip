// Context, errors, device buffers, the system set-up and small shared kernels.
#include "gf2_internal.h"

#include <cmath>
#include <cstdio>
#include <cstring>

namespace gf2 {

static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }

int fail(int code, const std::string &msg) {
    g_last_error = msg;
    return code;
}

int hip_fail(hipError_t e, const char *what, const char *file, int line) {
    char buf[512];
    std::snprintf(buf, sizeof(buf), "%s failed: %s (%s:%d)", what, hipGetErrorString(e), file,
                  line);
    g_last_error = buf;
    return e == hipErrorOutOfMemory ? GF2_ENOMEM : GF2_EHIP;
}

int DevBuf::ensure(size_t need) {
    if (need <= bytes && ptr) return GF2_OK;
    release();
    if (need == 0) need = 256;
    hipError_t e = hipMalloc(&ptr, need);
    if (e != hipSuccess) {
        ptr = nullptr;
        bytes = 0;
        (void)hipGetLastError();
        char buf[160];
        std::snprintf(buf, sizeof(buf), "hipMalloc of %zu bytes failed: %s", need,
                      hipGetErrorString(e));
        return fail(GF2_ENOMEM, buf);
    }
    bytes = need;
    return GF2_OK;
}

void DevBuf::release() {
    if (ptr) (void)hipFree(ptr);
    ptr = nullptr;
    bytes = 0;
}

// ---------------------------------------------------------------------------
// opt-in kernel timing

static hipEvent_t pool_get(gf2_ctx *c) {
    if (!c->prof_pool.empty()) {
        hipEvent_t e = c->prof_pool.back();
        c->prof_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

static void prof_resolve(gf2_ctx *c) {
    for (auto &p : c->prof_pending) {
        float ms = 0.0f;
        if (p.start && p.stop && hipEventSynchronize(p.stop) == hipSuccess &&
            hipEventElapsedTime(&ms, p.start, p.stop) == hipSuccess) {
            c->prof_ms[p.cls] += ms;
            c->prof_n[p.cls] += 1;
            c->prof_work[p.cls] += p.work;
        }
        if (p.start) c->prof_pool.push_back(p.start);
        if (p.stop) c->prof_pool.push_back(p.stop);
    }
    c->prof_pending.clear();
}

int prof_begin(gf2_ctx *c, int cls) {
    if (!c->prof) return -1;
    if (c->prof_pending.size() >= 8192) prof_resolve(c);
    gf2_prof_pending p{cls, pool_get(c), pool_get(c), 0.0};
    if (!p.start || !p.stop) return -1;
    (void)hipEventRecord(p.start, c->stream);
    c->prof_pending.push_back(p);
    return (int)c->prof_pending.size() - 1;
}

void prof_end(gf2_ctx *c, int handle, double work) {
    if (handle < 0 || handle >= (int)c->prof_pending.size()) return;
    auto &p = c->prof_pending[handle];
    p.work = work;
    (void)hipEventRecord(p.stop, c->stream);
}

void prof_release(gf2_ctx *c) {
    (void)hipStreamSynchronize(c->stream);
    prof_resolve(c);
    for (hipEvent_t e : c->prof_pool) (void)hipEventDestroy(e);
    c->prof_pool.clear();
}

// ---------------------------------------------------------------------------
// small kernels

__global__ void k_axpby(size_t n, double a, const double *__restrict__ x, double b,
                        double *__restrict__ y) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        y[i] = a * x[i] + b * y[i];
}

constexpr int RED_BLOCKS = 256;
constexpr int RED_THREADS = 256;

// op 0: max |a-b|; op 1: count of non-finite a; op 2: sum a*b
template <int OP>
__global__ __launch_bounds__(RED_THREADS) void k_reduce1(size_t n, const double *__restrict__ a,
                                                         const double *__restrict__ b,
                                                         double *__restrict__ part) {
    __shared__ double sh[RED_THREADS];
    double acc = 0.0;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x) {
        if (OP == 0) acc = fmax(acc, fabs(a[i] - b[i]));
        if (OP == 1) acc += isfinite(a[i]) ? 0.0 : 1.0;
        if (OP == 2) acc += a[i] * b[i];
    }
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int s = RED_THREADS / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            if (OP == 0) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + s]);
            else sh[threadIdx.x] += sh[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

template <int OP>
__global__ __launch_bounds__(RED_THREADS) void k_reduce2(const double *__restrict__ part,
                                                         double *__restrict__ out) {
    __shared__ double sh[RED_THREADS];
    sh[threadIdx.x] = part[threadIdx.x];
    __syncthreads();
    for (int s = RED_THREADS / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            if (OP == 0) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + s]);
            else sh[threadIdx.x] += sh[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = sh[0];
}

static_assert(RED_BLOCKS == RED_THREADS, "second pass reduces one value per thread");

template <int OP>
static int reduce_to_host(gf2_ctx *c, size_t n, const double *a, const double *b, double *out) {
    GF2_TRY(c->it_tmp.ensure((RED_BLOCKS + 8) * sizeof(double)));
    double *part = c->it_tmp.as<double>();
    hipLaunchKernelGGL(k_reduce1<OP>, dim3(RED_BLOCKS), dim3(RED_THREADS), 0, c->stream, n, a, b,
                       part);
    hipLaunchKernelGGL(k_reduce2<OP>, dim3(1), dim3(RED_THREADS), 0, c->stream, part,
                       part + RED_BLOCKS);
    GF2_HIP(hipGetLastError());
    GF2_HIP(hipMemcpyAsync(out, part + RED_BLOCKS, sizeof(double), hipMemcpyDeviceToHost,
                           c->stream));
    GF2_HIP(hipStreamSynchronize(c->stream));
    return GF2_OK;
}

int copy_d2d(gf2_ctx *c, void *dst, const void *src, size_t bytes) {
    if (dst == src || bytes == 0) return GF2_OK;
    GF2_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, c->stream));
    return GF2_OK;
}

__global__ void k_zero(size_t n, double *y) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        y[i] = 0.0;
}

int fill_zero(gf2_ctx *c, void *dst, size_t bytes) {
    size_t n = bytes / sizeof(double);
    if (n == 0) return GF2_OK;
    unsigned blocks = (unsigned)std::min<size_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_zero, dim3(blocks), dim3(256), 0, c->stream, n, (double *)dst);
    GF2_HIP(hipGetLastError());
    return GF2_OK;
}

int axpby(gf2_ctx *c, size_t n, double a, const double *x, double b, double *y) {
    unsigned blocks = (unsigned)std::min<size_t>((n + 255) / 256, 4096);
    if (blocks == 0) return GF2_OK;
    hipLaunchKernelGGL(k_axpby, dim3(blocks), dim3(256), 0, c->stream, n, a, x, b, y);
    GF2_HIP(hipGetLastError());
    return GF2_OK;
}

int max_abs_diff(gf2_ctx *c, size_t n, const double *a, const double *b, double *out) {
    return reduce_to_host<0>(c, n, a, b, out);
}

int any_nonfinite(gf2_ctx *c, size_t n, const double *x, int *out) {
    double cnt = 0.0;
    GF2_TRY(reduce_to_host<1>(c, n, x, x, &cnt));
    *out = cnt > 0.0 ? 1 : 0;
    return GF2_OK;
}

int dot(gf2_ctx *c, size_t n, const double *a, const double *b, double *out) {
    return reduce_to_host<2>(c, n, a, b, out);
}

// C = A B for small n x n FP64 matrices: one thread per output element.
__global__ void k_matmul_nn(int n, const double *__restrict__ A, const double *__restrict__ B,
                            double *__restrict__ C) {
    int i = blockIdx.y;
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || j >= n) return;
    double s = 0.0;
    for (int k = 0; k < n; ++k) s += A[(size_t)i * n + k] * B[(size_t)k * n + j];
    C[(size_t)i * n + j] = s;
}

int matmul_nn(gf2_ctx *c, int n, const double *A, const double *B, double *C) {
    dim3 grid((n + 63) / 64, n);
    hipLaunchKernelGGL(k_matmul_nn, grid, dim3(64), 0, c->stream, n, A, B, C);
    GF2_HIP(hipGetLastError());
    return GF2_OK;
}

// trigamma(x) = sum_{k>=0} 1/(x+k)^2: recurrence up to x >= 12, then the
// asymptotic series 1/x + 1/(2x^2) + sum B_2k / x^(2k+1).
double trigamma(double x) {
    double acc = 0.0;
    while (x < 12.0) {
        acc += 1.0 / (x * x);
        x += 1.0;
    }
    const double ix = 1.0 / x, ix2 = ix * ix;
    // Bernoulli numbers B2=1/6, B4=-1/30, B6=1/42, B8=-1/30, B10=5/66, B12=-691/2730
    double series = ix + 0.5 * ix2 +
                    ix * ix2 *
                        (1.0 / 6.0 +
                         ix2 * (-1.0 / 30.0 +
                                ix2 * (1.0 / 42.0 +
                                       ix2 * (-1.0 / 30.0 + ix2 * (5.0 / 66.0 +
                                                                   ix2 * (-691.0 / 2730.0))))));
    return acc + series;
}

// Gauss-Jordan inverse with partial pivoting on the host (n small, once per system).
static bool host_inverse(int n, const std::vector<double> &A_in, std::vector<double> &Ainv) {
    std::vector<double> A(A_in);
    Ainv.assign((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) Ainv[(size_t)i * n + i] = 1.0;
    double scale = 0.0;
    for (double x : A) scale = std::fmax(scale, std::fabs(x));
    for (int k = 0; k < n; ++k) {
        int r = k;
        for (int i = k + 1; i < n; ++i)
            if (std::fabs(A[(size_t)i * n + k]) > std::fabs(A[(size_t)r * n + k])) r = i;
        double piv = A[(size_t)r * n + k];
        if (!(std::fabs(piv) > 1e-14 * scale)) return false;
        if (r != k) {
            for (int j = 0; j < n; ++j) {
                std::swap(A[(size_t)r * n + j], A[(size_t)k * n + j]);
                std::swap(Ainv[(size_t)r * n + j], Ainv[(size_t)k * n + j]);
            }
        }
        double ip = 1.0 / piv;
        for (int j = 0; j < n; ++j) {
            A[(size_t)k * n + j] *= ip;
            Ainv[(size_t)k * n + j] *= ip;
        }
        for (int i = 0; i < n; ++i) {
            if (i == k) continue;
            double f = A[(size_t)i * n + k];
            if (f == 0.0) continue;
            for (int j = 0; j < n; ++j) {
                A[(size_t)i * n + j] -= f * A[(size_t)k * n + j];
                Ainv[(size_t)i * n + j] -= f * Ainv[(size_t)k * n + j];
            }
        }
    }
    return true;
}

}  // namespace gf2

using namespace gf2;

extern "C" {

const char *gf2_last_error(void) { return g_last_error.c_str(); }

int gf2_ctx_create(gf2_ctx **out, int device, void *stream) {
    if (!out) return fail(GF2_EINVAL, "gf2_ctx_create: ctx pointer is NULL");
    *out = nullptr;
    int ndev = 0;
    GF2_HIP(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev) return fail(GF2_EINVAL, "gf2_ctx_create: bad device");
    GF2_HIP(hipSetDevice(device));
    gf2_ctx *c = new (std::nothrow) gf2_ctx();
    if (!c) return fail(GF2_ENOMEM, "gf2_ctx_create: out of host memory");
    c->device = device;
    c->stream = static_cast<hipStream_t>(stream);
    *out = c;
    set_error("");
    return GF2_OK;
}

int gf2_ctx_destroy(gf2_ctx *c) {
    if (!c) return GF2_OK;
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    prof_release(c);
    sigma_release(c);
    dyson_round_release(c);
    gf2::DevBuf *bufs[] = {&c->S,        &c->Sinv,      &c->h,       &c->v,        &c->v_32,
                           &c->W2_64,    &c->W2_32,     &c->W2_b3,   &c->sig_T1,   &c->sig_X,    &c->sig_Gp,  &c->sig_Gq,
                           &c->sig_G,    &c->sig_Gb,    &c->sig_part, &c->four_c,  &c->four_C,
                           &c->four_fold, &c->four_twid, &c->dys_part, &c->dys_X,   &c->dys_aux,
                           &c->dys_out,  &c->fock_part, &c->occ_ws, &c->grid_tau, &c->grid_thom, &c->grid_W, &c->grid_T,
                           &c->grid_coef, &c->grid_plan, &c->it_Sig_iw, &c->it_G_iw, &c->it_Sig1,
                           &c->it_mom,   &c->it_Sig_new, &c->it_Pout, &c->it_Pin,  &c->it_F,
                           &c->it_tmp,   &c->it_hist,   &c->bat_tab,  &c->bat_boff,
                           &c->bat_out,  &c->sig_tab,  &c->it_red,  &c->bat_red,
                           &c->df_B64,   &c->df_Bt64,   &c->df_B32,   &c->df_Bt32,
                           &c->df_ws,    &c->df_T,      &c->df_part};
    for (auto *b : bufs) b->release();
    if (c->bat_red_h) (void)hipHostFree(c->bat_red_h);
    delete c;
    return GF2_OK;
}

int gf2_set_system(gf2_ctx *c, int n, const double *S, const double *h, const double *v) {
    if (!c) return fail(GF2_EINVAL, "gf2_set_system: ctx is NULL");
    if (n < 1) return fail(GF2_EINVAL, "gf2_set_system: n must be >= 1");
    if (!S || !h || !v) return fail(GF2_EINVAL, "gf2_set_system: NULL array");
    GF2_HIP(hipSetDevice(c->device));
    const size_t n2 = (size_t)n * n, n4 = n2 * n2;
    c->has_system = false;
    c->df_m = 0;
    c->have_f32_layouts = false;
    c->have_bf3_layouts = false;
    c->n = n;
    GF2_TRY(c->S.ensure(n2 * 8));
    GF2_TRY(c->Sinv.ensure(n2 * 8));
    GF2_TRY(c->h.ensure(n2 * 8));
    GF2_TRY(c->v.ensure(n4 * 8));
    GF2_TRY(copy_d2d(c, c->S.ptr, S, n2 * 8));
    GF2_TRY(copy_d2d(c, c->h.ptr, h, n2 * 8));
    GF2_TRY(copy_d2d(c, c->v.ptr, v, n4 * 8));
    c->S_host.resize(n2);
    c->h_host.resize(n2);
    GF2_HIP(hipMemcpyAsync(c->S_host.data(), S, n2 * 8, hipMemcpyDeviceToHost, c->stream));
    GF2_HIP(hipMemcpyAsync(c->h_host.data(), h, n2 * 8, hipMemcpyDeviceToHost, c->stream));
    GF2_HIP(hipStreamSynchronize(c->stream));
    if (!host_inverse(n, c->S_host, c->Sinv_host))
        return fail(GF2_EINVAL, "gf2_set_system: S is singular");
    GF2_HIP(hipMemcpyAsync(c->Sinv.ptr, c->Sinv_host.data(), n2 * 8, hipMemcpyHostToDevice,
                           c->stream));
    GF2_TRY(sigma_build_layouts(c, true));
    GF2_HIP(hipStreamSynchronize(c->stream));
    c->has_system = true;
    return GF2_OK;
}

int gf2_profile_enable(gf2_ctx *c, int on) {
    if (!c) return fail(GF2_EINVAL, "gf2_profile_enable: ctx is NULL");
    GF2_HIP(hipSetDevice(c->device));
    GF2_HIP(hipStreamSynchronize(c->stream));
    prof_resolve(c);
    if (on) {
        for (int k = 0; k < GF2_KC_COUNT; ++k) {
            c->prof_ms[k] = 0.0;
            c->prof_n[k] = 0;
            c->prof_work[k] = 0.0;
        }
    }
    c->prof = on != 0;
    return GF2_OK;
}

int gf2_profile_read(gf2_ctx *c, int nslots, double *ms, long long *launches, double *work) {
    if (!c || nslots < 0 || nslots > GF2_KC_COUNT) return fail(GF2_EINVAL, "gf2_profile_read: bad argument");
    GF2_HIP(hipSetDevice(c->device));
    GF2_HIP(hipStreamSynchronize(c->stream));
    prof_resolve(c);
    for (int k = 0; k < nslots; ++k) {
        if (ms) ms[k] = c->prof_ms[k];
        if (launches) launches[k] = c->prof_n[k];
        if (work) work[k] = c->prof_work[k];
    }
    return GF2_OK;
}

}  // extern "C"
