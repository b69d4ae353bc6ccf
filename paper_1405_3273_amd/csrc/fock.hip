// Eq. (FockMatrix): F_ij = h_ij + sum_kl P_kl (v_ijlk - v_iklj / 2)  (FP64).
//
// One pass over v.  Block (i, a-slice) streams the contiguous slab
// v[i][a][b][c] for its a-range; thread c accumulates
//   K_i[c] += v[i][a][b][c] P[a][b]    (v_iabc = v_{i k=a l=b j=c})
// and each a gives
//   J[i][a] = sum_{b,c} v[i][a][b][c] P[c][b]   (v_{i j=a l=b k=c})
// by a block reduction.  Partial K over a-slices are added in a fixed order.
#include "gf2_internal.h"

#include <algorithm>

namespace gf2 {

constexpr int FK_THREADS = 256;
constexpr int FK_ASPLIT = 8;

__global__ __launch_bounds__(FK_THREADS) void k_fock_jk(int n, const double *__restrict__ v,
                                                        const double *__restrict__ P,
                                                        double *__restrict__ J,
                                                        double *__restrict__ Kpart) {
    const int i = blockIdx.x;
    const int slice = blockIdx.y;
    const int per = (n + FK_ASPLIT - 1) / FK_ASPLIT;
    const int a0 = slice * per, a1 = min(n, a0 + per);
    __shared__ double red[FK_THREADS / 64];
    const size_t n2 = (size_t)n * n, n3 = n2 * n;
    // threads stride over c in chunks of FK_THREADS (n may exceed the block)
    for (int c0 = 0; c0 < n; c0 += FK_THREADS) {
        const int c = c0 + threadIdx.x;
        double kacc = 0.0;
        for (int a = a0; a < a1; ++a) {
            double jp = 0.0;
            if (c < n) {
                const double *row = v + (size_t)i * n3 + (size_t)a * n2;
                for (int b = 0; b < n; ++b) {
                    const double x = row[(size_t)b * n + c];
                    kacc += x * P[(size_t)a * n + b];
                    jp += x * P[(size_t)c * n + b];
                }
            }
            for (int off = 32; off > 0; off >>= 1) jp += __shfl_down(jp, off);
            if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = jp;
            __syncthreads();
            if (threadIdx.x == 0) {
                double s = 0.0;
                for (int t = 0; t < FK_THREADS / 64; ++t) s += red[t];
                if (c0 == 0) J[(size_t)i * n + a] = s;
                else J[(size_t)i * n + a] += s;
            }
            __syncthreads();
        }
        if (c < n) Kpart[(size_t)slice * n2 + (size_t)i * n + c] = kacc;
    }
}

__global__ void k_fock_sum(int n, int nslice, const double *__restrict__ h,
                           const double *__restrict__ J, const double *__restrict__ Kpart,
                           double *__restrict__ F) {
    const size_t n2 = (size_t)n * n;
    const size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    if (e >= n2) return;
    double k = 0.0;
    for (int s = 0; s < nslice; ++s) k += Kpart[s * n2 + e];
    F[e] = h[e] + J[e] - 0.5 * k;
}

int fock_run(gf2_ctx *c, const double *P, double *F) {
    const int n = c->n;
    const size_t n2 = (size_t)n * n;
    GF2_TRY(c->fock_part.ensure((FK_ASPLIT + 1) * n2 * 8));
    double *J = c->fock_part.as<double>();
    double *Kp = J + n2;
    const int ph = prof_begin(c, GF2_KC_FOCK);
    hipLaunchKernelGGL(k_fock_jk, dim3(n, FK_ASPLIT), dim3(FK_THREADS), 0, c->stream, n,
                       c->v.as<double>(), P, J, Kp);
    prof_end(c, ph, 8.0 * (double)n2 * n2);
    // every slice writes its K partial (zero for an empty a-range)
    hipLaunchKernelGGL(k_fock_sum, dim3((unsigned)((n2 + 255) / 256)), dim3(256), 0, c->stream, n,
                       FK_ASPLIT, c->h.as<double>(), J, Kp, F);
    GF2_HIP(hipGetLastError());
    return GF2_OK;
}

}  // namespace gf2

using namespace gf2;

extern "C" int gf2_fock(gf2_ctx *c, const double *P, double *F) {
    if (!c || !P || !F) return fail(GF2_EINVAL, "gf2_fock: NULL argument");
    if (!c->has_system) return fail(GF2_ESTATE, "gf2_fock: no system set");
    if (P == F) return fail(GF2_EINVAL, "gf2_fock: F aliases P");
    GF2_HIP(hipSetDevice(c->device));
    return fock_run(c, P, F);
}
