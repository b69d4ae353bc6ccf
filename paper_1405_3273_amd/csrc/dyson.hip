// Eq. (GF): G(i w_n) = [(mu + i w_n) S - F - Sigma(i w_n)]^-1 for every
// Matsubara frequency, with the reductions the loop needs (FP64).
//
// One workgroup inverts one frequency at a time (grid-stride over n).  The
// matrix lives in registers: a T x T grid of threads, thread (tr, tc) owns
// rows tr + T a and columns tc + T b (a, b < R, T = ceil(n/R) <= 26, so at
// most 11 waves per workgroup and ~168 registers per thread; n <= 5*26).  The inverse is an in-place Gauss-Jordan elimination with
// partial pivoting: step k picks the not-yet-used row r with the largest
// |Re| + |Im| in column k, scales it and eliminates column k from every
// other row.  Rows are never moved; the pivot order r_k is kept, and the
// physical element (i, j) ends up as G[rinv(i)][r(j)] (rinv = inverse of r).
// Two barriers per step: after the pivot candidates and column k are
// published, and after the pivot row is published.
//
// Reductions (per workgroup, then a fixed-order pass over workgroups):
//   TRACE:  sum_n Re tr[G_n S]                          -> tr(P S)
//   FULL:   P_acc += Re G_n + G2 / w_n^2 (LDS, n x n)    -> P
//   ENERGY: also sum_n Re tr[G_n Sigma_n]                -> E_2b
// with P = (4/beta) P_acc + G1 - (beta/2) G2,
//      tr(P S) = (4/beta)(sum Re tr G S + tr(G2 S) sum w^-2) + n - (beta/2) tr(G2 S),
//      E_2b = (2/beta) sum Re tr[G Sigma] - (2/beta) tr(G1 Sigma_1) (beta/2pi)^2 psi'(niw + 1/2).
#include "gf2_internal.h"

#include <algorithm>
#include <cmath>
#include <vector>

namespace gf2 {

constexpr int DY_MAXT = 26;
constexpr int DY_MAXR = 5;
constexpr int DY_MAXN = DY_MAXT * DY_MAXR;
constexpr int DY_THREADS = (DY_MAXT * DY_MAXT + 63) / 64 * 64;   // 704

struct DysonArgs {
    int n, T, niw, mode;
    double beta, mu;
    const double *S, *F, *G2;
    const double2 *Sig;     // may be NULL
    double2 *G;             // may be NULL
    double *partP;          // [gridDim.x][n*n]   (FULL/ENERGY)
    double *parts;          // [gridDim.x][4]     (trace, energy, singular flag)
};

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cinv(double2 a) {
    // 1/a with scaling to avoid overflow of |a|^2
    const double s = fmax(fabs(a.x), fabs(a.y));
    const double ar = a.x / s, ai = a.y / s;
    const double d = s * (ar * ar + ai * ai);
    return make_double2(ar / d, -ai / d);
}

template <int R>
__global__ __launch_bounds__(DY_THREADS) void k_dyson(DysonArgs a) {
    const int n = a.n, T = a.T;
    const int tid = threadIdx.x;
    const int nthr = blockDim.x;
    const int tr = tid / T, tc = tid % T;
    const bool active = tid < T * T;

    __shared__ double2 sh_col[2][DY_MAXN];
    __shared__ double2 sh_row[DY_MAXN];
    __shared__ double sh_pv[2][DY_MAXT];
    __shared__ int sh_pi[2][DY_MAXT];
    __shared__ int perm[DY_MAXN], rinv[DY_MAXN];
    __shared__ unsigned char pivoted[DY_MAXN];
    __shared__ double red[2][32];
    __shared__ int sing;
    extern __shared__ double shP[];   // n*n when FULL/ENERGY

    const bool full = a.mode != GF2_DYSON_TRACE;
    if (full)
        for (int e = tid; e < n * n; e += nthr) shP[e] = 0.0;
    if (tid == 0) sing = 0;

    double acc_tr = 0.0, acc_e = 0.0;
    double mr[R][R], mi[R][R];

    for (int nn = blockIdx.x; nn < a.niw; nn += gridDim.x) {
        const double w = M_PI * (double)(2 * nn + 1) / a.beta;
        const double2 *Sig = a.Sig ? a.Sig + (size_t)nn * n * n : nullptr;
        // The element addresses do not depend on nn; hiding the bases from the
        // optimiser keeps it from holding 3 R^2 pointers live across the
        // elimination (they would spill).
        const double *Sb = a.S, *Fb = a.F;
        int base = tr * n + tc;
        asm volatile("" : "+s"(Sb), "+s"(Fb), "+v"(base));
        // A = (i w + mu) S - F - Sigma_n
#pragma unroll
        for (int ia = 0; ia < R; ++ia)
#pragma unroll
            for (int jb = 0; jb < R; ++jb) {
                const int i = tr + T * ia, j = tc + T * jb;
                mr[ia][jb] = 0.0;
                mi[ia][jb] = 0.0;
                if (active && i < n && j < n) {
                    const int e = base + T * n * ia + T * jb;
                    const double s = Sb[e];
                    double re = a.mu * s - Fb[e], im = w * s;
                    if (Sig) {
                        const double2 sg = Sig[e];
                        re -= sg.x;
                        im -= sg.y;
                    }
                    mr[ia][jb] = re;
                    mi[ia][jb] = im;
                }
            }
        for (int e = tid; e < n; e += nthr) {
            pivoted[e] = 0;
            perm[e] = e;
            rinv[e] = e;
        }
        __syncthreads();

        for (int k = 0; k < n; ++k) {
            const int buf = k & 1;
            const int kc = k % T, cb = k / T;
            if (active && tc == kc) {
                double best = -1.0;
                int bi = n;
#pragma unroll
                for (int ia = 0; ia < R; ++ia) {
                    const int i = tr + T * ia;
                    if (i < n) {
                        double vr = 0.0, vi = 0.0;
#pragma unroll
                        for (int jb = 0; jb < R; ++jb)
                            if (jb == cb) { vr = mr[ia][jb]; vi = mi[ia][jb]; }
                        sh_col[buf][i] = make_double2(vr, vi);
                        if (!pivoted[i]) {
                            const double mag = fabs(vr) + fabs(vi);
                            if (mag > best) { best = mag; bi = i; }
                        }
                    }
                }
                sh_pv[buf][tr] = best;
                sh_pi[buf][tr] = bi;
            }
            __syncthreads();
            double best = -1.0;
            int r = n;
            for (int t = 0; t < T; ++t) {
                const double pv = sh_pv[buf][t];
                const int pi = sh_pi[buf][t];
                if (pv > best || (pv == best && pi < r)) { best = pv; r = pi; }
            }
            if (!(best > 0.0) || r >= n) {
                // singular (or NaN) matrix: flag and stop this frequency
                if (tid == 0) sing = 1;
                r = (r >= n) ? 0 : r;
            }
            if (active && tr == r % T) {
                const int ar = r / T;
#pragma unroll
                for (int jb = 0; jb < R; ++jb) {
                    const int j = tc + T * jb;
                    if (j < n) {
                        double vr = 0.0, vi = 0.0;
#pragma unroll
                        for (int ia = 0; ia < R; ++ia)
                            if (ia == ar) { vr = mr[ia][jb]; vi = mi[ia][jb]; }
                        sh_row[j] = make_double2(vr, vi);
                    }
                }
            }
            if (tid == 0) {
                pivoted[r] = 1;
                perm[k] = r;
                rinv[r] = k;
            }
            __syncthreads();
            if (active) {
                const double2 ipiv = cinv(sh_row[k]);
                double2 crow[R];
#pragma unroll
                for (int jb = 0; jb < R; ++jb) {
                    const int j = tc + T * jb;
                    crow[jb] = (j < n) ? sh_row[j] : make_double2(0.0, 0.0);
                }
#pragma unroll
                for (int ia = 0; ia < R; ++ia) {
                    const int i = tr + T * ia;
                    if (i >= n) continue;
                    if (i == r) {
#pragma unroll
                        for (int jb = 0; jb < R; ++jb) {
                            const int j = tc + T * jb;
                            const double2 v = (j == k) ? ipiv : cmul(crow[jb], ipiv);
                            mr[ia][jb] = v.x;
                            mi[ia][jb] = v.y;
                        }
                    } else {
                        const double2 f = cmul(sh_col[buf][i], ipiv);
#pragma unroll
                        for (int jb = 0; jb < R; ++jb) {
                            const int j = tc + T * jb;
                            if (j == k) {
                                mr[ia][jb] = -f.x;
                                mi[ia][jb] = -f.y;
                            } else {
                                // M -= f * crow
                                mr[ia][jb] -= f.x * crow[jb].x - f.y * crow[jb].y;
                                mi[ia][jb] -= f.x * crow[jb].y + f.y * crow[jb].x;
                            }
                        }
                    }
                }
            }
        }
        __syncthreads();   // perm / rinv complete

        // physical (i, j) holds G[rinv(i)][perm(j)]
        const double iw2 = 1.0 / (w * w);
#pragma unroll
        for (int ia = 0; ia < R; ++ia)
#pragma unroll
            for (int jb = 0; jb < R; ++jb) {
                const int i = tr + T * ia, j = tc + T * jb;
                if (!(active && i < n && j < n)) continue;
                const int ga = rinv[i], gb = perm[j];
                const size_t e = (size_t)ga * n + gb;
                if (!full) {
                    acc_tr += mr[ia][jb] * a.S[(size_t)gb * n + ga];
                } else {
                    shP[e] += mr[ia][jb] + a.G2[e] * iw2;
                    if (a.G) a.G[(size_t)nn * n * n + e] = make_double2(mr[ia][jb], mi[ia][jb]);
                    if (a.mode == GF2_DYSON_ENERGY && Sig) {
                        const double2 sg = Sig[(size_t)gb * n + ga];
                        acc_e += mr[ia][jb] * sg.x - mi[ia][jb] * sg.y;
                    }
                }
            }
        __syncthreads();   // shP / perm reuse by the next frequency
    }

    // block reductions (fixed order)
    {
        double v0 = acc_tr, v1 = acc_e;
        for (int off = 32; off > 0; off >>= 1) {
            v0 += __shfl_down(v0, off);
            v1 += __shfl_down(v1, off);
        }
        const int wv = tid >> 6;
        if ((tid & 63) == 0) {
            red[0][wv] = v0;
            red[1][wv] = v1;
        }
        __syncthreads();
        if (tid == 0) {
            double s0 = 0.0, s1 = 0.0;
            const int nw = (nthr + 63) / 64;
            for (int t = 0; t < nw; ++t) {
                s0 += red[0][t];
                s1 += red[1][t];
            }
            double *ps = a.parts + (size_t)blockIdx.x * 4;
            ps[0] = s0;
            ps[1] = s1;
            ps[2] = (double)sing;
            ps[3] = 0.0;
        }
    }
    if (full)
        for (int e = tid; e < n * n; e += nthr) a.partP[(size_t)blockIdx.x * n * n + e] = shP[e];
}

// P = (4/beta) sum_b partP[b] + G1 - (beta/2) G2
__global__ void k_reduce_P(int ne, int nb, double beta, const double *__restrict__ partP,
                           const double *__restrict__ G1, const double *__restrict__ G2,
                           double *__restrict__ P) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= ne) return;
    double s = 0.0;
    for (int b = 0; b < nb; ++b) s += partP[(size_t)b * ne + e];
    P[e] = (4.0 / beta) * s + G1[e] - 0.5 * beta * G2[e];
}

// out[0] = sum_b parts[b][0], out[1] = sum parts[b][1], out[2] = max flag,
// out[3] = <X, Y> (Frobenius), out[4] = <U, V>
__global__ __launch_bounds__(256) void k_finish(int nb, const double *__restrict__ parts, int ne,
                                                const double *__restrict__ X,
                                                const double *__restrict__ Y,
                                                const double *__restrict__ U,
                                                const double *__restrict__ V,
                                                double *__restrict__ out) {
    __shared__ double sh[5][256];
    const int t = threadIdx.x;
    double a0 = 0, a1 = 0, a2 = 0, a3 = 0, a4 = 0;
    for (int b = t; b < nb; b += 256) {
        a0 += parts[(size_t)b * 4];
        a1 += parts[(size_t)b * 4 + 1];
        a2 = fmax(a2, parts[(size_t)b * 4 + 2]);
    }
    if (X && Y)
        for (int e = t; e < ne; e += 256) a3 += X[e] * Y[e];
    if (U && V)
        for (int e = t; e < ne; e += 256) a4 += U[e] * V[e];
    sh[0][t] = a0; sh[1][t] = a1; sh[2][t] = a2; sh[3][t] = a3; sh[4][t] = a4;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (t < s) {
            sh[0][t] += sh[0][t + s];
            sh[1][t] += sh[1][t + s];
            sh[2][t] = fmax(sh[2][t], sh[2][t + s]);
            sh[3][t] += sh[3][t + s];
            sh[4][t] += sh[4][t + s];
        }
        __syncthreads();
    }
    if (t < 5) out[t] = sh[t][0];
}

template <int R>
static int launch_dyson(dim3 grid, dim3 block, size_t shm, hipStream_t s, const DysonArgs &a) {
    if (shm > 0)
        GF2_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(&k_dyson<R>),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm));
    hipLaunchKernelGGL(k_dyson<R>, grid, block, shm, s, a);
    return GF2_OK;
}

// Tail moments on the device: G1 = Sinv, G2 = Sinv H Sinv, G3 = Sinv H G2 + Sinv Sig1 Sinv,
// H = F - mu S.  Writes mom[0..2]; scratch: 3 n x n.
static int moments(gf2_ctx *c, double mu, const double *F, const double *Sig1, double *mom,
                   double *scratch) {
    const int n = c->n;
    const size_t ne = (size_t)n * n;
    double *H = scratch, *Y = scratch + ne, *Z = scratch + 2 * ne;
    GF2_TRY(copy_d2d(c, H, F, ne * 8));
    GF2_TRY(axpby(c, ne, -mu, c->S.as<double>(), 1.0, H));
    GF2_TRY(copy_d2d(c, mom, c->Sinv.ptr, ne * 8));
    GF2_TRY(matmul_nn(c, n, c->Sinv.as<double>(), H, Y));          // Sinv H
    GF2_TRY(matmul_nn(c, n, Y, c->Sinv.as<double>(), mom + ne));   // G2
    GF2_TRY(matmul_nn(c, n, Y, mom + ne, mom + 2 * ne));           // Sinv H G2
    if (Sig1) {
        GF2_TRY(matmul_nn(c, n, c->Sinv.as<double>(), Sig1, Z));
        GF2_TRY(matmul_nn(c, n, Z, c->Sinv.as<double>(), H));
        GF2_TRY(axpby(c, ne, 1.0, H, 1.0, mom + 2 * ne));
    }
    return GF2_OK;
}

int dyson_run(gf2_ctx *c, const gf2_dims *d, int mode, double mu, const double *F,
              const double2 *Sig_iw, const double *Sig1, double2 *G_iw, double *P,
              double *mom_out, double *out) {
    const int n = c->n, niw = d->niw;
    const size_t ne = (size_t)n * n;
    if (n > DY_MAXN) return fail(GF2_EINVAL, "gf2_dyson: n > 130 is not supported yet");
    const int R = (n + DY_MAXT - 1) / DY_MAXT;
    const int T = (n + R - 1) / R;
    const int nthr = (T * T + 63) / 64 * 64;   // whole waves: the shuffles need full waves
    const int nblocks = std::min(niw, 512);
    const bool full = mode != GF2_DYSON_TRACE;

    GF2_TRY(c->dys_X.ensure(6 * ne * 8));
    GF2_TRY(c->dys_aux.ensure((size_t)nblocks * 4 * 8 + 64));
    GF2_TRY(c->dys_out.ensure(8 * 8));
    if (full) GF2_TRY(c->dys_part.ensure((size_t)nblocks * ne * 8));
    double *mom = c->dys_X.as<double>();          // [3][n][n]
    double *scr = mom + 3 * ne;                    // [3][n][n]
    GF2_TRY(moments(c, mu, F, (mode == GF2_DYSON_TRACE) ? nullptr : Sig1, mom, scr));

    DysonArgs a{};
    a.n = n; a.T = T; a.niw = niw; a.mode = mode;
    a.beta = d->beta; a.mu = mu;
    a.S = c->S.as<double>(); a.F = F; a.G2 = mom + ne;
    a.Sig = Sig_iw; a.G = full ? G_iw : nullptr;
    a.partP = full ? c->dys_part.as<double>() : nullptr;
    a.parts = c->dys_aux.as<double>();
    const size_t shm = full ? ne * 8 : 0;
    dim3 grid(nblocks), block(nthr);
    switch (R) {
        case 1: GF2_TRY(launch_dyson<1>(grid, block, shm, c->stream, a)); break;
        case 2: GF2_TRY(launch_dyson<2>(grid, block, shm, c->stream, a)); break;
        case 3: GF2_TRY(launch_dyson<3>(grid, block, shm, c->stream, a)); break;
        case 4: GF2_TRY(launch_dyson<4>(grid, block, shm, c->stream, a)); break;
        default: GF2_TRY(launch_dyson<5>(grid, block, shm, c->stream, a)); break;
    }
    GF2_HIP(hipGetLastError());

    double *dout = c->dys_out.as<double>();
    if (full) {
        hipLaunchKernelGGL(k_reduce_P, dim3((unsigned)((ne + 255) / 256)), dim3(256), 0, c->stream,
                           (int)ne, nblocks, d->beta, c->dys_part.as<double>(), mom, mom + ne, P);
        // out: [0] sum tr (unused), [1] sum Re tr(G Sigma), [2] flag, [3] tr(P S), [4] tr(G1 Sigma1)
        hipLaunchKernelGGL(k_finish, dim3(1), dim3(256), 0, c->stream, nblocks, a.parts, (int)ne,
                           P, c->S.as<double>(), (mode == GF2_DYSON_ENERGY && Sig1) ? mom : nullptr,
                           Sig1, dout);
    } else {
        // out: [0] sum Re tr(G S), [3] tr(G2 S)
        hipLaunchKernelGGL(k_finish, dim3(1), dim3(256), 0, c->stream, nblocks, a.parts, (int)ne,
                           mom + ne, c->S.as<double>(), nullptr, nullptr, dout);
    }
    GF2_HIP(hipGetLastError());
    if (mom_out) GF2_TRY(copy_d2d(c, mom_out, mom, 3 * ne * 8));
    double h[5];
    GF2_HIP(hipMemcpyAsync(h, dout, 5 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    GF2_HIP(hipStreamSynchronize(c->stream));
    if (h[2] != 0.0) return fail(GF2_ENONFINITE, "gf2_dyson: singular or non-finite matrix");
    const double beta = d->beta;
    if (full) {
        out[0] = h[3];
        out[1] = 0.0;
        if (mode == GF2_DYSON_ENERGY && Sig_iw) {
            const double tg = h[4];
            const double tail = -(2.0 / beta) * tg * (beta / (2.0 * M_PI)) * (beta / (2.0 * M_PI)) *
                                trigamma(niw + 0.5);
            out[1] = (2.0 / beta) * h[1] + tail;
        }
    } else {
        double sw = 0.0;   // sum_{n<niw} 1/w_n^2
        for (int k = 0; k < niw; ++k) {
            const double w = M_PI * (double)(2 * k + 1) / beta;
            sw += 1.0 / (w * w);
        }
        const double trG2S = h[3];
        out[0] = (4.0 / beta) * (h[0] + trG2S * sw) + (double)n - 0.5 * beta * trG2S;
        out[1] = 0.0;
    }
    if (!std::isfinite(out[0]) || !std::isfinite(out[1]))
        return fail(GF2_ENONFINITE, "gf2_dyson: non-finite result");
    return GF2_OK;
}

}  // namespace gf2

using namespace gf2;

extern "C" int gf2_dyson(gf2_ctx *c, const gf2_dims *d, int mode, double mu, const double *F,
                         const void *Sigma_iw, const double *Sigma1, void *G_iw, double *P,
                         double *host_out) {
    if (!c || !d || !F || !host_out) return fail(GF2_EINVAL, "gf2_dyson: NULL argument");
    if (!c->has_system) return fail(GF2_ESTATE, "gf2_dyson: no system set");
    if (d->n != c->n) return fail(GF2_EINVAL, "gf2_dyson: dims->n differs from the system");
    if (d->niw < 1 || !(d->beta > 0.0)) return fail(GF2_EINVAL, "gf2_dyson: bad niw or beta");
    if (mode < GF2_DYSON_TRACE || mode > GF2_DYSON_ENERGY)
        return fail(GF2_EINVAL, "gf2_dyson: bad mode");
    if (mode != GF2_DYSON_TRACE && !P) return fail(GF2_EINVAL, "gf2_dyson: FULL/ENERGY need P");
    GF2_HIP(hipSetDevice(c->device));
    return dyson_run(c, d, mode, mu, F, static_cast<const double2 *>(Sigma_iw), Sigma1,
                     static_cast<double2 *>(G_iw), P, nullptr, host_out);
}
