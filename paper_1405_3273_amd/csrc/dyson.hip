// Eq. (GF): G(i w_n) = [(mu + i w_n) S - F - Sigma(i w_n)]^-1 for every
// Matsubara frequency, with the reductions the loop needs (FP64).
//
// One workgroup inverts one frequency at a time (grid-stride over n).  The
// matrix lives in registers: thread (tr, tc), tr < 16, tc < TC, owns rows
// tr + 16 a (a < RA) and columns tc + TC b (b < CB), RA = ceil(n/16).  For
// n <= 112, TC = 16 and CB = RA (4 waves, one per SIMD); for n <= 160,
// TC = 32 and CB = ceil(n/32) (8 waves).  Threads are numbered column-major
// (tid = 16 tc + tr), so the 16 owners of a column sit in 16 consecutive
// lanes of one wave.
// The inverse is an in-place Gauss-Jordan elimination with partial pivoting:
// step k picks the not-yet-used row r with the largest |Re| + |Im| in column
// k (a 16-lane shuffle argmax), scales it and eliminates column k from every
// other row.  Rows are never moved; the pivot order r_k is kept, and the
// physical element (i, j) ends up as G[rinv(i)][r(j)] (rinv = inverse of r).
// Two barriers per step: after column k and the pivot are published, and
// after the pivot row is published.
//
#include "gf2_internal.h"

#include <algorithm>
#include <cmath>
#include <vector>

namespace gf2 {

constexpr int DY_TR = 16;          // threads per column
constexpr int DY_MAXN = 160;
constexpr int DY_MAXTHREADS = 512;

struct DysonArgs {
    int n, niw, mode;
    double beta, mu;
    const double *S, *F, *G2;
    const double2 *Sig;     // may be NULL
    double2 *G;             // may be NULL
    double *partP;          // [gridDim.x][n*n]   (FULL/ENERGY)
    double *parts;          // [gridDim.x][4]     (trace, energy, singular flag)
    int p_in_lds;           // FULL/ENERGY: accumulate P in LDS (else in partP directly)
};

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// 1/x to full FP64 precision: hardware reciprocal estimate + two Newton steps
__device__ __forceinline__ double rcp_nr(double x) {
    double y = __builtin_amdgcn_rcp(x);
    double e = fma(-x, y, 1.0);
    y = fma(y, e, y);
    e = fma(-x, y, 1.0);
    return fma(y, e, y);
}

// 1/a for complex a, scaled so that |a|^2 cannot overflow or underflow
__device__ __forceinline__ double2 cinv(double2 a) {
    const double s = fmax(fabs(a.x), fabs(a.y));
    const double is = rcp_nr(s);
    const double ar = a.x * is, ai = a.y * is;
    const double id = rcp_nr(ar * ar + ai * ai) * is;
    return make_double2(ar * id, -ai * id);
}

// Rotate a value by k lanes within each row of 16 lanes (DPP row_ror:k).
template <int K> __device__ __forceinline__ int ror16(int v) {
    return __builtin_amdgcn_update_dpp(0, v, 0x120 + K, 0xF, 0xF, false);
}
template <int K> __device__ __forceinline__ double ror16(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = ror16<K>((int)(b & 0xffffffffLL));
    const int hi = ror16<K>((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
template <int K> __device__ __forceinline__ void argmax_step(double &best, int &bi) {
    const double ob = ror16<K>(best);
    const int oi = ror16<K>(bi);
    const bool take = ob > best || (ob == best && oi < bi);
    best = take ? ob : best;
    bi = take ? oi : bi;
}

template <int RA, int CB, int TC>
__global__ __launch_bounds__(DY_TR * TC, 2) void k_dyson(DysonArgs a) {
    const int n = a.n;
    const int tid = threadIdx.x;
    const int nthr = blockDim.x;
    const int tr = tid & (DY_TR - 1), tc = tid >> 4;
    const bool active = tc < TC;
    const int lane = tid & 63;

    __shared__ double2 sh_col[2][DY_TR * RA];   // padded rows hold zeros
    __shared__ double2 sh_row[TC * CB];         // padded columns hold zeros
    __shared__ int sh_r[2];
    __shared__ int perm[DY_MAXN], rinv[DY_MAXN];
    __shared__ double red[2][DY_MAXTHREADS / 64];
    __shared__ int sing;
    extern __shared__ double shP[];   // n*n when FULL/ENERGY and p_in_lds

    const bool full = a.mode != GF2_DYSON_TRACE;
    double *Pacc = a.p_in_lds ? shP : (a.partP + (size_t)blockIdx.x * n * n);
    if (full)
        for (int e = tid; e < n * n; e += nthr) Pacc[e] = 0.0;
    if (tid == 0) sing = 0;

    double acc_tr = 0.0, acc_e = 0.0;
    double mr[RA][CB], mi[RA][CB];

    for (int nn = blockIdx.x; nn < a.niw; nn += gridDim.x) {
        const double w = M_PI * (double)(2 * nn + 1) / a.beta;
        const double2 *Sig = a.Sig ? a.Sig + (size_t)nn * n * n : nullptr;
        // The element addresses do not depend on nn; hiding the bases from the
        // optimiser keeps it from holding the pointers live across the elimination.
        const double *Sb = a.S, *Fb = a.F;
        int base = tr * n + tc;
        asm volatile("" : "+s"(Sb), "+s"(Fb), "+v"(base));
        // A = (i w + mu) S - F - Sigma_n
#pragma unroll
        for (int ia = 0; ia < RA; ++ia)
#pragma unroll
            for (int jb = 0; jb < CB; ++jb) {
                const int i = tr + DY_TR * ia, j = tc + TC * jb;
                mr[ia][jb] = 0.0;
                mi[ia][jb] = 0.0;
                if (active && i < n && j < n) {
                    const int e = base + DY_TR * n * ia + TC * jb;
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
        unsigned pivmask = 0;   // bit a: row tr + 16 a already used as a pivot
        __syncthreads();        // previous frequency done with perm / sh_*

        // Each step is the uniform update M[i][j] -= f_i c_j with
        //   c_j = M[r][j] (j != k), c_k = 1,  M[i][k] preset to 0 (i != r), 1 (i = r),
        //   f_i = M[i][k]/p (i != r),  f_r = 1 - 1/p,   p = M[r][k],
        // which leaves exactly the in-place Gauss-Jordan result (row r scaled by
        // 1/p, column k = -f_i, pivot 1/p) with no per-element special cases.
        // Padding rows/columns (index >= n) hold zeros and stay zero.
        for (int k = 0; k < n; ++k) {
            const int buf = k & 1;
            const int kc = k % TC;
            const int cb = __builtin_amdgcn_readfirstlane(k / TC);
            if (active && tc == kc) {
                double best = -1.0;
                int bi = n;
#pragma unroll
                for (int jb = 0; jb < CB; ++jb) {
                    if (jb == cb) {   // scalar branch: cb is wave-uniform
#pragma unroll
                        for (int ia = 0; ia < RA; ++ia) {
                            const int i = tr + DY_TR * ia;
                            const double vr = mr[ia][jb], vi = mi[ia][jb];
                            sh_col[buf][i] = make_double2(vr, vi);
                            const double mag = fabs(vr) + fabs(vi);
                            const bool cand = !((pivmask >> ia) & 1u) && mag > best;
                            best = cand ? mag : best;
                            bi = cand ? i : bi;
                            mr[ia][jb] = 0.0;   // preset column k (row r gets 1 below)
                            mi[ia][jb] = 0.0;
                        }
                    }
                }
                // argmax over the 16 owners (one DPP row of 16 lanes); ties -> smaller row
                argmax_step<8>(best, bi);
                argmax_step<4>(best, bi);
                argmax_step<2>(best, bi);
                argmax_step<1>(best, bi);
                if (tr == 0) sh_r[buf] = (best > 0.0 && bi < n) ? bi : -1;
            }
            __syncthreads();
            int r = sh_r[buf];
            if (r < 0) {
                // singular (or NaN) matrix: flag, continue with a valid index
                if (tid == 0) sing = 1;
                r = k;
            }
            const int rr = r & (DY_TR - 1);
            const int ra = __builtin_amdgcn_readfirstlane(r >> 4);
            // the pivot is already published with column k: invert it while the
            // row owners publish row r
            const double2 ipiv = cinv(sh_col[buf][r]);
            if (active && tr == rr) {
                pivmask |= 1u << ra;
#pragma unroll
                for (int ia = 0; ia < RA; ++ia) {
                    if (ia == ra) {   // scalar branch
#pragma unroll
                        for (int jb = 0; jb < CB; ++jb) {
                            const int j = tc + TC * jb;
                            if (jb == cb && tc == kc) mr[ia][jb] = 1.0;
                            sh_row[j] = make_double2(mr[ia][jb], mi[ia][jb]);
                        }
                    }
                }
            }
            if (tid == 0) {
                perm[k] = r;
                rinv[r] = k;
            }
            __syncthreads();
            if (active) {
                double2 crow[CB];
#pragma unroll
                for (int jb = 0; jb < CB; ++jb) crow[jb] = sh_row[tc + TC * jb];
#pragma unroll
                for (int ia = 0; ia < RA; ++ia) {
                    const int i = tr + DY_TR * ia;
                    const double2 cv = sh_col[buf][i];
                    double fx = cv.x * ipiv.x - cv.y * ipiv.y;
                    double fy = cv.x * ipiv.y + cv.y * ipiv.x;
                    const bool is_r = (i == r);
                    fx = is_r ? 1.0 - ipiv.x : fx;
                    fy = is_r ? -ipiv.y : fy;
#pragma unroll
                    for (int jb = 0; jb < CB; ++jb) {
                        mr[ia][jb] = fma(-fx, crow[jb].x, mr[ia][jb]);
                        mr[ia][jb] = fma(fy, crow[jb].y, mr[ia][jb]);
                        mi[ia][jb] = fma(-fx, crow[jb].y, mi[ia][jb]);
                        mi[ia][jb] = fma(-fy, crow[jb].x, mi[ia][jb]);
                    }
                }
            }
        }
        __syncthreads();   // perm / rinv complete

        // physical (i, j) holds G[rinv(i)][perm(j)]
        const double iw2 = 1.0 / (w * w);
#pragma unroll
        for (int ia = 0; ia < RA; ++ia)
#pragma unroll
            for (int jb = 0; jb < CB; ++jb) {
                const int i = tr + DY_TR * ia, j = tc + TC * jb;
                if (!(active && i < n && j < n)) continue;
                const int ga = rinv[i], gb = perm[j];
                const size_t e = (size_t)ga * n + gb;
                if (!full) {
                    acc_tr += mr[ia][jb] * a.S[(size_t)gb * n + ga];
                } else {
                    Pacc[e] += mr[ia][jb] + a.G2[e] * iw2;
                    if (a.G) a.G[(size_t)nn * n * n + e] = make_double2(mr[ia][jb], mi[ia][jb]);
                    if (a.mode == GF2_DYSON_ENERGY && Sig) {
                        const double2 sg = Sig[(size_t)gb * n + ga];
                        acc_e += mr[ia][jb] * sg.x - mi[ia][jb] * sg.y;
                    }
                }
            }
    }
    __syncthreads();

    // block reductions (fixed order)
    {
        double v0 = acc_tr, v1 = acc_e;
        for (int off = 32; off > 0; off >>= 1) {
            v0 += __shfl_down(v0, off);
            v1 += __shfl_down(v1, off);
        }
        const int wv = tid >> 6;
        if (lane == 0) {
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
    if (full && a.p_in_lds)
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

template <int RA, int CB, int TC>
static int launch_dyson(dim3 grid, size_t shm, hipStream_t s, const DysonArgs &a) {
    if (shm > 0)
        GF2_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(&k_dyson<RA, CB, TC>),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm));
    hipLaunchKernelGGL((k_dyson<RA, CB, TC>), grid, dim3(DY_TR * TC), shm, s, a);
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
    if (n > DY_MAXN) return fail(GF2_EINVAL, "gf2_dyson: n > 160 is not supported");
    const int RA = (n + DY_TR - 1) / DY_TR;
    const bool full = mode != GF2_DYSON_TRACE;
    // a large LDS accumulator would keep a second workgroup off the CU
    const bool p_in_lds = full && ne * 8 <= 32 * 1024;
    const size_t shm = p_in_lds ? ne * 8 : 0;
    int dev_cus = 256;
    (void)hipDeviceGetAttribute(&dev_cus, hipDeviceAttributeMultiprocessorCount, c->device);
    // two resident workgroups per CU give each one a partner to overlap barriers with
    const int nblocks = std::max(1, std::min(niw, 2 * dev_cus));

    GF2_TRY(c->dys_X.ensure(6 * ne * 8));
    GF2_TRY(c->dys_aux.ensure((size_t)nblocks * 4 * 8 + 64));
    GF2_TRY(c->dys_out.ensure(8 * 8));
    if (full) GF2_TRY(c->dys_part.ensure((size_t)nblocks * ne * 8));
    double *mom = c->dys_X.as<double>();          // [3][n][n]
    double *scr = mom + 3 * ne;                    // [3][n][n]
    GF2_TRY(moments(c, mu, F, (mode == GF2_DYSON_TRACE) ? nullptr : Sig1, mom, scr));

    DysonArgs a{};
    a.n = n; a.niw = niw; a.mode = mode;
    a.beta = d->beta; a.mu = mu;
    a.S = c->S.as<double>(); a.F = F; a.G2 = mom + ne;
    a.Sig = Sig_iw; a.G = full ? G_iw : nullptr;
    a.partP = full ? c->dys_part.as<double>() : nullptr;
    a.parts = c->dys_aux.as<double>();
    a.p_in_lds = p_in_lds ? 1 : 0;
    dim3 grid(nblocks);
    const int ph = prof_begin(c, GF2_KC_DYSON);
    switch (RA) {
        case 1: GF2_TRY((launch_dyson<1, 1, 16>(grid, shm, c->stream, a))); break;
        case 2: GF2_TRY((launch_dyson<2, 2, 16>(grid, shm, c->stream, a))); break;
        case 3: GF2_TRY((launch_dyson<3, 3, 16>(grid, shm, c->stream, a))); break;
        case 4: GF2_TRY((launch_dyson<4, 4, 16>(grid, shm, c->stream, a))); break;
        case 5: GF2_TRY((launch_dyson<5, 5, 16>(grid, shm, c->stream, a))); break;
        case 6: GF2_TRY((launch_dyson<6, 6, 16>(grid, shm, c->stream, a))); break;
        case 7: GF2_TRY((launch_dyson<7, 7, 16>(grid, shm, c->stream, a))); break;
        case 8: GF2_TRY((launch_dyson<8, 4, 32>(grid, shm, c->stream, a))); break;
        case 9: GF2_TRY((launch_dyson<9, 5, 32>(grid, shm, c->stream, a))); break;
        default: GF2_TRY((launch_dyson<10, 5, 32>(grid, shm, c->stream, a))); break;
    }
    prof_end(c, ph, 8.0 * (double)n * n * n * niw);
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
