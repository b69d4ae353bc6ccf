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
// One workgroup barrier per step, after column k and the pivot are
// published.  The pivot row is published through LDS per column: every wave
// holds all rows of its own columns, so its lanes read only entries written
// by lanes of the same wave and need no second barrier.
//
#include "gf2_internal.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <string>
#include <map>
#include <mutex>
#include <vector>

namespace gf2 {

constexpr int DY_TR = 16;          // threads per column
constexpr int DY_MAXN = 160;
constexpr int DY_MAXTHREADS = 512;

// One system's Dyson evaluation.  The single-system call passes one job by
// value; the batched driver passes a device table of jobs (one per system)
// and the block offsets of each system in the launch.  Every kernel below
// resolves its job the same way, so a system gets identical arithmetic in
// both cases.
struct DysonJob {
    int n, niw, mode;       // mode < 0: idle (batched rounds)
    int p_in_lds;           // FULL/ENERGY: P accumulated in LDS: 1 whole, 2 upper triangle
                            // (block class; P is symmetric), 0 in partP directly
    int nbl;                // workgroups of this job in the Dyson launch
    double beta, mu;
    const double *S, *Sinv, *F, *Sig1;   // Sig1 may be NULL
    const double2 *Sig;     // may be NULL
    double2 *G;             // may be NULL
    double *P;              // FULL/ENERGY output
    double *mom;            // [3][n][n] tail moments G1, G2, G3 (computed here)
    double *scr;            // [3][n][n] scratch
    double *partP;          // [nbl][n*n]   (FULL/ENERGY) per-slot P accumulators
    double *partW;          // [npw][n*n]   per-workgroup P partials that k_reduce_P sums
    int npw;
    double *parts;          // [nbl][4]     (trace, energy, singular flag)
    double *out;            // [5] reduced results
};

struct DysonRef {
    DysonJob one;           // used when nsys == 0
    const DysonJob *tab;    // [nsys]
    const int *boff;        // [nsys + 1] first Dyson workgroup of each job
    int nsys;
};

__device__ __forceinline__ DysonJob job_of(const DysonRef &g, int s) {
    return g.nsys == 0 ? g.one : g.tab[s];
}

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

// 1/a for complex a: a scaled by the power of two 2^-e of its larger part
// (exact), so |a|^2 of the scaled value lies in [1/4, 2); 1/a = 2^-e conj(a')/|a'|^2
__device__ __forceinline__ double2 cinv(double2 a) {
    int e;
    (void)frexp(fmax(fabs(a.x), fabs(a.y)), &e);
    const double ar = ldexp(a.x, -e), ai = ldexp(a.y, -e);
    const double id = rcp_nr(fma(ar, ar, ai * ai));
    return make_double2(ldexp(ar * id, -e), ldexp(-ai * id, -e));
}

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Rotate a value by k lanes within each row of 16 lanes (DPP row_ror:k).
template <int K> __device__ __forceinline__ int ror16(int v) {
    // every lane reads a valid source lane, so no fallback value is needed
    // (update_dpp with an explicit one costs a move per call)
    return __builtin_amdgcn_mov_dpp(v, 0x120 + K, 0xF, 0xF, false);
}
template <int K> __device__ __forceinline__ double ror16(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = ror16<K>((int)(b & 0xffffffffLL));
    const int hi = ror16<K>((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
// value of v in lane `lane` (wave-uniform index) as a scalar
__device__ __forceinline__ double readlane_d(double v, int lane) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), lane);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
template <int K> __device__ __forceinline__ void argmax_step(double &best, int &bi) {
    const double ob = ror16<K>(best);
    const int oi = ror16<K>(bi);
    const bool take = (ob > best) | ((ob == best) & (oi < bi));   // no branches
    best = take ? ob : best;
    bi = take ? oi : bi;
}

// lb: this workgroup's index among the nbl workgroups of its job
template <int RA, int CB, int TC>
__device__ __forceinline__ void dyson_body(const DysonJob &a, const int lb, const int nbl) {
    const int n = a.n;
    const int tid = threadIdx.x;
    const int nthr = blockDim.x;
    const int tr = tid & (DY_TR - 1), tc = tid >> 4;
    const bool active = tc < TC;
    const int lane = tid & 63;

    __shared__ double2 sh_f[2][DY_TR * RA];     // factors f_i of the step
    __shared__ double2 sh_row[TC * CB];         // padded columns hold zeros
    __shared__ int sh_r[2];
    __shared__ int perm[DY_MAXN], rinv[DY_MAXN];
    __shared__ double red[2][DY_MAXTHREADS / 64];
    __shared__ int sing;
    extern __shared__ double shP[];   // FULL/ENERGY: n*n (p_in_lds 1) or n(n+1)/2 (2)

    const bool full = a.mode != GF2_DYSON_TRACE;
    const int pm = a.p_in_lds;
    double *Pacc = pm == 1 ? shP : (a.partP + (size_t)lb * n * n);
    if (full) {
        const int cnt = pm == 2 ? n * (n + 1) / 2 : n * n;
        for (int e = tid; e < cnt; e += nthr) (pm == 2 ? shP : Pacc)[e] = 0.0;
    }
    if (tid == 0) sing = 0;

    double acc_tr = 0.0, acc_e = 0.0;
    double mr[RA][CB], mi[RA][CB];
    const GF2_GLOBAL double *gS = (const GF2_GLOBAL double *)a.S;
    const GF2_GLOBAL double *gF = (const GF2_GLOBAL double *)a.F;
    const GF2_GLOBAL double *gM = (const GF2_GLOBAL double *)a.mom;
    typedef double d2_t __attribute__((ext_vector_type(2)));   // (re, im), as double2
    GF2_GLOBAL d2_t *gG = (GF2_GLOBAL d2_t *)a.G;

    for (int nn = lb; nn < a.niw; nn += nbl) {
        const double w = M_PI * (double)(2 * nn + 1) / a.beta;
        const GF2_GLOBAL d2_t *Sig =
            a.Sig ? (const GF2_GLOBAL d2_t *)a.Sig + (size_t)nn * n * n : nullptr;
        // The element addresses do not depend on nn; hiding the bases from the
        // optimiser keeps it from holding the pointers live across the elimination.
        const GF2_GLOBAL double *Sb = gS, *Fb = gF;
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
                        const d2_t sg = Sig[e];
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
#pragma unroll
                for (int jb = 0; jb < CB; ++jb) {
                    if (jb == cb) {   // scalar branch: cb is wave-uniform
                        double best = -1.0;
                        int bi = n;
#pragma unroll
                        for (int ia = 0; ia < RA; ++ia) {
                            const int i = tr + DY_TR * ia;
                            const double mag = fabs(mr[ia][jb]) + fabs(mi[ia][jb]);
                            const bool cand = !((pivmask >> ia) & 1u) & (mag > best);
                            best = cand ? mag : best;
                            bi = cand ? i : bi;
                        }
                        // argmax over the 16 owners (one DPP row of 16 lanes); ties -> smaller row
                        argmax_step<8>(best, bi);
                        argmax_step<4>(best, bi);
                        argmax_step<2>(best, bi);
                        argmax_step<1>(best, bi);
                        const int rk = (best > 0.0 && bi < n) ? bi : -1;
                        // pivot row (singular or NaN: continue with row k); the pivot
                        // value comes from its owner lane (wave-uniform lane index)
                        const int rp = __builtin_amdgcn_readfirstlane(rk < 0 ? k : rk);
                        const int src = 16 * (kc & 3) + (rp & (DY_TR - 1));
                        const int pa = rp >> 4;
                        double pvr = 0.0, pvi = 0.0;
#pragma unroll
                        for (int ia = 0; ia < RA; ++ia) {
                            if (ia == pa) {   // scalar branch
                                pvr = readlane_d(mr[ia][jb], src);
                                pvi = readlane_d(mi[ia][jb], src);
                            }
                        }
                        const double2 ip = cinv(make_double2(pvr, pvi));
                        // the owners form the factors once: f_i = M[i][k]/p (i != r),
                        // f_r = 1 - 1/p; then column k is preset to 0 (row r gets 1
                        // when it is published)
#pragma unroll
                        for (int ia = 0; ia < RA; ++ia) {
                            const int i = tr + DY_TR * ia;
                            const double vr = mr[ia][jb], vi = mi[ia][jb];
                            sh_f[buf][i] = make_double2(fma(vr, ip.x, -(vi * ip.y)), fma(vi, ip.x, vr * ip.y));
                            mr[ia][jb] = 0.0;
                            mi[ia][jb] = 0.0;
                        }
                        // then the pivot row's owner lane overwrites its factor with
                        // 1 - 1/p (one lane, so its two LDS writes stay in order)
                        if (tr == (rp & (DY_TR - 1))) sh_f[buf][rp] = make_double2(1.0 - ip.x, -ip.y);
                        if (tr == 0) sh_r[buf] = rk;
                    }
                }
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
            // Each lane reads only the sh_row entries of its own columns, written
            // by the row-r owner of its 16-lane group in the same wave: LDS order
            // within a wave suffices, no workgroup barrier.
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            if (active) {
                double2 crow[CB];
#pragma unroll
                for (int jb = 0; jb < CB; ++jb) crow[jb] = sh_row[tc + TC * jb];
#pragma unroll
                for (int ia = 0; ia < RA; ++ia) {
                    const double2 fv = sh_f[buf][tr + DY_TR * ia];
                    const double fx = fv.x, fy = fv.y;
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
        const bool en = full && a.mode == GF2_DYSON_ENERGY && Sig;
        double e_r = 0.0, e_i = 0.0;   // this frequency: Re G.(mu S - F), Im G.S
#pragma unroll
        for (int ia = 0; ia < RA; ++ia)
#pragma unroll
            for (int jb = 0; jb < CB; ++jb) {
                const int i = tr + DY_TR * ia, j = tc + TC * jb;
                if (!(active && i < n && j < n)) continue;
                const int ga = rinv[i], gb = perm[j];
                const size_t e = (size_t)ga * n + gb;
                const size_t et = (size_t)gb * n + ga;
                const double sv = gS[et];
                acc_tr += mr[ia][jb] * sv;
                if (full) {
                    const double pv = mr[ia][jb] + gM[n * n + e] * iw2;
                    if (pm == 2) {
                        // upper triangle, row-major: (ga, gb), ga <= gb
                        if (ga <= gb) shP[ga * n - ga * (ga - 1) / 2 + (gb - ga)] += pv;
                    } else {
                        Pacc[e] += pv;
                    }
                    if (gG) gG[(size_t)nn * n * n + e] = d2_t{mr[ia][jb], mi[ia][jb]};
                    if (en) {
                        e_r += mr[ia][jb] * fma(a.mu, sv, -gF[et]);
                        e_i += mi[ia][jb] * sv;
                    }
                }
            }
        // Re tr[G Sigma] from G A = 1: tr[G Sigma] = tr[G ((i w + mu) S - F)] - n
        // (S and F are small and stay in L2; Sigma(i w) is not read a second time)
        if (en) acc_e += e_r - w * e_i - (tid == 0 ? (double)n : 0.0);
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
            double *ps = a.parts + (size_t)lb * 4;
            ps[0] = s0;
            ps[1] = s1;
            ps[2] = (double)sing;
            ps[3] = 0.0;
        }
    }
    if (full && pm == 1)
        for (int e = tid; e < n * n; e += nthr) a.partP[(size_t)lb * n * n + e] = shP[e];
    if (full && pm == 2)
        for (int e = tid; e < n * n; e += nthr) {
            const int r = e / n, q = e - r * n;
            const int lo = min(r, q), hi = max(r, q);
            a.partP[(size_t)lb * n * n + e] = shP[lo * n - lo * (lo - 1) / 2 + (hi - lo)];
        }
}

// ---------------------------------------------------------------------------
// Small matrices (n <= 48): one wave per frequency, DW waves per workgroup,
// no workgroup barrier.  Lane = 16 c + t (c < 4 column groups, t < 16): rows
// t + 16a (a < RA), columns c + 4b (b < CB).  The 16 owners of a column are one
// DPP row, so the pivot argmax stays a 16-lane reduction; pivot column,
// factors and pivot row go through wave-private LDS (LDS operations of one
// wave execute in order).  The owners of column k also form the factors
// f_i = M[i][k]/p (f_r = 1 - 1/p), so the other lanes only read them.
// Partial sums: one slot per wave (slot = workgroup * DW + wave).
constexpr int DW = 4;

template <int RA, int CB>
__device__ __forceinline__ void dyson_wave(const DysonJob &a, const int lb, const int nwg) {
    constexpr int NR = 16 * RA, NC = 4 * CB;
    const int n = a.n;
    const int tid = threadIdx.x;
    const int wv = tid >> 6, lane = tid & 63;
    const int tr = lane & 15, tc = lane >> 4;
    const int slot = lb * DW + wv, nslot = nwg * DW;

    __shared__ double2 s_col[DW][NR];
    __shared__ double2 s_f[DW][NR];
    __shared__ double2 s_row[DW][NC];
    __shared__ int s_r[DW];
    __shared__ int s_perm[DW][NC > NR ? NC : NR], s_rinv[DW][NC > NR ? NC : NR];
    extern __shared__ double shP[];   // [DW][n*n] when FULL/ENERGY and p_in_lds
    double2 *col = s_col[wv], *fv = s_f[wv], *row = s_row[wv];
    int *perm = s_perm[wv], *rinv = s_rinv[wv];

    const bool full = a.mode != GF2_DYSON_TRACE;
    double *Pacc = a.p_in_lds ? shP + (size_t)wv * n * n : (a.partP + (size_t)slot * n * n);
    if (full)
        for (int e = lane; e < n * n; e += 64) Pacc[e] = 0.0;
    int sing = 0;
    double acc_tr = 0.0, acc_e = 0.0;
    double mr[RA][CB], mi[RA][CB];

    for (int nn = slot; nn < a.niw; nn += nslot) {
        const double w = M_PI * (double)(2 * nn + 1) / a.beta;
        const double2 *Sig = a.Sig ? a.Sig + (size_t)nn * n * n : nullptr;
#pragma unroll
        for (int ia = 0; ia < RA; ++ia)
#pragma unroll
            for (int jb = 0; jb < CB; ++jb) {
                const int i = tr + 16 * ia, j = tc + 4 * jb;
                mr[ia][jb] = 0.0;
                mi[ia][jb] = 0.0;
                if (i < n && j < n) {
                    const int e = i * n + j;
                    const double sv = a.S[e];
                    double re = a.mu * sv - a.F[e], im = w * sv;
                    if (Sig) {
                        const double2 sg = Sig[e];
                        re -= sg.x;
                        im -= sg.y;
                    }
                    mr[ia][jb] = re;
                    mi[ia][jb] = im;
                }
            }
        unsigned pivmask = 0;
        wave_sync();   // previous frequency done with perm / rinv
        for (int k = 0; k < n; ++k) {
            const int kc = k & 3;
            const int cb = __builtin_amdgcn_readfirstlane(k >> 2);
            if (tc == kc) {
                double best = -1.0;
                int bi = n;
#pragma unroll
                for (int jb = 0; jb < CB; ++jb) {
                    if (jb == cb) {   // scalar branch
#pragma unroll
                        for (int ia = 0; ia < RA; ++ia) {
                            const int i = tr + 16 * ia;
                            col[i] = make_double2(mr[ia][jb], mi[ia][jb]);
                            const double mag = fabs(mr[ia][jb]) + fabs(mi[ia][jb]);
                            const bool cand = !((pivmask >> ia) & 1u) && mag > best;
                            best = cand ? mag : best;
                            bi = cand ? i : bi;
                        }
                    }
                }
                argmax_step<8>(best, bi);
                argmax_step<4>(best, bi);
                argmax_step<2>(best, bi);
                argmax_step<1>(best, bi);
                const int r = (best > 0.0 && bi < n) ? bi : -1;
                wave_sync();
                const double2 ip = cinv(col[r < 0 ? k : r]);
#pragma unroll
                for (int jb = 0; jb < CB; ++jb) {
                    if (jb == cb) {   // scalar branch
#pragma unroll
                        for (int ia = 0; ia < RA; ++ia) {
                            const int i = tr + 16 * ia;
                            const double vx = mr[ia][jb], vy = mi[ia][jb];
                            fv[i] = make_double2(fma(vx, ip.x, -(vy * ip.y)), fma(vx, ip.y, vy * ip.x));
                            mr[ia][jb] = 0.0;   // preset column k
                            mi[ia][jb] = 0.0;
                        }
                    }
                }
                // the pivot row's owner lane overwrites its factor with 1 - 1/p
                if (r >= 0 && tr == (r & 15)) fv[r] = make_double2(1.0 - ip.x, -ip.y);
                if (tr == 0) s_r[wv] = r;
            }
            wave_sync();
            int r = s_r[wv];
            if (r < 0) {
                sing = 1;
                r = k;
            }
            const int rr = r & 15;
            const int ra = __builtin_amdgcn_readfirstlane(r >> 4);
            if (tr == rr) {
                pivmask |= 1u << ra;
#pragma unroll
                for (int ia = 0; ia < RA; ++ia) {
                    if (ia == ra) {   // scalar branch
#pragma unroll
                        for (int jb = 0; jb < CB; ++jb) {
                            if (jb == cb && tc == kc) mr[ia][jb] = 1.0;
                            row[tc + 4 * jb] = make_double2(mr[ia][jb], mi[ia][jb]);
                        }
                    }
                }
            }
            if (lane == 0) {
                perm[k] = r;
                rinv[r] = k;
            }
            wave_sync();
            double2 fr[RA];
#pragma unroll
            for (int ia = 0; ia < RA; ++ia) fr[ia] = fv[tr + 16 * ia];
#pragma unroll
            for (int jb = 0; jb < CB; ++jb) {
                const double2 c = row[tc + 4 * jb];
#pragma unroll
                for (int ia = 0; ia < RA; ++ia) {
                    mr[ia][jb] = fma(-fr[ia].x, c.x, mr[ia][jb]);
                    mr[ia][jb] = fma(fr[ia].y, c.y, mr[ia][jb]);
                    mi[ia][jb] = fma(-fr[ia].x, c.y, mi[ia][jb]);
                    mi[ia][jb] = fma(-fr[ia].y, c.x, mi[ia][jb]);
                }
            }
            wave_sync();   // this step's reads before the next step's writes
        }
        // physical (i, j) holds G[rinv(i)][perm(j)]
        const double iw2 = 1.0 / (w * w);
        const bool en = full && a.mode == GF2_DYSON_ENERGY && Sig;
        double e_r = 0.0, e_i = 0.0;   // this frequency: Re G.(mu S - F), Im G.S
#pragma unroll
        for (int ia = 0; ia < RA; ++ia)
#pragma unroll
            for (int jb = 0; jb < CB; ++jb) {
                const int i = tr + 16 * ia, j = tc + 4 * jb;
                if (!(i < n && j < n)) continue;
                const int ga = rinv[i], gb = perm[j];
                const size_t e = (size_t)ga * n + gb;
                const size_t et = (size_t)gb * n + ga;
                const double sv = a.S[et];
                acc_tr += mr[ia][jb] * sv;
                if (full) {
                    Pacc[e] += mr[ia][jb] + a.mom[n * n + e] * iw2;
                    if (a.G) a.G[(size_t)nn * n * n + e] = make_double2(mr[ia][jb], mi[ia][jb]);
                    if (en) {
                        e_r += mr[ia][jb] * fma(a.mu, sv, -a.F[et]);
                        e_i += mi[ia][jb] * sv;
                    }
                }
            }
        // Re tr[G Sigma] = Re tr[G ((i w + mu) S - F)] - n  (G A = 1)
        if (en) acc_e += e_r - w * e_i - (lane == 0 ? (double)n : 0.0);
    }
    // wave reductions (fixed order)
    double v0 = acc_tr, v1 = acc_e;
    for (int off = 32; off > 0; off >>= 1) {
        v0 += __shfl_down(v0, off);
        v1 += __shfl_down(v1, off);
    }
    if (lane == 0) {
        double *ps = a.parts + (size_t)slot * 4;
        ps[0] = v0;
        ps[1] = v1;
        ps[2] = (double)sing;
        ps[3] = 0.0;
    }
    if (full) {
        // the DW slots of this workgroup into one partial, waves in order
        __syncthreads();
        const int ne = n * n;
        double *dst = a.partW + (size_t)lb * ne;
        for (int e = tid; e < ne; e += 64 * DW) {
            double s = 0.0;
            for (int w = 0; w < DW; ++w)
                s += a.p_in_lds ? shP[(size_t)w * ne + e] : a.partP[(size_t)(lb * DW + w) * ne + e];
            dst[e] = s;
        }
    }
}

template <int RA, int CB, bool GRP>
__global__ __launch_bounds__(64 * DW) void k_dyson_w(DysonRef g) {
    if constexpr (GRP) {
        int sys = 0;
        while (sys + 1 < g.nsys && g.boff[sys + 1] <= (int)blockIdx.x) ++sys;
        sys = __builtin_amdgcn_readfirstlane(sys);
        const DysonJob a = g.tab[sys];
        if (a.mode < 0) return;
        dyson_wave<RA, CB>(a, (int)blockIdx.x - g.boff[sys], a.nbl / DW);
    } else {
        dyson_wave<RA, CB>(g.one, (int)blockIdx.x, (int)gridDim.x);
    }
}

// GRP: the jobs come from the table (batched launch), else the job is the
// kernel argument itself (its fields stay reloadable kernel-argument reads).
template <int RA, int CB, int TC, bool GRP>
__global__ __launch_bounds__(DY_TR * TC, 2) void k_dyson(DysonRef g) {
    if constexpr (GRP) {
        int sys = 0;
        while (sys + 1 < g.nsys && g.boff[sys + 1] <= (int)blockIdx.x) ++sys;
        sys = __builtin_amdgcn_readfirstlane(sys);
        const DysonJob a = g.tab[sys];
        if (a.mode < 0) return;
        dyson_body<RA, CB, TC>(a, (int)blockIdx.x - g.boff[sys], a.nbl);
    } else {
        dyson_body<RA, CB, TC>(g.one, (int)blockIdx.x, (int)gridDim.x);
    }
}

// Tail moments of every job, in three stages (grid: x over elements, y over
// jobs; one launch per stage):
//   0: G1 = Sinv,  Y = Sinv (F - mu S)
//   1: G2 = Y Sinv,  Z = Sinv Sig1 (FULL/ENERGY with Sig1)
//   2: G3 = Y G2 (+ Z Sinv)
// Each element is one plain row-by-column sum.
__global__ __launch_bounds__(256) void k_moments(DysonRef g, int stage) {
    const DysonJob a = job_of(g, blockIdx.y);
    if (a.mode < 0) return;
    const int n = a.n, ne = n * n;
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= ne) return;
    const int i = e / n, j = e - i * n;
    double *Y = a.scr, *Z = a.scr + ne;
    double *G1 = a.mom, *G2 = a.mom + ne, *G3 = a.mom + 2 * ne;
    const bool with_sig1 = a.mode != GF2_DYSON_TRACE && a.Sig1;
    const double *Si = a.Sinv + (size_t)i * n;
    if (stage == 0) {
        double s = 0.0;
        for (int k = 0; k < n; ++k) {
            const size_t kj = (size_t)k * n + j;
            s += Si[k] * fma(-a.mu, a.S[kj], a.F[kj]);
        }
        Y[e] = s;
        G1[e] = a.Sinv[e];
    } else if (stage == 1) {
        const double *Yi = Y + (size_t)i * n;
        double s = 0.0, z = 0.0;
        for (int k = 0; k < n; ++k) s += Yi[k] * a.Sinv[(size_t)k * n + j];
        G2[e] = s;
        if (with_sig1) {
            for (int k = 0; k < n; ++k) z += Si[k] * a.Sig1[(size_t)k * n + j];
            Z[e] = z;
        }
    } else {
        const double *Yi = Y + (size_t)i * n, *Zi = Z + (size_t)i * n;
        double s = 0.0, z = 0.0;
        for (int k = 0; k < n; ++k) s += Yi[k] * G2[(size_t)k * n + j];
        if (with_sig1)
            for (int k = 0; k < n; ++k) z += Zi[k] * a.Sinv[(size_t)k * n + j];
        G3[e] = s + z;
    }
}

static void launch_moments(const DysonRef &g, int njobs, int maxne, hipStream_t st) {
    const dim3 grid((unsigned)((maxne + 255) / 256), (unsigned)njobs);
    for (int stage = 0; stage < 3; ++stage)
        hipLaunchKernelGGL(k_moments, grid, dim3(256), 0, st, g, stage);
}

// P = (4/beta) sum_b partW[b] + G1 - (beta/2) G2.  Grid: x over 64-element
// chunks, y over jobs; the four waves of a workgroup sum quarters of the
// partials (four interleaved accumulators each) and are combined in order.
// When the partials hold the upper triangle mirrored (p_in_lds 2), the tail
// terms are taken from the upper triangle too, so P is exactly symmetric and
// every term of an element comes from the same (a <= b) entries.
__global__ __launch_bounds__(256) void k_reduce_P(DysonRef g) {
    const DysonJob a = job_of(g, blockIdx.y);
    if (a.mode <= GF2_DYSON_TRACE) return;
    const int ne = a.n * a.n;
    if ((int)blockIdx.x * 64 >= ne) return;
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int e = blockIdx.x * 64 + lane;
    __shared__ double sh[4][64];
    const int q = (a.npw + 3) / 4;
    const int b0 = wv * q, b1 = min(a.npw, b0 + q);
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    if (e < ne) {
        const double *p = a.partW + e;
        int b = b0;
        for (; b + 4 <= b1; b += 4) {
            s0 += p[(size_t)b * ne];
            s1 += p[(size_t)(b + 1) * ne];
            s2 += p[(size_t)(b + 2) * ne];
            s3 += p[(size_t)(b + 3) * ne];
        }
        for (; b < b1; ++b) s0 += p[(size_t)b * ne];
    }
    sh[wv][lane] = (s0 + s1) + (s2 + s3);
    __syncthreads();
    if (wv == 0 && e < ne) {
        const double s = (sh[0][lane] + sh[1][lane]) + (sh[2][lane] + sh[3][lane]);
        int et = e;
        if (a.p_in_lds == 2) {
            const int r = e / a.n, c = e - r * a.n;
            et = min(r, c) * a.n + max(r, c);
        }
        a.P[e] = (4.0 / a.beta) * s + a.mom[et] - 0.5 * a.beta * a.mom[ne + et];
    }
}

// out[0] = sum_b parts[b][0], out[1] = sum parts[b][1], out[2] = max flag,
// out[3] = <X, Y> (Frobenius), out[4] = <U, V>, out[5] = <G2, S>; TRACE: X = G2,
// Y = S; FULL/ENERGY: X = P, Y = S, U = G1, V = Sig1 (ENERGY with Sig1).  One
// workgroup per job.
__global__ __launch_bounds__(256) void k_finish(DysonRef g) {
    const DysonJob a = job_of(g, blockIdx.x);
    if (a.mode < 0) return;
    const int ne = a.n * a.n;
    const bool full = a.mode != GF2_DYSON_TRACE;
    const double *X = full ? a.P : a.mom + ne;
    const double *Y = a.S;
    const double *U = (a.mode == GF2_DYSON_ENERGY && a.Sig1) ? a.mom : nullptr;
    const double *V = a.Sig1;
    __shared__ double sh[6][256];
    const int t = threadIdx.x;
    double a0 = 0, a1 = 0, a2 = 0, a3 = 0, a4 = 0, a5 = 0;
    for (int b = t; b < a.nbl; b += 256) {
        a0 += a.parts[(size_t)b * 4];
        a1 += a.parts[(size_t)b * 4 + 1];
        a2 = fmax(a2, a.parts[(size_t)b * 4 + 2]);
    }
    for (int e = t; e < ne; e += 256) a3 += X[e] * Y[e];
    if (U && V)
        for (int e = t; e < ne; e += 256) a4 += U[e] * V[e];
    if (full)
        for (int e = t; e < ne; e += 256) a5 += a.mom[ne + e] * Y[e];
    sh[0][t] = a0; sh[1][t] = a1; sh[2][t] = a2; sh[3][t] = a3; sh[4][t] = a4; sh[5][t] = a5;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (t < s) {
            sh[0][t] += sh[0][t + s];
            sh[1][t] += sh[1][t + s];
            sh[2][t] = fmax(sh[2][t], sh[2][t + s]);
            sh[3][t] += sh[3][t + s];
            sh[4][t] += sh[4][t + s];
            sh[5][t] += sh[5][t + s];
        }
        __syncthreads();
    }
    if (t < 6) a.out[t] = sh[t][0];
}

// attr_only: set the dynamic-LDS limit without launching (before a capture)
template <int RA, int CB, int TC>
static int launch_dyson(dim3 grid, size_t shm, hipStream_t s, const DysonRef &g,
                        bool attr_only = false) {
    const void *fn = (g.nsys > 0) ? reinterpret_cast<const void *>(&k_dyson<RA, CB, TC, true>)
                                  : reinterpret_cast<const void *>(&k_dyson<RA, CB, TC, false>);
    if (shm > 0) GF2_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm));
    if (attr_only) return GF2_OK;
    if (g.nsys > 0)
        hipLaunchKernelGGL((k_dyson<RA, CB, TC, true>), grid, dim3(DY_TR * TC), shm, s, g);
    else
        hipLaunchKernelGGL((k_dyson<RA, CB, TC, false>), grid, dim3(DY_TR * TC), shm, s, g);
    return GF2_OK;
}

template <int RA, int CB>
static int launch_dyson_w(dim3 grid, size_t shm, hipStream_t s, const DysonRef &g,
                          bool attr_only = false) {
    const void *fn = (g.nsys > 0) ? reinterpret_cast<const void *>(&k_dyson_w<RA, CB, true>)
                                  : reinterpret_cast<const void *>(&k_dyson_w<RA, CB, false>);
    if (shm > 0) GF2_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm));
    if (attr_only) return GF2_OK;
    if (g.nsys > 0)
        hipLaunchKernelGGL((k_dyson_w<RA, CB, true>), grid, dim3(64 * DW), shm, s, g);
    else
        hipLaunchKernelGGL((k_dyson_w<RA, CB, false>), grid, dim3(64 * DW), shm, s, g);
    return GF2_OK;
}

// Size class of the register-resident inverse (rows per thread); classes 1-3
// (n <= 48) use the wave-per-frequency kernel.
static int dyson_class(int n) { return (n + DY_TR - 1) / DY_TR; }
static bool dyson_wave_class(int ra) { return ra <= 3; }

static int launch_dyson_class(int ra, dim3 grid, size_t shm, hipStream_t s, const DysonRef &g,
                              bool attr_only = false) {
    switch (ra) {
        case 1: return launch_dyson_w<1, 4>(grid, shm, s, g, attr_only);
        case 2: return launch_dyson_w<2, 8>(grid, shm, s, g, attr_only);
        case 3: return launch_dyson_w<3, 12>(grid, shm, s, g, attr_only);
        case 4: return launch_dyson<4, 4, 16>(grid, shm, s, g, attr_only);
        case 5: return launch_dyson<5, 5, 16>(grid, shm, s, g, attr_only);
        case 6: return launch_dyson<6, 6, 16>(grid, shm, s, g, attr_only);
        case 7: return launch_dyson<7, 7, 16>(grid, shm, s, g, attr_only);
        case 8: return launch_dyson<8, 4, 32>(grid, shm, s, g, attr_only);
        case 9: return launch_dyson<9, 5, 32>(grid, shm, s, g, attr_only);
        default: return launch_dyson<10, 5, 32>(grid, shm, s, g, attr_only);
    }
}

// Partial-sum slots of a job and its workgroups.  Workgroup kernel: one slot
// per workgroup, two resident per CU (each has a partner to overlap barriers
// with).  Wave kernel: one slot per wave, DW waves per workgroup, about eight
// waves per CU.
static int dyson_slots(gf2_ctx *c, int n, int niw) {
    int dev_cus = 256;
    (void)hipDeviceGetAttribute(&dev_cus, hipDeviceAttributeMultiprocessorCount, c->device);
    if (dyson_wave_class(dyson_class(n))) {
        const int waves = std::max(1, std::min(niw, 8 * dev_cus));
        return (waves + DW - 1) / DW * DW;
    }
    return std::max(1, std::min(niw, 2 * dev_cus));
}
static int dyson_workgroups(int n, int slots) {
    return dyson_wave_class(dyson_class(n)) ? slots / DW : slots;
}
// Where a FULL/ENERGY solve accumulates P (DysonJob::p_in_lds): the whole
// matrix in LDS when it takes <= 32 KB (per wave slot in the wave class), else
// in the block class its upper triangle (<= 104 KB: n <= 160; up to n = 112 it
// keeps two workgroups of 4 waves per CU), else global memory.
static int dyson_pmode(int n, int mode) {
    if (mode == GF2_DYSON_TRACE) return 0;
    const size_t ne8 = (size_t)n * n * 8;
    if (dyson_wave_class(dyson_class(n))) return DW * ne8 <= 32 * 1024 ? 1 : 0;
    if (ne8 <= 32 * 1024) return 1;
    return (size_t)n * (n + 1) / 2 * 8 <= 104 * 1024 ? 2 : 0;
}
static size_t dyson_shm(int n, int mode) {
    const size_t ne8 = (size_t)n * n * 8;
    switch (dyson_pmode(n, mode)) {
    case 1: return dyson_wave_class(dyson_class(n)) ? DW * ne8 : ne8;
    case 2: return (size_t)n * (n + 1) / 2 * 8;
    default: return 0;
    }
}

// P partials of a FULL/ENERGY solve: the wave class sums the DW slots of a
// workgroup into one partial (after the per-slot accumulators when those are
// in global memory); the workgroup class writes one partial per workgroup.
struct PartLayout {
    size_t bytes;   // dys_part size
    size_t off_w;   // element offset of the per-workgroup partials
    int npw;        // their count
};
static PartLayout part_layout(int n, int slots, int mode) {
    const size_t ne = (size_t)n * n;
    PartLayout L{};
    if (dyson_wave_class(dyson_class(n))) {
        L.npw = slots / DW;
        L.off_w = dyson_shm(n, mode) > 0 ? 0 : (size_t)slots * ne;
    } else {
        L.npw = slots;
        L.off_w = 0;
    }
    L.bytes = (L.off_w + (size_t)L.npw * ne) * 8;
    return L;
}

// N(mu) + n... : tr(P S) from the per-frequency traces tr(G(i w) S) and the
// tail: (4/beta) (sum_n Re tr(G S) + tr(G2 S) sum_n 1/w_n^2) + n - (beta/2) tr(G2 S)
static double trace_formula(const DysonJob &j, double sum_tr, double trG2S) {
    const double beta = j.beta;
    double sw = 0.0;   // sum_{n<niw} 1/w_n^2
    for (int k = 0; k < j.niw; ++k) {
        const double w = M_PI * (double)(2 * k + 1) / beta;
        sw += 1.0 / (w * w);
    }
    return (4.0 / beta) * (sum_tr + trG2S * sw) + (double)j.n - 0.5 * beta * trG2S;
}

// Host part of a job's result: h = out[0..5] of k_finish.  out[0]: tr(P S)
// (FULL/ENERGY: of the assembled P; TRACE: the trace formula), out[1]: the
// energy term, out[2]: the trace formula in every mode.
static int dyson_post(const DysonJob &j, const double *h, double *out) {
    if (h[2] != 0.0) return fail(GF2_ENONFINITE, "gf2_dyson: singular or non-finite matrix");
    const double beta = j.beta;
    if (j.mode != GF2_DYSON_TRACE) {
        out[0] = h[3];
        out[1] = 0.0;
        if (j.mode == GF2_DYSON_ENERGY && j.Sig) {
            const double tg = h[4];
            const double tail = -(2.0 / beta) * tg * (beta / (2.0 * M_PI)) * (beta / (2.0 * M_PI)) *
                                trigamma(j.niw + 0.5);
            out[1] = (2.0 / beta) * h[1] + tail;
        }
        out[2] = trace_formula(j, h[0], h[5]);
    } else {
        out[0] = trace_formula(j, h[0], h[3]);
        out[1] = 0.0;
        out[2] = out[0];
    }
    if (!std::isfinite(out[0]) || !std::isfinite(out[1]) || !std::isfinite(out[2]))
        return fail(GF2_ENONFINITE, "gf2_dyson: non-finite result");
    return GF2_OK;
}

// Device workspace of one single-system solve: tail moments and their
// scratch ([6][n][n]), per-slot (trace, energy, flag) partials, the reduced
// results and, for FULL/ENERGY, the P partials.  Every kernel writes (or
// zeroes) what it later reads, so the workspace needs no clearing.
struct DysonWs {
    double *X, *aux, *out, *part;
};
struct DysonWsSize {
    int nblocks;
    size_t x, aux, out, part;   // bytes
};
static DysonWsSize dyson_ws_size(gf2_ctx *c, int n, int niw, int mode) {
    DysonWsSize s{};
    const size_t ne = (size_t)n * n;
    s.nblocks = dyson_slots(c, n, niw);
    s.x = 6 * ne * 8;
    s.aux = (size_t)s.nblocks * 4 * 8 + 64;
    s.out = 8 * 8;
    s.part = mode != GF2_DYSON_TRACE ? part_layout(n, s.nblocks, mode).bytes : 0;
    return s;
}

static int dyson_run_ws(gf2_ctx *c, const gf2_dims *d, int mode, double mu, const double *F,
                        const double2 *Sig_iw, const double *Sig1, double2 *G_iw, double *P,
                        double *mom_out, double *out, double *trace_n, int nblocks,
                        const DysonWs &ws) {
    const int n = c->n, niw = d->niw;
    const size_t ne = (size_t)n * n;
    const bool full = mode != GF2_DYSON_TRACE;
    const size_t shm = dyson_shm(n, mode);
    const PartLayout pl = part_layout(n, nblocks, mode);

    DysonRef g{};
    DysonJob &a = g.one;
    a.n = n; a.niw = niw; a.mode = mode;
    a.p_in_lds = dyson_pmode(n, mode);
    a.nbl = nblocks;
    a.beta = d->beta; a.mu = mu;
    a.S = c->S.as<double>(); a.Sinv = c->Sinv.as<double>(); a.F = F;
    a.Sig1 = full ? Sig1 : nullptr;
    a.Sig = Sig_iw; a.G = full ? G_iw : nullptr;
    a.P = full ? P : nullptr;
    a.mom = ws.X;
    a.scr = a.mom + 3 * ne;
    a.partP = full ? ws.part : nullptr;
    a.partW = full ? ws.part + pl.off_w : nullptr;
    a.npw = pl.npw;
    a.parts = ws.aux;
    a.out = ws.out;
    g.nsys = 0;

    launch_moments(g, 1, (int)ne, c->stream);
    const int ph = prof_begin(c, GF2_KC_DYSON);
    GF2_TRY(launch_dyson_class(dyson_class(n), dim3(dyson_workgroups(n, nblocks)), shm, c->stream, g));
    prof_end(c, ph, 8.0 * (double)n * n * n * niw);
    GF2_HIP(hipGetLastError());
    if (full)
        hipLaunchKernelGGL(k_reduce_P, dim3((unsigned)((ne + 63) / 64), 1), dim3(256), 0,
                           c->stream, g);
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(256), 0, c->stream, g);
    GF2_HIP(hipGetLastError());
    if (mom_out) GF2_TRY(copy_d2d(c, mom_out, a.mom, 3 * ne * 8));
    double h[6], o[3];
    GF2_HIP(hipMemcpyAsync(h, a.out, 6 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    GF2_HIP(hipStreamSynchronize(c->stream));
    GF2_TRY(dyson_post(a, h, o));
    out[0] = o[0];
    out[1] = o[1];
    if (trace_n) *trace_n = o[2];
    return GF2_OK;
}

int dyson_run(gf2_ctx *c, const gf2_dims *d, int mode, double mu, const double *F,
              const double2 *Sig_iw, const double *Sig1, double2 *G_iw, double *P,
              double *mom_out, double *out, double *trace_n) {
    if (c->n > DY_MAXN) return fail(GF2_EINVAL, "gf2_dyson: n > 160 is not supported");
    const DysonWsSize s = dyson_ws_size(c, c->n, d->niw, mode);
    GF2_TRY(c->dys_X.ensure(s.x));
    GF2_TRY(c->dys_aux.ensure(s.aux));
    GF2_TRY(c->dys_out.ensure(s.out));
    if (s.part) GF2_TRY(c->dys_part.ensure(s.part));
    const DysonWs ws{c->dys_X.as<double>(), c->dys_aux.as<double>(), c->dys_out.as<double>(),
                     c->dys_part.as<double>()};
    return dyson_run_ws(c, d, mode, mu, F, Sig_iw, Sig1, G_iw, P, mom_out, out, trace_n,
                        s.nblocks, ws);
}

// ---------------------------------------------------------------------------
// Workspace of gf2_dyson_noalloc: one fixed device array per GPU, allocated
// with the code object, so the call itself allocates nothing.  Host code
// reaches it only through the address hipGetSymbolAddress returns for the
// current device (the array's name in host code is a host-side stand-in).
static __device__ __align__(256) unsigned char scratch[GF2_NOALLOC_SCRATCH_BYTES];

static std::mutex g_scratch_mu;
static std::map<int, unsigned char *> g_scratch_ptr;   // device -> address of its scratch

static int scratch_address(int device, unsigned char **ptr) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch_ptr.find(device);
    if (it != g_scratch_ptr.end()) {
        *ptr = it->second;
        return GF2_OK;
    }
    void *p = nullptr;
    GF2_HIP(hipSetDevice(device));
    GF2_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(GF2_EHIP, "gf2_dyson_noalloc: no address for the scratch array");
    *ptr = static_cast<unsigned char *>(p);
    g_scratch_ptr[device] = *ptr;
    return GF2_OK;
}

static size_t round256(size_t b) { return (b + 255) / 256 * 256; }

// ---------------------------------------------------------------------------
// Batched rounds.  The jobs of all systems sit in one device table ordered by
// size class; the round is k_moments (all jobs), one k_dyson per size class,
// k_reduce_P and k_finish (all jobs).  That sequence is captured once into a
// HIP graph per batch shape and replayed every round after the table upload.
// Each job gets as many workgroups as dyson_run gives it, so its arithmetic
// (and rounding) equals the single-system call.

struct RoundShape {
    std::vector<int> order;        // table position -> request index
    std::vector<int> cls_begin;    // per class: first table position (size = ncls + 1)
    std::vector<int> cls_ra;       // per class: rows per thread
    std::vector<int> boff;         // per class: block offsets, concatenated (class c at cls_begin[c] + c)
    std::vector<size_t> shm;       // per class dynamic LDS
    long long key = 0;
};

static void release_graph(gf2_ctx *lead) {
    if (lead->bat_graph) {
        (void)hipGraphExecDestroy(static_cast<hipGraphExec_t>(lead->bat_graph));
        lead->bat_graph = nullptr;
    }
    lead->bat_key = 0;
}

void dyson_round_release(gf2_ctx *lead) {
    release_graph(lead);
    if (lead->bat_cap) {
        (void)hipStreamDestroy(lead->bat_cap);
        lead->bat_cap = nullptr;
    }
    if (lead->bat_host) {
        (void)hipHostFree(lead->bat_host);
        lead->bat_host = nullptr;
        lead->bat_host_bytes = 0;
    }
}

static int enqueue_round(gf2_ctx *lead, hipStream_t st, const RoundShape &sh, int nsys) {
    const DysonJob *tab = lead->bat_tab.as<DysonJob>();
    const int *boff = lead->bat_boff.as<int>();
    DysonRef all{};
    all.tab = tab;
    all.nsys = nsys;
    const int ncls = (int)sh.cls_ra.size();
    int maxne = 1;
    for (int k = 0; k < ncls; ++k) maxne = std::max(maxne, 16 * sh.cls_ra[k] * 16 * sh.cls_ra[k]);
    launch_moments(all, nsys, maxne, st);
    for (int k = 0; k < ncls; ++k) {
        DysonRef g{};
        g.tab = tab + sh.cls_begin[k];
        g.nsys = sh.cls_begin[k + 1] - sh.cls_begin[k];
        g.boff = boff + sh.cls_begin[k] + k;
        const int nblk = sh.boff[sh.cls_begin[k + 1] + k];
        GF2_TRY(launch_dyson_class(sh.cls_ra[k], dim3(nblk), sh.shm[k], st, g));
    }
    hipLaunchKernelGGL(k_reduce_P, dim3((unsigned)((maxne + 63) / 64), (unsigned)nsys), dim3(256),
                       0, st, all);
    hipLaunchKernelGGL(k_finish, dim3(nsys), dim3(256), 0, st, all);
    GF2_HIP(hipGetLastError());
    return GF2_OK;
}

int dyson_round(gf2_ctx *lead, const std::vector<DysonReq> &req, std::vector<double> &res) {
    const int nsys = (int)req.size();
    res.assign((size_t)3 * nsys, 0.0);
    // shape: systems ordered by size class (stable), workgroups per job
    RoundShape sh;
    std::vector<int> ra(nsys), nbl(nsys);
    for (int s = 0; s < nsys; ++s) {
        if (req[s].c->n > DY_MAXN) return fail(GF2_EINVAL, "gf2_dyson: n > 160 is not supported");
        ra[s] = dyson_class(req[s].c->n);
        nbl[s] = dyson_slots(req[s].c, req[s].c->n, req[s].d->niw);
    }
    long long key = nsys;
    for (int r = 1; r <= 10; ++r) {
        bool any = false;
        for (int s = 0; s < nsys; ++s)
            if (ra[s] == r) {
                if (!any) {
                    sh.cls_begin.push_back((int)sh.order.size());
                    sh.cls_ra.push_back(r);
                    any = true;
                }
                sh.order.push_back(s);
            }
    }
    sh.cls_begin.push_back(nsys);
    const int ncls = (int)sh.cls_ra.size();
    for (int k = 0; k < ncls; ++k) {
        int acc = 0;
        size_t shm = 0;
        for (int t = sh.cls_begin[k]; t < sh.cls_begin[k + 1]; ++t) {
            const int s = sh.order[t];
            sh.boff.push_back(acc);
            acc += dyson_workgroups(req[s].c->n, nbl[s]);
            shm = std::max(shm, dyson_shm(req[s].c->n, GF2_DYSON_FULL));
            key = key * 1000003LL + (long long)req[s].c->n * 7919 + nbl[s];
        }
        sh.boff.push_back(acc);
        sh.shm.push_back(shm);
    }
    // per-job workspaces (each system's own context)
    for (int s = 0; s < nsys; ++s) {
        gf2_ctx *c = req[s].c;
        const size_t ne = (size_t)c->n * c->n;
        GF2_TRY(c->dys_X.ensure(6 * ne * 8));
        GF2_TRY(c->dys_aux.ensure((size_t)nbl[s] * 4 * 8 + 64));
        GF2_TRY(c->dys_part.ensure(part_layout(req[s].c->n, nbl[s], GF2_DYSON_FULL).bytes));
    }
    const size_t tab_bytes = (size_t)nsys * sizeof(DysonJob);
    const size_t boff_bytes = sh.boff.size() * sizeof(int);
    GF2_TRY(lead->bat_tab.ensure(tab_bytes));
    GF2_TRY(lead->bat_boff.ensure(boff_bytes));
    GF2_TRY(lead->bat_out.ensure((size_t)nsys * 8 * 8));
    // the captured graph holds these addresses
    key = key * 1000003LL + (long long)(uintptr_t)lead->bat_tab.ptr;
    key = key * 1000003LL + (long long)(uintptr_t)lead->bat_boff.ptr;
    const size_t host_need = tab_bytes + (size_t)nsys * 8 * 8 + 64;
    if (lead->bat_host_bytes < host_need) {
        if (lead->bat_host) GF2_HIP(hipHostFree(lead->bat_host));
        lead->bat_host = nullptr;
        lead->bat_host_bytes = 0;
        GF2_HIP(hipHostMalloc(&lead->bat_host, host_need, hipHostMallocDefault));
        lead->bat_host_bytes = host_need;
    }
    DysonJob *tab_h = static_cast<DysonJob *>(lead->bat_host);
    double *out_h = reinterpret_cast<double *>(static_cast<char *>(lead->bat_host) + tab_bytes);
    double *out_d = lead->bat_out.as<double>();
    for (int t = 0; t < nsys; ++t) {
        const int s = sh.order[t];
        const DysonReq &q = req[s];
        gf2_ctx *c = q.c;
        const int n = c->n;
        const size_t ne = (size_t)n * n;
        DysonJob a{};
        a.n = n;
        a.niw = q.d->niw;
        a.mode = q.mode;
        a.p_in_lds = dyson_pmode(n, q.mode);
        a.nbl = nbl[s];
        a.beta = q.d->beta;
        a.mu = q.mu;
        a.S = c->S.as<double>();
        a.Sinv = c->Sinv.as<double>();
        a.F = q.F;
        const bool full = q.mode > GF2_DYSON_TRACE;
        a.Sig1 = full ? q.Sig1 : nullptr;
        a.Sig = q.Sig;
        a.G = full ? q.G_iw : nullptr;
        a.P = full ? q.P : nullptr;
        a.mom = (full && q.mom) ? q.mom : c->dys_X.as<double>();
        a.scr = c->dys_X.as<double>() + 3 * ne;
        const PartLayout pl = part_layout(n, nbl[s], full ? q.mode : GF2_DYSON_FULL);
        a.partP = c->dys_part.as<double>();
        a.partW = a.partP + pl.off_w;
        a.npw = pl.npw;
        a.parts = c->dys_aux.as<double>();
        a.out = out_d + (size_t)t * 8;
        tab_h[t] = a;
    }
    GF2_HIP(hipMemcpyAsync(lead->bat_tab.ptr, tab_h, tab_bytes, hipMemcpyHostToDevice, lead->stream));
    // (re)capture the round when the shape changed; the upload above is not part of it
    if (!lead->bat_graph || lead->bat_key != key) {
        release_graph(lead);
        GF2_HIP(hipMemcpyAsync(lead->bat_boff.ptr, sh.boff.data(), boff_bytes,
                               hipMemcpyHostToDevice, lead->stream));
        for (int k = 0; k < ncls; ++k)   // attributes are set outside the capture
            if (sh.shm[k] > 0) {
                DysonRef g{};
                g.nsys = 1;
                GF2_TRY(launch_dyson_class(sh.cls_ra[k], dim3(1), sh.shm[k], lead->stream, g, true));
            }
        GF2_HIP(hipStreamSynchronize(lead->stream));
        // capture on a private stream (the caller's may be the legacy default
        // stream, which cannot be captured); the graph is launched on the caller's
        if (!lead->bat_cap) GF2_HIP(hipStreamCreateWithFlags(&lead->bat_cap, hipStreamNonBlocking));
        hipGraph_t graph = nullptr;
        GF2_HIP(hipStreamBeginCapture(lead->bat_cap, hipStreamCaptureModeThreadLocal));
        const int rc = enqueue_round(lead, lead->bat_cap, sh, nsys);
        const hipError_t ec = hipStreamEndCapture(lead->bat_cap, &graph);
        if (rc != GF2_OK) {
            if (graph) (void)hipGraphDestroy(graph);
            return rc;
        }
        GF2_HIP(ec);
        hipGraphExec_t exec = nullptr;
        const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        GF2_HIP(ei);
        lead->bat_graph = exec;
        lead->bat_key = key;
    }
    const int ph = prof_begin(lead, GF2_KC_DYSON);
    GF2_HIP(hipGraphLaunch(static_cast<hipGraphExec_t>(lead->bat_graph), lead->stream));
    double work = 0.0;
    for (int s = 0; s < nsys; ++s)
        if (req[s].mode >= 0) work += 8.0 * std::pow((double)req[s].c->n, 3) * req[s].d->niw;
    prof_end(lead, ph, work);
    GF2_HIP(hipMemcpyAsync(out_h, out_d, (size_t)nsys * 8 * 8, hipMemcpyDeviceToHost, lead->stream));
    GF2_HIP(hipStreamSynchronize(lead->stream));
    for (int t = 0; t < nsys; ++t) {
        const int s = sh.order[t];
        if (req[s].mode < 0) continue;
        GF2_TRY(dyson_post(tab_h[t], out_h + (size_t)t * 8, &res[(size_t)3 * s]));
    }
    return GF2_OK;
}

}  // namespace gf2

using namespace gf2;

static int dyson_check(gf2_ctx *c, const gf2_dims *d, int mode, const double *F, double *P,
                       double *host_out, const char *who) {
    if (!c || !d || !F || !host_out) return fail(GF2_EINVAL, std::string(who) + ": NULL argument");
    if (!c->has_system) return fail(GF2_ESTATE, std::string(who) + ": no system set");
    if (d->n != c->n) return fail(GF2_EINVAL, std::string(who) + ": dims->n differs from the system");
    if (d->niw < 1 || !(d->beta > 0.0)) return fail(GF2_EINVAL, std::string(who) + ": bad niw or beta");
    if (mode < GF2_DYSON_TRACE || mode > GF2_DYSON_ENERGY)
        return fail(GF2_EINVAL, std::string(who) + ": bad mode");
    if (mode != GF2_DYSON_TRACE && !P) return fail(GF2_EINVAL, std::string(who) + ": FULL/ENERGY need P");
    return GF2_OK;
}

extern "C" int gf2_dyson(gf2_ctx *c, const gf2_dims *d, int mode, double mu, const double *F,
                         const void *Sigma_iw, const double *Sigma1, void *G_iw, double *P,
                         double *host_out) {
    GF2_TRY(dyson_check(c, d, mode, F, P, host_out, "gf2_dyson"));
    GF2_HIP(hipSetDevice(c->device));
    return dyson_run(c, d, mode, mu, F, static_cast<const double2 *>(Sigma_iw), Sigma1,
                     static_cast<double2 *>(G_iw), P, nullptr, host_out);
}

extern "C" int gf2_dyson_noalloc(gf2_ctx *c, const gf2_dims *d, int mode, double mu,
                                 const double *F, const void *Sigma_iw, const double *Sigma1,
                                 void *G_iw, double *P, double *host_out) {
    GF2_TRY(dyson_check(c, d, mode, F, P, host_out, "gf2_dyson_noalloc"));
    if (c->n > DY_MAXN) return fail(GF2_EINVAL, "gf2_dyson_noalloc: n > 160 is not supported");
    unsigned char *base = nullptr;
    GF2_TRY(scratch_address(c->device, &base));
    GF2_HIP(hipSetDevice(c->device));
    const DysonWsSize s = dyson_ws_size(c, c->n, d->niw, mode);
    const size_t need = round256(s.x) + round256(s.aux) + round256(s.out) + round256(s.part);
    if (need > (size_t)GF2_NOALLOC_SCRATCH_BYTES) {
        char buf[200];
        std::snprintf(buf, sizeof(buf),
                      "gf2_dyson_noalloc: this solve needs %zu bytes of workspace, more than the "
                      "fixed %zu (use gf2_dyson)", need, (size_t)GF2_NOALLOC_SCRATCH_BYTES);
        return fail(GF2_EINVAL, buf);
    }
    DysonWs ws{};
    size_t off = 0;
    ws.X = reinterpret_cast<double *>(base + off);   off += round256(s.x);
    ws.aux = reinterpret_cast<double *>(base + off); off += round256(s.aux);
    ws.out = reinterpret_cast<double *>(base + off); off += round256(s.out);
    ws.part = s.part ? reinterpret_cast<double *>(base + off) : nullptr;
    return dyson_run_ws(c, d, mode, mu, F, static_cast<const double2 *>(Sigma_iw), Sigma1,
                        static_cast<double2 *>(G_iw), P, nullptr, host_out, nullptr, s.nblocks, ws);
}
