// Density-fitted form of Eq. (Sigma).
//
// The Implementation section proposes (and the Conclusions recall) factored
// integrals as the cheaper route to the self-energy: v_ijkl = sum_P B^P_ij
// B^P_kl over m auxiliary functions P.  Substituting the factors into both
// integrals of Eq. (Sigma) and grouping the sums gives, with G = G(tau),
// Gb = G(-tau), Y^P = B^P G and X^{PQ} = Y^P B^Q (all N x N),
//
//     Sigma = -( 2 sum_{PQ} tr(X^{PQ} Gb) X^{PQ} - sum_{PQ} X^{PQ} Gb X^{PQ} ),
//
// the direct and the exchange diagram.  For symmetric G, Gb and B^P the
// device evaluates it as
//
//     Z^Q = B^Q Gb,   W^Q = Gb Y^Q,   Pi_PQ = sum_ac B^P_ac W^Q_ac  (= tr(X^{PQ} Gb)),
//     U^P = sum_Q (Z^Q Y^P) B^Q - 2 sum_Q Pi_PQ B^Q,
//     Sigma = sum_P Y^P U^P,
//
// since sum_PQ X^{PQ} Gb X^{PQ} = sum_P Y^P sum_Q (B^Q Gb Y^P) B^Q.  The direct
// term costs 4 m^2 N^2 + 6 m N^3 flops (Pi, its contraction with B, Y, W and the
// final product): the O(m N^3) the method's estimate names.  The exchange term
// needs every pair (P, Q): 4 m^2 N^3 flops as pair products, or 4 m N^4 through
// the N^4 tensor sum_Q Z^Q (x) B^Q (see df_run); neither is O(m N^3).
//
// Layouts (T = double or float, one tau point at a time):
//   B[P][a][b], Bt[a][P][b] (= B^P_ab), Yt[i][P][b] (= Y^P_ib),
//   Zt[a][Q][b] (= Z^Q_ab), W[Q][a][c], Pi[P][Q], U[P][b][j], and for a
//   chunk of P the exchange products Tx[P][a][Q][c] = (Z^Q Y^P)_ac.
// Every step is then a GEMM with plain leading dimensions:
//   Yt = Bt (mN x N) G,  Zt = Bt Gb,  W^Q = Gb Y^Q (batched over Q),
//   Pi = B (m x N^2) W^T,  U = -2 Pi B,  Tx^P = Zt (mN x N) Y^P (batched over P),
//   U += Tx (rows (P, a), K = (Q, c)) B (rows (Q, c)),  Sigma = Yt (N x mN) U.
#include <algorithm>
#include <cstdio>

#include "gf2_internal.h"

namespace gf2 {
namespace {

typedef double df_v4d __attribute__((ext_vector_type(4)));
typedef float df_v4f __attribute__((ext_vector_type(4)));

template <class T> struct DfAcc;
template <> struct DfAcc<double> { typedef df_v4d type; };
template <> struct DfAcc<float> { typedef df_v4f type; };

// C(r, c) = alpha sum_k A(r, k) B(k, c) + beta C(r, c) for z = 0 .. batch-1:
//   A(r, k) = A[z sA + r lda + k]   (or A[z sA + k lda + r], the transposed form),
//   B(k, c) = B[z sB + k ldb + c]   (or B[z sB + c ldb + k], the transposed form),
//   C(r, c) = C[z sC + r ldc + c].
// split = 1 (batch 1): z is a slice of kz along K and the kernel writes the
// slice's sum to FP64 partials part[z][M][N]; k_df_reduce adds them in order.
struct DfGemm {
    const void *A;
    long long lda, sA;
    const void *B;
    long long ldb, sB;
    void *C;
    long long ldc, sC;
    int M, N, K;
    int kz, split;
    double alpha, beta;
    double *part;
    int ctrans;   // C(r, c) lives at C[c ldc + r] (through FP64 partials and k_df_reduce_t)
    int pn;       // > 0: C(a pn + b, c pn + j) lives at C[((b pn + c) pn + a) pn + j] (no split)
};

constexpr int DF_THREADS = 256;
constexpr int DF_RT = 2;                  // 16-row tiles per wave
constexpr int DF_BM = 64 * DF_RT;         // 4 waves stacked along rows
constexpr int DF_BK = 16;
constexpr int DF_FLUSH = 512 / DF_BK;     // FP32 form: chunks between FP64 flushes

// Two workgroups per CU (two waves per SIMD: one loads and stores its next
// chunk while the other runs MFMAs), except for the widest FP32 tile, whose
// FP64 flush registers would then spill.  ONE: the launch's K is at most one
// flush interval, so the FP32 accumulators are converted once at the end and
// need no FP64 copy (the same sums; the widest tile then keeps two per CU).
template <class T, int NT, bool ONE> struct DfWaves {
    static constexpr int value = (sizeof(T) == 8 || NT <= 7 || ONE) ? 2 : 1;
};

template <class T, bool AT, bool BT, int NT, class OutT, bool ONE>
__global__ __launch_bounds__(DF_THREADS, (DfWaves<T, NT, ONE>::value)) void k_df_gemm(DfGemm g) {
    using acc_t = typename DfAcc<T>::type;
    constexpr bool F64 = sizeof(T) == 8;
    constexpr int BN = 16 * NT;
    constexpr int SA = DF_BM + 16;                    // padded row strides
    constexpr int SB = BN + ((16 - BN % 32) + 32) % 32;
    __shared__ __attribute__((aligned(16))) T As[DF_BK][SA];
    __shared__ T Bs[DF_BK][SB];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const long long r0 = (long long)blockIdx.x * DF_BM;
    const int c0 = blockIdx.y * BN;
    const int z = blockIdx.z;
    const T *A = static_cast<const T *>(g.A);
    const T *B = static_cast<const T *>(g.B);
    int K = g.K;
    if (g.split) {
        const long long k0 = (long long)z * g.kz;
        K = (int)std::min<long long>(g.kz, g.K - k0);
        A += AT ? k0 * g.lda : k0;
        B += BT ? k0 : k0 * g.ldb;
    } else {
        A += (long long)z * g.sA;
        B += (long long)z * g.sB;
    }

    acc_t acc[DF_RT][NT];
    constexpr bool FLUSH = !F64 && !ONE;
    double accd[FLUSH ? DF_RT : 1][FLUSH ? NT : 1][4];
#pragma unroll
    for (int r = 0; r < DF_RT; ++r)
#pragma unroll
        for (int c = 0; c < NT; ++c) {
            acc[r][c] = acc_t{0, 0, 0, 0};
            if constexpr (FLUSH) {
#pragma unroll
                for (int e = 0; e < 4; ++e) accd[r][c][e] = 0.0;
            }
        }

    constexpr int A_PER = DF_BK * DF_BM / DF_THREADS;
    constexpr int B_PER = (DF_BK * BN + DF_THREADS - 1) / DF_THREADS;
    // FP32, transposed A with aligned rows: thread t takes A_PER consecutive rows of
    // chunk row t / 16 as 16-byte loads (one LDS row segment), else one element per
    // step (FP64 keeps the element steps: its 16-byte form measured slower).
    constexpr int VEC = 16 / (int)sizeof(T);
    static_assert(DF_BM / A_PER * DF_BK == DF_THREADS && A_PER % VEC == 0, "A chunk layout");
    typedef T vec_t __attribute__((ext_vector_type(VEC)));
    const bool avec = AT && !F64 && g.lda % VEC == 0 && g.sA % VEC == 0 && (uintptr_t)A % 16 == 0;
    const int ak = tid / (DF_BM / A_PER), am = (tid % (DF_BM / A_PER)) * A_PER;
    T ra[A_PER], rb[B_PER];
    auto load = [&](int kb) {
        if (avec) {
            const long long gr = r0 + am;
            const int gk = kb + ak;
            const T *src = A + (long long)gk * g.lda + gr;
            if (gk < K && gr + A_PER <= g.M) {
#pragma unroll
                for (int v = 0; v < A_PER / VEC; ++v) {
                    const vec_t t = *reinterpret_cast<const vec_t *>(src + VEC * v);
#pragma unroll
                    for (int e = 0; e < VEC; ++e) ra[VEC * v + e] = t[e];
                }
            } else {
#pragma unroll
                for (int e = 0; e < A_PER; ++e) ra[e] = (gk < K && gr + e < g.M) ? src[e] : T(0);
            }
        } else {
#pragma unroll
            for (int e = 0; e < A_PER; ++e) {
                const int idx = tid + e * DF_THREADS;
                const long long gr = r0 + (AT ? idx % DF_BM : idx / DF_BK);
                const int gk = kb + (AT ? idx / DF_BM : idx % DF_BK);
                ra[e] = (gr < g.M && gk < K) ? (AT ? A[(long long)gk * g.lda + gr] : A[gr * g.lda + gk])
                                             : T(0);
            }
        }
#pragma unroll
        for (int e = 0; e < B_PER; ++e) {
            const int idx = tid + e * DF_THREADS;
            const int k = BT ? idx % DF_BK : idx / BN;
            const int c = BT ? idx / DF_BK : idx % BN;
            const int gk = kb + k, gc = c0 + c;
            const bool ok = idx < DF_BK * BN && gk < K && gc < g.N;
            rb[e] = ok ? (BT ? B[(long long)gc * g.ldb + gk] : B[(long long)gk * g.ldb + gc]) : T(0);
        }
    };
    auto store = [&]() {
        if (avec) {
#pragma unroll
            for (int v = 0; v < A_PER / VEC; ++v) {
                vec_t t;
#pragma unroll
                for (int e = 0; e < VEC; ++e) t[e] = ra[VEC * v + e];
                *reinterpret_cast<vec_t *>(&As[ak][am + VEC * v]) = t;
            }
        } else {
#pragma unroll
            for (int e = 0; e < A_PER; ++e) {
                const int idx = tid + e * DF_THREADS;
                if constexpr (AT) As[idx / DF_BM][idx % DF_BM] = ra[e];
                else As[idx % DF_BK][idx / DF_BK] = ra[e];
            }
        }
#pragma unroll
        for (int e = 0; e < B_PER; ++e) {
            const int idx = tid + e * DF_THREADS;
            if (idx < DF_BK * BN) {
                if constexpr (BT) Bs[idx % DF_BK][idx / DF_BK] = rb[e];
                else Bs[idx / BN][idx % BN] = rb[e];
            }
        }
    };

    const int nch = (K + DF_BK - 1) / DF_BK;
    load(0);
    for (int ch = 0; ch < nch; ++ch) {
        __syncthreads();
        store();
        __syncthreads();
        if (ch + 1 < nch) load((ch + 1) * DF_BK);
#pragma unroll
        for (int k0 = 0; k0 < DF_BK; k0 += 4) {
            const int kr = k0 + (lane >> 4);
            T af[DF_RT], bf[NT];
#pragma unroll
            for (int r = 0; r < DF_RT; ++r) af[r] = As[kr][wave * (16 * DF_RT) + 16 * r + (lane & 15)];
#pragma unroll
            for (int c = 0; c < NT; ++c) bf[c] = Bs[kr][16 * c + (lane & 15)];
#pragma unroll
            for (int r = 0; r < DF_RT; ++r)
#pragma unroll
                for (int c = 0; c < NT; ++c) {
                    if constexpr (F64)
                        acc[r][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[r], bf[c], acc[r][c], 0, 0, 0);
                    else
                        acc[r][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[r], bf[c], acc[r][c], 0, 0, 0);
                }
        }
        if constexpr (FLUSH) {
            if ((ch + 1) % DF_FLUSH == 0 || ch + 1 == nch) {
#pragma unroll
                for (int r = 0; r < DF_RT; ++r)
#pragma unroll
                    for (int c = 0; c < NT; ++c) {
#pragma unroll
                        for (int e = 0; e < 4; ++e) accd[r][c][e] += (double)acc[r][c][e];
                        acc[r][c] = acc_t{0, 0, 0, 0};
                    }
            }
        }
    }

    // register e of a lane holds row lane/16 + 4e (FP64 MFMA) or 4 (lane/16) + e
    // (FP32 MFMA), column lane % 16, of each 16 x 16 tile
#pragma unroll
    for (int r = 0; r < DF_RT; ++r)
#pragma unroll
        for (int c = 0; c < NT; ++c)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int row = F64 ? (lane >> 4) + 4 * e : 4 * (lane >> 4) + e;
                const long long m = r0 + wave * (16 * DF_RT) + 16 * r + row;
                const int n = c0 + 16 * c + (lane & 15);
                if (m >= g.M || n >= g.N) continue;
                double val;
                if constexpr (FLUSH) val = accd[r][c][e];
                else val = (double)acc[r][c][e];
                if (g.split) {
                    g.part[((long long)z * g.M + m) * g.N + n] = val;
                } else {
                    long long off = (long long)z * g.sC + m * g.ldc + n;
                    if (g.pn > 0) {   // regrouped output (16 consecutive j per row of lanes)
                        const int pn = g.pn, mi = (int)m;
                        const int a = mi / pn, b = mi - a * pn, cq = n / pn, j = n - cq * pn;
                        off = (((long long)b * pn + cq) * pn + a) * pn + j;
                    }
                    OutT *cp = static_cast<OutT *>(g.C) + off;
                    double o = g.alpha * val;
                    if (g.beta != 0.0) o += g.beta * (double)*cp;
                    *cp = (OutT)o;
                }
            }
}

// C(r, c) = alpha sum_z part[z][r][c] + beta C(r, c), slices added in order.
// The same with C(r, c) at C[c ldc + r]: 32 x 32 tiles through LDS, so that both
// the partials and C are read and written along rows.  Block 32 x 8 threads.
template <class OutT>
__global__ void k_df_reduce_t(int M, int N, int nz, const double *__restrict__ part, OutT *C,
                              long long ldc, double alpha, double beta) {
    __shared__ double t[32][33];
    const int r0 = blockIdx.y * 32, c0 = blockIdx.x * 32;
    const int tx = threadIdx.x, ty = threadIdx.y;
    const long long MN = (long long)M * N;
    for (int i = ty; i < 32; i += 8) {
        const int r = r0 + i, c = c0 + tx;
        double s = 0.0;
        if (r < M && c < N)
            for (int z = 0; z < nz; ++z) s += part[z * MN + (long long)r * N + c];
        t[i][tx] = s;
    }
    __syncthreads();
    for (int i = ty; i < 32; i += 8) {
        const int c = c0 + i, r = r0 + tx;
        if (r < M && c < N) {
            OutT *cp = C + (long long)c * ldc + r;
            double o = alpha * t[tx][i];
            if (beta != 0.0) o += beta * (double)*cp;
            *cp = (OutT)o;
        }
    }
}

template <class OutT>
__global__ void k_df_reduce(int M, int N, int nz, const double *__restrict__ part, OutT *C,
                            long long ldc, double alpha, double beta) {
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long MN = (long long)M * N;
    if (idx >= MN) return;
    double s = 0.0;
    for (int z = 0; z < nz; ++z) s += part[z * MN + idx];
    OutT *cp = C + (idx / N) * ldc + idx % N;
    double o = alpha * s;
    if (beta != 0.0) o += beta * (double)*cp;
    *cp = (OutT)o;
}

// B[P][a][b] (FP64) -> B and Bt[a][P][b] in T
template <class T>
__global__ void k_df_layouts(int n, int m, const double *__restrict__ B, T *__restrict__ Bf,
                             T *__restrict__ Bt) {
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long n2 = (long long)n * n;
    if (idx >= n2 * m) return;
    const long long P = idx / n2, ab = idx % n2, a = ab / n, b = ab % n;
    const T x = (T)B[idx];
    Bf[idx] = x;
    Bt[(a * m + P) * n + b] = x;
}

// G = G(tau_k), Gb = G(-tau_k) = -G(tau_{M-k}) in T
template <class T>
__global__ void k_df_stage(int n2, const double *__restrict__ Gk, const double *__restrict__ Gmk,
                           T *__restrict__ G, T *__restrict__ Gb) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n2) return;
    G[idx] = (T)Gk[idx];
    Gb[idx] = (T)(-Gmk[idx]);
}

// Sigma_ij for j < i := Sigma_ji (the product is symmetric up to rounding;
// the returned matrix is exactly symmetric, as the dense path's)
__global__ void k_df_mirror(int n, double *S) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n * n) return;
    const int i = idx / n, j = idx % n;
    if (j < i) S[idx] = S[(long long)j * n + i];
}


// Column tiles per block: ceil(N/16) tiles in the fewest blocks of <= 8, or, when
// those would carry more than 5% idle tiles, in blocks of 4..8 tiles that divide
// them exactly (N = 400: 5 blocks of 5 tiles instead of 4 of 7).
void df_col_blocking(int N, int &nt, int &nblk) {
    const int tiles = (N + 15) / 16;
    nblk = (tiles + 7) / 8;
    nt = (tiles + nblk - 1) / nblk;
    if ((nblk * nt - tiles) * 20 > nblk * nt)
        for (int e = 8; e >= 4; --e)
            if (tiles % e == 0) {
                nt = e;
                nblk = tiles / e;
                break;
            }
}

template <class T, bool AT, bool BT, class OutT>
void df_launch(int nt, dim3 grid, hipStream_t s, const DfGemm &g) {
    // FP32, widest tile, K of the launch within one flush interval: no FP64 copy
    if constexpr (sizeof(T) == 4) {
        if (nt == 8 && (g.split ? g.kz : g.K) <= DF_FLUSH * DF_BK) {
            hipLaunchKernelGGL((k_df_gemm<T, AT, BT, 8, OutT, true>), grid, dim3(DF_THREADS), 0, s, g);
            return;
        }
    }
    switch (nt) {
#define GF2_DF_CASE(N_) \
    case N_: hipLaunchKernelGGL((k_df_gemm<T, AT, BT, N_, OutT, false>), grid, dim3(DF_THREADS), 0, s, g); break;
        GF2_DF_CASE(1) GF2_DF_CASE(2) GF2_DF_CASE(3) GF2_DF_CASE(4)
        GF2_DF_CASE(5) GF2_DF_CASE(6) GF2_DF_CASE(7) GF2_DF_CASE(8)
#undef GF2_DF_CASE
        default: break;
    }
}

// Workgroups a launch should reach before K is split (a few per CU).
constexpr long long DF_TARGET_WG = 1024;
constexpr int DF_MIN_KSLICE = 256;

// One GEMM (batch 1, possibly split along K) or a batch of them.
template <class T, bool AT, bool BT, class OutT>
int df_gemm(gf2_ctx *c, DfGemm g, int batch) {
    int nt, nblk;
    df_col_blocking(g.N, nt, nblk);
    const long long rblk = (g.M + DF_BM - 1) / DF_BM;
    const long long wg = rblk * nblk * batch;
    if (rblk > 0x7fffffffLL || batch > 65535) return fail(GF2_EINVAL, "gf2_sigma_tau_df: problem too large");
    int nz = batch;
    g.split = 0;
    g.kz = g.K;
    if (g.ctrans && batch != 1) return fail(GF2_EINVAL, "gf2_sigma_tau_df: transposed batched GEMM");
    if (g.ctrans && g.pn > 0) return fail(GF2_EINVAL, "gf2_sigma_tau_df: transposed regrouped GEMM");
    if (batch == 1 && g.pn == 0 && (g.ctrans || (wg < DF_TARGET_WG && g.K >= 2 * DF_MIN_KSLICE))) {
        long long s = 1;
        if (wg < DF_TARGET_WG && g.K >= 2 * DF_MIN_KSLICE) {
            s = std::min<long long>((DF_TARGET_WG + wg - 1) / wg, g.K / DF_MIN_KSLICE);
            // up to twice as many slices when that fills the last round of resident
            // workgroups better (two per CU, one for the widest FP32 tile)
            int cus = 256;
            (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->device);
            const double slots = (double)cus * ((sizeof(T) == 8 || nt <= 7) ? 2 : 1);
            auto fill = [&](long long q) {
                const double rounds = (double)(wg * q) / slots;
                return rounds / std::ceil(rounds);
            };
            const long long s0 = s, smax = std::min<long long>(2 * s0, g.K / DF_MIN_KSLICE);
            for (long long q = s0 + 1; q <= smax; ++q)
                if (fill(q) > fill(s) + 0.01) s = q;
        }
        const int kz = (int)(((g.K + s - 1) / s + DF_BK - 1) / DF_BK * DF_BK);
        s = (g.K + kz - 1) / kz;
        if (s > 1 || g.ctrans) {
            GF2_TRY(c->df_part.ensure((size_t)s * g.M * g.N * sizeof(double)));
            g.split = 1;
            g.kz = kz;
            g.part = c->df_part.as<double>();
            nz = (int)s;
        }
    }
    df_launch<T, AT, BT, OutT>(nt, dim3((unsigned)rblk, (unsigned)nblk, (unsigned)nz), c->stream, g);
    GF2_HIP(hipGetLastError());
    if (g.split && g.ctrans) {
        hipLaunchKernelGGL(k_df_reduce_t<OutT>, dim3((unsigned)((g.N + 31) / 32), (unsigned)((g.M + 31) / 32)),
                           dim3(32, 8), 0, c->stream, g.M, g.N, nz, (const double *)g.part,
                           static_cast<OutT *>(g.C), g.ldc, g.alpha, g.beta);
        GF2_HIP(hipGetLastError());
    } else if (g.split) {
        const long long MN = (long long)g.M * g.N;
        hipLaunchKernelGGL(k_df_reduce<OutT>, dim3((unsigned)((MN + 255) / 256)), dim3(256), 0, c->stream,
                           g.M, g.N, nz, (const double *)g.part, static_cast<OutT *>(g.C), g.ldc, g.alpha,
                           g.beta);
        GF2_HIP(hipGetLastError());
    }
    return GF2_OK;
}

DfGemm mk(const void *A, long long lda, const void *B, long long ldb, void *C, long long ldc, int M,
          int N, int K, double alpha = 1.0, double beta = 0.0) {
    DfGemm g{};
    g.A = A; g.lda = lda;
    g.B = B; g.ldb = ldb;
    g.C = C; g.ldc = ldc;
    g.M = M; g.N = N; g.K = K;
    g.alpha = alpha; g.beta = beta;
    return g;
}

// Exchange products held at once: at most this many bytes (whole P slabs).
constexpr size_t DF_T_BYTES = size_t(1) << 30;
// The tensor route's N^4 array may take at most this many bytes.
constexpr size_t DF_V_BYTES = size_t(16) << 30;

// Two evaluations of the exchange term, equal up to rounding:
//   pair route:   U^P += sum_Q (Z^Q Y^P) B^Q, the products of every (P, Q) pair in
//                 chunks of P: 4 m^2 N^3 flops, O(m N^2) memory besides a 1 GiB chunk;
//   tensor route: V[(a,b)][(c,j)] = sum_Q Z^Q_ab B^Q_cj once (one GEMM over Q), then
//                 U^P_aj += sum_{b,c} Y^P_bc V[(a,b)][(c,j)] for all P (one GEMM over
//                 (b, c)): 4 m N^4 flops and one N^4 array (the first GEMM writes V
//                 regrouped as Vp[(b,c)][(a,j)]).
// The tensor route needs fewer flops when m > N (every configuration here), the pair
// route less memory; the tensor route is taken when m > N and its arrays fit in
// DF_V_BYTES.  GF2_DF_ROUTE=pair|tensor in the environment forces one (tests).
template <class T>
int df_run(gf2_ctx *c, const gf2_dims *d, const double *G_tau, double *Sigma_tau) {
    const int N = c->n, m = c->df_m, ntau = d->ntau;
    const long long N2 = (long long)N * N, N4 = N2 * N2, mN = (long long)m * N, mN2 = mN * N;
    bool tensor = m > N && (size_t)N4 * sizeof(T) <= DF_V_BYTES;
    if (const char *e = std::getenv("GF2_DF_ROUTE")) {
        if (e[0] == 'p') tensor = false;
        if (e[0] == 't') tensor = true;
    }
    const size_t slab = (size_t)mN2 * sizeof(T);      // Tx of one P (pair route)
    const int pc = (int)std::max<size_t>(1, std::min<size_t>(m, DF_T_BYTES / slab));
    const size_t ws = (size_t)(2 * N2 + 5 * mN2 + (long long)m * m) * sizeof(T);
    GF2_TRY(c->df_ws.ensure(ws));
    GF2_TRY(c->df_T.ensure(tensor ? (size_t)N4 * sizeof(T) : (size_t)pc * slab));
    T *G = c->df_ws.as<T>(), *Gb = G + N2, *Yt = Gb + N2, *Zt = Yt + mN2, *W = Zt + mN2,
      *U = W + mN2, *Y = U + mN2, *Pi = Y + mN2;
    T *Tx = c->df_T.as<T>();
    T *Vp = Tx;                                      // tensor route
    T *Z = Zt;                                       // tensor route: Z[Q][a][b] in Zt's space
    const T *Bf = sizeof(T) == 8 ? (const T *)c->df_B64.ptr : (const T *)c->df_B32.ptr;
    const T *Bt = sizeof(T) == 8 ? (const T *)c->df_Bt64.ptr : (const T *)c->df_Bt32.ptr;
    const double flops = tensor ? 4.0 * m * (double)N4 + 10.0 * mN2 * N + 4.0 * m * (double)m * N2
                                : 4.0 * m * (double)m * N2 * N + 4.0 * m * (double)m * N2 + 8.0 * mN2 * N;

    for (int k = 0; k < ntau; ++k) {
        const int ph = c->prof ? prof_begin(c, GF2_KC_SIGMA_DF) : -1;
        hipLaunchKernelGGL(k_df_stage<T>, dim3((unsigned)((N2 + 255) / 256)), dim3(256), 0, c->stream,
                           (int)N2, G_tau + k * N2, G_tau + (long long)(ntau - 1 - k) * N2, G, Gb);
        GF2_HIP(hipGetLastError());
        // Yt = Bt G (rows (i, P))
        GF2_TRY((df_gemm<T, false, false, T>(c, mk(Bt, N, G, N, Yt, N, (int)mN, N, N), 1)));
        // W^Q = Gb Y^Q, Y^Q(b, c) = Yt[b][Q][c]
        {
            DfGemm g = mk(Gb, N, Yt, mN, W, N, N, N, N);
            g.sA = 0; g.sB = N; g.sC = N2;
            GF2_TRY((df_gemm<T, false, false, T>(c, g, m)));
        }
        // Pi_PQ = sum_k B[P][k] W[Q][k]
        GF2_TRY((df_gemm<T, false, true, T>(c, mk(Bf, N2, W, N2, Pi, m, m, m, (int)N2), 1)));
        // U = -2 Pi B
        GF2_TRY((df_gemm<T, false, false, T>(c, mk(Pi, m, Bf, N2, U, N2, m, (int)N2, m, -2.0), 1)));
        if (tensor) {
            // Y[P][b][c] = B^P G, Z[Q][a][b] = B^Q Gb (rows (P, b) of B)
            GF2_TRY((df_gemm<T, false, false, T>(c, mk(Bf, N, G, N, Y, N, (int)mN, N, N), 1)));
            GF2_TRY((df_gemm<T, false, false, T>(c, mk(Bf, N, Gb, N, Z, N, (int)mN, N, N), 1)));
            // V[(a,b)][(c,j)] = sum_Q Z[Q][(a,b)] B[Q][(c,j)], written regrouped as
            // Vp[(b,c)][(a,j)] by the GEMM's epilogue
            {
                DfGemm g = mk(Z, N2, Bf, N2, Vp, N2, (int)N2, (int)N2, m);
                g.pn = N;
                GF2_TRY((df_gemm<T, true, false, T>(c, g, 1)));
            }
            // U[P][(a,j)] += sum_{(b,c)} Y[P][(b,c)] Vp[(b,c)][(a,j)], computed as its
            // transpose (rows (a, j), columns P): the m columns then fill whole
            // 16-wide tiles (the m rows of the direct form fill 128-row blocks only
            // partly: 400 of 512), and the reduction adds it into U transposed back
            DfGemm g = mk(Vp, N2, Y, N2, U, N2, (int)N2, m, (int)N2, 1.0, 1.0);
            g.ctrans = 1;
            GF2_TRY((df_gemm<T, true, true, T>(c, g, 1)));
        } else {
            // Zt = Bt Gb; Tx^P = Zt Y^P, then U[P0 ..] += Tx B
            GF2_TRY((df_gemm<T, false, false, T>(c, mk(Bt, N, Gb, N, Zt, N, (int)mN, N, N), 1)));
            for (int P0 = 0; P0 < m; P0 += pc) {
                const int np = std::min(pc, m - P0);
                DfGemm g = mk(Zt, N, Yt + (long long)P0 * N, mN, Tx, N, (int)mN, N, N);
                g.sA = 0; g.sB = N; g.sC = mN2;
                GF2_TRY((df_gemm<T, false, false, T>(c, g, np)));
                GF2_TRY((df_gemm<T, false, false, T>(c, mk(Tx, mN, Bf, N, U + (long long)P0 * N2, N, np * N,
                                                          N, (int)mN, 1.0, 1.0), 1)));
            }
        }
        // Sigma(tau_k) = Yt U (K = (P, b))
        double *Sk = Sigma_tau + k * N2;
        GF2_TRY((df_gemm<T, false, false, double>(c, mk(Yt, mN, U, N, Sk, N, N, N, (int)mN), 1)));
        hipLaunchKernelGGL(k_df_mirror, dim3((unsigned)((N2 + 255) / 256)), dim3(256), 0, c->stream, N, Sk);
        GF2_HIP(hipGetLastError());
        if (c->prof) prof_end(c, ph, flops);
    }
    return GF2_OK;
}

}  // namespace

int sigma_df_run(gf2_ctx *c, const gf2_dims *d, int prec, const double *G_tau, double *Sigma_tau) {
    if (c->df_m < 1) return fail(GF2_ESTATE, "Sigma(tau) from factors: no density-fitting factors set");
    if (prec == GF2_PREC_FP64) return df_run<double>(c, d, G_tau, Sigma_tau);
    if (prec == GF2_PREC_FP32) return df_run<float>(c, d, G_tau, Sigma_tau);
    return fail(GF2_EINVAL, "Sigma(tau) from factors: prec must be GF2_PREC_FP64 or GF2_PREC_FP32");
}

}  // namespace gf2

using namespace gf2;

extern "C" int gf2_set_df_factors(gf2_ctx *c, int naux, const double *B) {
    if (!c || !B) return fail(GF2_EINVAL, "gf2_set_df_factors: NULL argument");
    if (naux < 1) return fail(GF2_EINVAL, "gf2_set_df_factors: naux must be >= 1");
    if (!c->has_system) return fail(GF2_ESTATE, "gf2_set_df_factors: no system set");
    GF2_HIP(hipSetDevice(c->device));
    c->df_m = 0;
    const size_t cnt = (size_t)naux * c->n * c->n;
    GF2_TRY(c->df_B64.ensure(cnt * sizeof(double)));
    GF2_TRY(c->df_Bt64.ensure(cnt * sizeof(double)));
    GF2_TRY(c->df_B32.ensure(cnt * sizeof(float)));
    GF2_TRY(c->df_Bt32.ensure(cnt * sizeof(float)));
    const unsigned blocks = (unsigned)((cnt + 255) / 256);
    hipLaunchKernelGGL(k_df_layouts<double>, dim3(blocks), dim3(256), 0, c->stream, c->n, naux, B,
                       c->df_B64.as<double>(), c->df_Bt64.as<double>());
    GF2_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_df_layouts<float>, dim3(blocks), dim3(256), 0, c->stream, c->n, naux, B,
                       c->df_B32.as<float>(), c->df_Bt32.as<float>());
    GF2_HIP(hipGetLastError());
    c->df_m = naux;
    return GF2_OK;
}

extern "C" int gf2_sigma_tau_df(gf2_ctx *c, const gf2_dims *d, int prec, const double *G_tau,
                                double *Sigma_tau) {
    if (!c || !d || !G_tau || !Sigma_tau) return fail(GF2_EINVAL, "gf2_sigma_tau_df: NULL argument");
    if (!c->has_system) return fail(GF2_ESTATE, "gf2_sigma_tau_df: no system set");
    if (c->df_m < 1) return fail(GF2_ESTATE, "gf2_sigma_tau_df: no density-fitting factors set");
    if (d->n != c->n) return fail(GF2_EINVAL, "gf2_sigma_tau_df: dims->n differs from the system");
    if (d->ntau < 4) return fail(GF2_EINVAL, "gf2_sigma_tau_df: ntau must be >= 4");
    if (prec != GF2_PREC_FP64 && prec != GF2_PREC_FP32)
        return fail(GF2_EINVAL, "gf2_sigma_tau_df: prec must be GF2_PREC_FP64 or GF2_PREC_FP32");
    if ((const void *)G_tau == (const void *)Sigma_tau)
        return fail(GF2_EINVAL, "gf2_sigma_tau_df: Sigma_tau aliases G_tau");
    GF2_HIP(hipSetDevice(c->device));
    GF2_TRY(sigma_df_run(c, d, prec, G_tau, Sigma_tau));
    int bad = 0;
    GF2_TRY(any_nonfinite(c, (size_t)d->ntau * d->n * d->n, Sigma_tau, &bad));
    if (bad) return fail(GF2_ENONFINITE, "gf2_sigma_tau_df: non-finite self-energy");
    return GF2_OK;
}
