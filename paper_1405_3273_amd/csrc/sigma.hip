// Eq. (Sigma): the second-order self-energy in imaginary time on MFMA.
//
// For every tau point (G = G(tau), Gb = G(-tau) = -G(beta - tau)) the
// six-index sum is evaluated as four index transforms of 2 N^5 flops each:
//
//   S1   T1[i][n][q][k] = sum_m G[m][n] v_imqk                (GEMM batched over i)
//   S23  X[i][n][p][l]  = sum_{q,k} Gb[q][p] T1[i][n][q][k] G[k][l]
//                         (two products per N x N slab, fused in one kernel)
//   S4   Sigma[i][j]    = - sum_{n,p,l} X[i][n][p][l] W2[n][p][l][j]
//                         W2[n][p][l][j] = 2 v_lpnj - v_nplj   (split-K GEMM, K = N^3)
//
// A batch of b tau points runs per pass: S1 stacks the b G matrices along
// its rows, S23 and S4 index the batch in their grids/rows.  G is symmetric,
// so G and Gb are used as stored.  The split-K partial sums of S4 are added
// in FP64 in a fixed order, so results do not depend on scheduling.
//
// Arithmetic: FP64 MFMA (v_mfma_f64_16x16x4f64), FP32 MFMA
// (v_mfma_f32_16x16x4f32), or split BF16 on v_mfma_f32_16x16x32_bf16 with
// FP32 accumulation: each FP32 operand x is split into bf16 terms
// x = h + m (+ l), and of the products of the terms those of order 1 and
// 2^-8 (BF16x3: h*h, h*m, m*h) or also 2^-16 (BF16x6: m*m, h*l, l*h) are
// issued (the two- and three-term splits of Henry, Tang and Heinecke, "Leveraging
// the bfloat16 artificial intelligence datatype for higher-precision
// computations", ARITH 2019).  In S4 the FP32 accumulators are flushed into
// FP64 registers every 512 K.
#include "gf2_internal.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <type_traits>
#include <vector>

namespace gf2 {

// ---------------------------------------------------------------------------
// XCD-aware block order.  Consecutive workgroup ids are handed to the 8 XCDs
// in turn; the remap gives every XCD a contiguous range of logical blocks, so
// blocks that share operands (neighbouring logical ids) share one L2.  The
// grid is launched with 8 * ceil(total / 8) blocks; ids past `total` exit.
constexpr int NXCD = 8;
__device__ __forceinline__ int xcd_logical(int total) {
    const int per = (total + NXCD - 1) / NXCD;
    return (int)(blockIdx.x % NXCD) * per + (int)(blockIdx.x / NXCD);
}
static unsigned xcd_grid(long long total) {
    return (unsigned)(((total + NXCD - 1) / NXCD) * NXCD);
}


typedef float v4f __attribute__((ext_vector_type(4)));
typedef double v4d __attribute__((ext_vector_type(4)));
typedef double v2d __attribute__((ext_vector_type(2)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef unsigned short v8us __attribute__((ext_vector_type(8)));

template <int MODE> struct ModeT;
template <> struct ModeT<MODE_F64> { using in_t = double; using acc_t = v4d; static constexpr int BK = 16; };
template <> struct ModeT<MODE_F32> { using in_t = float;  using acc_t = v4f; static constexpr int BK = 16; };
template <> struct ModeT<MODE_BF3> { using in_t = float;  using acc_t = v4f; static constexpr int BK = 32; };
template <> struct ModeT<MODE_BF6> { using in_t = float;  using acc_t = v4f; static constexpr int BK = 32; };

struct GemmArgs {
    const void *A;
    long long lda, sA;   // A(k, m) = A[k*lda + m] (k-major) or A[m*lda + k] (m-major)
    const void *B;
    long long ldb, sB;   // B(k, n) = B[k*ldb + n]
    void *C;
    long long ldc, sC;   // C[m*ldc + n]
    int M, N, K;         // K: total reduction length
    int kz;              // K handled per z index when split != 0
    int split;           // z indexes K slices (1) or independent batches (0)
    double alpha;
    int vecA;            // 1 if 4-element vector loads of A are aligned
    // bf16 hi/lo plane output (gemm_bf3<.., PLANES = true>): column n = q*pn + k
    // goes to C[z*sC + m*ldc + q*pld + k] (hi) and the same index + plane (lo)
    int pn, pld;
    long long plane;
    // XCD-ordered 1-D launch when gx > 0: logical block (x, y, z), x fastest,
    // so the row blocks that share a B column block run on one XCD
    int gx, gy, gz;
};

// Kernel argument of the Sigma kernels: one problem (nsys == 0, the args
// themselves) or a table of problems of many systems run by one launch.  The
// launch is a 1-D grid in XCD order over `total` logical blocks; system s owns
// logical blocks [boff[s], boff[s+1]) and gets its own block index from 0.
template <class A> struct KRef {
    A one;
    const A *tab;
    const int *boff;
    int nsys;
    int total;
};

// a, L: the problem of this workgroup and its local logical block (false:
// an id past the padded grid).  Single problems give `total_one` blocks.
template <class A>
__device__ __forceinline__ bool kresolve(const KRef<A> &r, int total_one, A &a, int &L) {
    if (r.nsys == 0) {
        L = xcd_logical(total_one);
        if (L >= total_one) return false;
        a = r.one;
        return true;
    }
    const int Lg = xcd_logical(r.total);
    if (Lg >= r.total) return false;
    int sys = 0;
    while (sys + 1 < r.nsys && r.boff[sys + 1] <= Lg) ++sys;
    sys = __builtin_amdgcn_readfirstlane(sys);
    a = r.tab[sys];
    L = Lg - r.boff[sys];
    return true;
}

// Block coordinates of a GEMM workgroup (false: an id past the XCD-padded grid).
// gx > 0: logical (x, y, z), x fastest, from the XCD-ordered 1-D grid (single
// problem or a table); gx == 0: the 3-D grid as launched (single problem only).
__device__ __forceinline__ bool gemm_block(const KRef<GemmArgs> &r, GemmArgs &g, int &bx, int &by,
                                           int &bz) {
    if (r.nsys == 0 && r.one.gx <= 0) {
        g = r.one;
        bx = blockIdx.x;
        by = blockIdx.y;
        bz = blockIdx.z;
        return true;
    }
    int L;
    if (!kresolve(r, r.one.gx * r.one.gy * r.one.gz, g, L)) return false;
    bx = L % g.gx;
    by = (L / g.gx) % g.gy;
    bz = L / (g.gx * g.gy);
    return true;
}

constexpr int NTHREADS = 256;
constexpr int BM = 128;  // 4 waves x 2 row tiles x 16
constexpr int RT = 2;    // row tiles per wave

// NP-term split, x = o[0] + ... + o[NP-1] + O(2^-8NP |x|): each term is the
// bf16 rounding (nearest even, v_cvt_pk_bf16_f32) of the residual, which is
// exact in FP32.  The first two terms of the three-term split are the
// two-term split.
template <int NP>
__device__ __forceinline__ void split_bf16n(float x, unsigned short (&o)[NP]) {
#pragma unroll
    for (int i = 0; i < NP; ++i) {
        const __bf16 h = (__bf16)x;
        o[i] = __builtin_bit_cast(unsigned short, h);
        x -= (float)h;
    }
}

// The same split for two values at once, one 32-bit word per plane (x0's term
// in the low half, x1's in the high half: two consecutive elements of a bf16
// vector).  One v_cvt_pk_bf16_f32 rounds both (nearest even, as the scalar
// conversion), and the terms return to FP32 by a shift or a mask, so the planes
// are bitwise those of split_bf16n at half the instructions.
typedef float v2f_t __attribute__((ext_vector_type(2)));
typedef __bf16 v2bf_t __attribute__((ext_vector_type(2)));
template <int NP>
__device__ __forceinline__ void split_pair(float x0, float x1, unsigned (&w)[NP]) {
#pragma unroll
    for (int i = 0; i < NP; ++i) {
        const unsigned u = __builtin_bit_cast(unsigned, __builtin_convertvector(v2f_t{x0, x1}, v2bf_t));
        w[i] = u;
        if (i + 1 < NP) {
            x0 -= __uint_as_float(u << 16);
            x1 -= __uint_as_float(u & 0xffff0000u);
        }
    }
}

// Eight values into NP bf16 vectors of 8 (one per plane).
typedef unsigned v4u_t __attribute__((ext_vector_type(4)));
template <int NP>
__device__ __forceinline__ void split8(const float (&x)[8], v8us (&o)[NP]) {
    unsigned w[4][NP];
#pragma unroll
    for (int e = 0; e < 4; ++e) split_pair<NP>(x[2 * e], x[2 * e + 1], w[e]);
#pragma unroll
    for (int pl = 0; pl < NP; ++pl)
        o[pl] = __builtin_bit_cast(v8us, v4u_t{w[0][pl], w[1][pl], w[2][pl], w[3][pl]});
}

template <class T> __device__ __forceinline__ T ldg(const T *p) { return *p; }

// ---------------------------------------------------------------------------
// FP64 / FP32 kernel: LDS tiles As[k][m], Bs[k][n]
// OUT64: FP64 output (FP32 accumulators flushed into FP64 every 512 K);
// BK_: K chunk (0 = the mode's default; the k-major form needs 16).
template <int MODE, bool AK, int NT, bool OUT64, int BK_>
__global__ __launch_bounds__(NTHREADS) void gemm_fp(KRef<GemmArgs> r) {
    using in_t = typename ModeT<MODE>::in_t;
    using acc_t = typename ModeT<MODE>::acc_t;
    constexpr int BK = BK_ ? BK_ : ModeT<MODE>::BK;
    static_assert(!AK || BK == 16, "k-major A loads assume 16-element chunks");
    static_assert(BK % 4 == 0 && (BK * BM) % NTHREADS == 0, "bad chunk");
    constexpr int BN = 16 * NT;
    constexpr int SA = BM + 16;                       // padded row strides
    constexpr int SB = BN + ((16 - BN % 32) + 32) % 32;
    constexpr int FLUSH = 512 / BK;                   // chunks between FP64 flushes

    __shared__ in_t As[BK][SA];
    __shared__ in_t Bs[BK][SB];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    GemmArgs g;
    int bx, by, z;
    if (!gemm_block(r, g, bx, by, z)) return;
    const long long mb = (long long)bx * BM;
    const int nb = by * BN;

    const GF2_GLOBAL in_t *A = (const GF2_GLOBAL in_t *)g.A + (long long)z * g.sA;
    const GF2_GLOBAL in_t *B = (const GF2_GLOBAL in_t *)g.B + (long long)z * g.sB;
    const int Kz = g.split ? min(g.kz, g.K - z * g.kz) : g.K;
    if (Kz <= 0) return;

    acc_t acc[RT][NT];
    double accd[RT][NT][4];
#pragma unroll
    for (int r = 0; r < RT; ++r)
#pragma unroll
        for (int c = 0; c < NT; ++c) {
            acc[r][c] = acc_t{0, 0, 0, 0};
#pragma unroll
            for (int e = 0; e < 4; ++e) accd[r][c][e] = 0.0;
        }

    // register staging of the next chunk
    constexpr int A_PER = BK * BM / NTHREADS;   // 8
    constexpr int B_PER = (BK * BN + NTHREADS - 1) / NTHREADS;
    in_t ra[A_PER];
    in_t rb[B_PER];

    auto load_chunk = [&](int kb) {
        if constexpr (AK) {
            const int kk = tid / (BM / A_PER);
            const int mm = (tid % (BM / A_PER)) * A_PER;
            const long long gk = kb + kk;
            const long long gm = mb + mm;
            const GF2_GLOBAL in_t *p = A + gk * g.lda + gm;
            if (gk < Kz && gm + A_PER <= g.M && g.vecA) {
                if constexpr (MODE == MODE_F64) {
#pragma unroll
                    for (int e = 0; e < A_PER; e += 2) {
                        const v2d t = *(const GF2_GLOBAL v2d *)(p + e);
                        ra[e] = t.x;
                        ra[e + 1] = t.y;
                    }
                } else {
#pragma unroll
                    for (int e = 0; e < A_PER; e += 4) {
                        const v4f t = *(const GF2_GLOBAL v4f *)(p + e);
                        ra[e] = t.x; ra[e + 1] = t.y; ra[e + 2] = t.z; ra[e + 3] = t.w;
                    }
                }
            } else {
#pragma unroll
                for (int e = 0; e < A_PER; ++e)
                    ra[e] = (gk < Kz && gm + e < g.M) ? p[e] : in_t(0);
            }
        } else {
#pragma unroll
            for (int e = 0; e < A_PER; ++e) {
                const int idx = tid + e * NTHREADS;
                const int m = idx / BK, k = idx % BK;
                const long long gm = mb + m, gk = kb + k;
                ra[e] = (gm < g.M && gk < Kz) ? A[gm * g.lda + gk] : in_t(0);
            }
        }
#pragma unroll
        for (int e = 0; e < B_PER; ++e) {
            const int idx = tid + e * NTHREADS;
            const int k = idx / BN, n = idx % BN;
            const long long gk = kb + k;
            const int gn = nb + n;
            rb[e] = (idx < BK * BN && gk < Kz && gn < g.N) ? B[gk * g.ldb + gn] : in_t(0);
        }
    };
    auto store_chunk = [&]() {
        if constexpr (AK) {
            const int kk = tid / (BM / A_PER);
            const int mm = (tid % (BM / A_PER)) * A_PER;
#pragma unroll
            for (int e = 0; e < A_PER; ++e) As[kk][mm + e] = ra[e];
        } else {
#pragma unroll
            for (int e = 0; e < A_PER; ++e) {
                const int idx = tid + e * NTHREADS;
                As[idx % BK][idx / BK] = ra[e];
            }
        }
#pragma unroll
        for (int e = 0; e < B_PER; ++e) {
            const int idx = tid + e * NTHREADS;
            if (idx < BK * BN) Bs[idx / BN][idx % BN] = rb[e];
        }
    };

    const int nchunks = (Kz + BK - 1) / BK;
    load_chunk(0);
    for (int ch = 0; ch < nchunks; ++ch) {
        __syncthreads();
        store_chunk();
        __syncthreads();
        if (ch + 1 < nchunks) load_chunk((ch + 1) * BK);
#pragma unroll
        for (int k0 = 0; k0 < BK; k0 += 4) {
            const int kr = k0 + (lane >> 4);
            in_t af[RT], bf[NT];
#pragma unroll
            for (int r = 0; r < RT; ++r) af[r] = As[kr][wave * (16 * RT) + r * 16 + (lane & 15)];
#pragma unroll
            for (int c = 0; c < NT; ++c) bf[c] = Bs[kr][c * 16 + (lane & 15)];
#pragma unroll
            for (int r = 0; r < RT; ++r)
#pragma unroll
                for (int c = 0; c < NT; ++c) {
                    if constexpr (MODE == MODE_F64)
                        acc[r][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[r], bf[c], acc[r][c], 0, 0, 0);
                    else
                        acc[r][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[r], bf[c], acc[r][c], 0, 0, 0);
                }
        }
        if constexpr (OUT64 && MODE != MODE_F64) {
            if ((ch + 1) % FLUSH == 0 || ch + 1 == nchunks) {
#pragma unroll
                for (int r = 0; r < RT; ++r)
#pragma unroll
                    for (int c = 0; c < NT; ++c) {
#pragma unroll
                        for (int e = 0; e < 4; ++e) accd[r][c][e] += (double)acc[r][c][e];
                        acc[r][c] = acc_t{0, 0, 0, 0};
                    }
            }
        }
    }

    // epilogue: register e of a lane holds row 4*(lane/16) + e (FP32 MFMA) or
    // row lane/16 + 4*e (FP64 MFMA), column lane%16, of each 16x16 tile
#pragma unroll
    for (int r = 0; r < RT; ++r)
#pragma unroll
        for (int c = 0; c < NT; ++c)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int row = (MODE == MODE_F64) ? ((lane >> 4) + 4 * e) : (4 * (lane >> 4) + e);
                const long long m = mb + wave * (16 * RT) + r * 16 + row;
                const int n = nb + c * 16 + (lane & 15);
                if (m < g.M && n < g.N) {
                    if constexpr (OUT64) {
                        double val;
                        if constexpr (MODE == MODE_F64) val = acc[r][c][e];
                        else val = accd[r][c][e];
                        ((GF2_GLOBAL double *)g.C)[(long long)z * g.sC + m * g.ldc + n] = g.alpha * val;
                    } else {
                        ((GF2_GLOBAL in_t *)g.C)[(long long)z * g.sC + m * g.ldc + n] =
                            (in_t)(g.alpha * (double)acc[r][c][e]);
                    }
                }
            }
}

// ---------------------------------------------------------------------------
// Split-BF16 kernel: FP32 operands split into NP bf16 planes in LDS, tiles
// As[m][k], Bs[n][k]; NP = 2 (BF16x3) or 3 (BF16x6).
// PLANES: output split into NP bf16 planes (see GemmArgs), else FP32.
template <int NP>
__device__ __forceinline__ v4f mma_split(const v8bf (&a)[NP], const v8bf (&b)[NP], v4f acc) {
    // smallest terms first
    if constexpr (NP == 3) {
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1], b[1], acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0], b[2], acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[2], b[0], acc, 0, 0, 0);
    }
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0], b[1], acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1], b[0], acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0], b[0], acc, 0, 0, 0);
    return acc;
}

template <bool AK, int NT, bool PLANES, int NP>
__global__ __launch_bounds__(NTHREADS) void gemm_bf3(KRef<GemmArgs> r) {
    constexpr int BK = 32;
    constexpr int BN = 16 * NT;
    constexpr int SK = BK + 8;       // padded k stride (bf16 elements)

    __shared__ __attribute__((aligned(16))) unsigned short As[NP][BM][SK];
    __shared__ __attribute__((aligned(16))) unsigned short Bs[NP][BN][SK];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    GemmArgs g;
    int bx, by, z;
    if (!gemm_block(r, g, bx, by, z)) return;
    const long long mb = (long long)bx * BM;
    const int nb = by * BN;

    const GF2_GLOBAL float *A = (const GF2_GLOBAL float *)g.A + (long long)z * g.sA;
    const GF2_GLOBAL float *B = (const GF2_GLOBAL float *)g.B + (long long)z * g.sB;
    const int Kz = g.split ? min(g.kz, g.K - z * g.kz) : g.K;
    if (Kz <= 0) return;

    v4f acc[RT][NT];
#pragma unroll
    for (int r = 0; r < RT; ++r)
#pragma unroll
        for (int c = 0; c < NT; ++c) acc[r][c] = v4f{0, 0, 0, 0};

    // A staging: each thread owns one row m and 16 consecutive k (BM*BK/256 = 16)
    const int a_m = AK ? (tid % BM) : (tid / 2);
    const int a_k0 = AK ? (tid / BM) * 16 : (tid % 2) * 16;
    float ra[16];
    // B staging: (n, 8 consecutive k) groups; BN*4 groups
    constexpr int BG = BN * (BK / 8);
    constexpr int B_ITERS = (BG + NTHREADS - 1) / NTHREADS;
    float rb[B_ITERS][8];

    auto load_chunk = [&](int kb) {
        const long long gm = mb + a_m;
        if constexpr (AK) {
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                const long long gk = kb + a_k0 + e;
                ra[e] = (gm < g.M && gk < Kz) ? A[gk * g.lda + gm] : 0.0f;
            }
        } else {
            const long long gk = kb + a_k0;
            const GF2_GLOBAL float *p = A + gm * g.lda + gk;
            if (gm < g.M && gk + 16 <= Kz && g.vecA) {
#pragma unroll
                for (int e = 0; e < 16; e += 4) {
                    const v4f t = *(const GF2_GLOBAL v4f *)(p + e);
                    ra[e] = t.x; ra[e + 1] = t.y; ra[e + 2] = t.z; ra[e + 3] = t.w;
                }
            } else {
#pragma unroll
                for (int e = 0; e < 16; ++e) ra[e] = (gm < g.M && gk + e < Kz) ? p[e] : 0.0f;
            }
        }
#pragma unroll
        for (int it = 0; it < B_ITERS; ++it) {
            const int grp = tid + it * NTHREADS;
            const int n = grp % BN, kg = grp / BN;
            const int gn = nb + n;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const long long gk = kb + kg * 8 + e;
                rb[it][e] = (grp < BG && gn < g.N && gk < Kz) ? B[gk * g.ldb + gn] : 0.0f;
            }
        }
    };
    auto store_chunk = [&]() {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            float x8[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) x8[e] = ra[h * 8 + e];
            v8us t[NP];
            split8<NP>(x8, t);
#pragma unroll
            for (int pl = 0; pl < NP; ++pl)
                *reinterpret_cast<v8us *>(&As[pl][a_m][a_k0 + h * 8]) = t[pl];
        }
#pragma unroll
        for (int it = 0; it < B_ITERS; ++it) {
            const int grp = tid + it * NTHREADS;
            if (grp < BG) {
                const int n = grp % BN, kg = grp / BN;
                v8us t[NP];
                split8<NP>(rb[it], t);
#pragma unroll
                for (int pl = 0; pl < NP; ++pl)
                    *reinterpret_cast<v8us *>(&Bs[pl][n][kg * 8]) = t[pl];
            }
        }
    };

    const int nchunks = (Kz + BK - 1) / BK;
    load_chunk(0);
    for (int ch = 0; ch < nchunks; ++ch) {
        __syncthreads();
        store_chunk();
        __syncthreads();
        if (ch + 1 < nchunks) load_chunk((ch + 1) * BK);
        const int kq = (lane >> 4) * 8;
        v8bf av[RT][NP];
#pragma unroll
        for (int r = 0; r < RT; ++r) {
            const int m = wave * (16 * RT) + r * 16 + (lane & 15);
#pragma unroll
            for (int pl = 0; pl < NP; ++pl)
                av[r][pl] = __builtin_bit_cast(v8bf, *reinterpret_cast<const v8us *>(&As[pl][m][kq]));
        }
#pragma unroll
        for (int c = 0; c < NT; ++c) {
            const int n = c * 16 + (lane & 15);
            v8bf bv[NP];
#pragma unroll
            for (int pl = 0; pl < NP; ++pl)
                bv[pl] = __builtin_bit_cast(v8bf, *reinterpret_cast<const v8us *>(&Bs[pl][n][kq]));
#pragma unroll
            for (int r = 0; r < RT; ++r) acc[r][c] = mma_split<NP>(av[r], bv, acc[r][c]);
        }
    }

#pragma unroll
    for (int c = 0; c < NT; ++c) {
        const int n = nb + c * 16 + (lane & 15);
        int pq = 0, pk = 0;
        if constexpr (PLANES) {
            pq = n / g.pn;
            pk = n - pq * g.pn;
        }
#pragma unroll
        for (int r = 0; r < RT; ++r)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const long long m = mb + wave * (16 * RT) + r * 16 + 4 * (lane >> 4) + e;
                if (m < g.M && n < g.N) {
                    const float x = (float)(g.alpha * (double)acc[r][c][e]);
                    if constexpr (PLANES) {
                        unsigned short o[NP];
                        split_bf16n<NP>(x, o);
                        GF2_GLOBAL unsigned short *C = (GF2_GLOBAL unsigned short *)g.C;
                        const long long idx = (long long)z * g.sC + m * g.ldc + (long long)pq * g.pld + pk;
#pragma unroll
                        for (int pl = 0; pl < NP; ++pl) C[idx + pl * g.plane] = o[pl];
                    } else {
                        ((GF2_GLOBAL float *)g.C)[(long long)z * g.sC + m * g.ldc + n] = x;
                    }
                }
            }
    }
}

// ---------------------------------------------------------------------------
// host-side dispatch

// OUT64: FP64 output for gemm_fp; for gemm_bf3 it selects the hi/lo plane output.
template <int MODE, bool AK, bool OUT64, int BK_>
static void launch_nt(int nt, dim3 grid, hipStream_t s, const KRef<GemmArgs> &r) {
#define GF2_NT_CASE(T)                                                                      \
    case T:                                                                                 \
        if constexpr (split_planes(MODE) > 0)                                               \
            hipLaunchKernelGGL((gemm_bf3<AK, T, OUT64, split_planes(MODE)>), grid,           \
                               dim3(NTHREADS), 0, s, r);                                    \
        else                                                                                \
            hipLaunchKernelGGL((gemm_fp<MODE, AK, T, OUT64, BK_>), grid, dim3(NTHREADS), 0, s, r); \
        break;
    switch (nt) {
        GF2_NT_CASE(1) GF2_NT_CASE(2) GF2_NT_CASE(3) GF2_NT_CASE(4)
        GF2_NT_CASE(5) GF2_NT_CASE(6) GF2_NT_CASE(7) GF2_NT_CASE(8)
        default: break;
    }
#undef GF2_NT_CASE
}

// Column tiles per block: split ceil(N/16) tiles into the fewest blocks of <= 8.
static void col_blocking(int N, int &nt, int &nblocks) {
    int tiles = (N + 15) / 16;
    nblocks = (tiles + 7) / 8;
    nt = (tiles + nblocks - 1) / nblocks;
}

static dim3 gemm_grid(const GemmArgs &g, int zcount, int &nt) {
    int nblk;
    col_blocking(g.N, nt, nblk);
    return dim3((unsigned)((g.M + BM - 1) / BM), (unsigned)nblk, (unsigned)zcount);
}

int gemm_f64_kmajor(gf2_ctx *c, const GemmArgsF64 &a) {
    GemmArgs g{};
    g.A = a.A; g.lda = a.lda; g.sA = 0;
    g.B = a.B; g.ldb = a.ldb; g.sB = 0;
    g.C = a.C; g.ldc = a.ldc; g.sC = 0;
    g.M = a.M; g.N = a.N; g.K = a.K; g.kz = a.K; g.split = 0;
    g.alpha = a.alpha;
    g.vecA = (a.lda % 2 == 0) ? 1 : 0;
    int nt;
    const dim3 grid = gemm_grid(g, 1, nt);
    KRef<GemmArgs> r{};
    r.one = g;
    launch_nt<MODE_F64, true, true, 0>(nt, grid, c->stream, r);
    GF2_HIP(hipGetLastError());
    return GF2_OK;
}

// k / n for k < 2^22 (K = n^3 <= 160^3): the float quotient is within 1/8 of
// k / n, so its truncation is off by at most one and one correction fixes it.
__device__ __forceinline__ unsigned udiv22(unsigned k, unsigned n, float inv_n) {
    unsigned q = (unsigned)((float)k * inv_n);
    const int r = (int)k - (int)(q * n);
    if (r < 0) --q;
    else if (r >= (int)n) ++q;
    return q;
}

// ---------------------------------------------------------------------------
// layouts of v (built once per system)

// W2[n][p][l][j] = 2 v_lpnj - v_nplj (idx = ((n*N + p)*N + l)*N + j)
template <class T>
__global__ void k_build_w2(int n, const double *__restrict__ v, T *__restrict__ W2) {
    const size_t n2 = (size_t)n * n, n3 = n2 * n, n4 = n3 * n;
    for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < n4;
         idx += (size_t)gridDim.x * blockDim.x) {
        const size_t a = idx / n3, b = (idx / n2) % n, cc = (idx / n) % n, d = idx % n;
        W2[idx] = (T)(2.0 * v[((cc * n + b) * n + a) * n + d] - v[((a * n + b) * n + cc) * n + d]);
    }
}

__global__ void k_to_f32(size_t count, const double *__restrict__ x, float *__restrict__ y) {
    for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < count;
         idx += (size_t)gridDim.x * blockDim.x)
        y[idx] = (float)x[idx];
}

int sigma_build_layouts(gf2_ctx *c, bool want_f32) {
    const size_t n = c->n, n4 = n * n * n * n;
    const unsigned blocks = (unsigned)std::min<size_t>((n4 + 255) / 256, 65536);
    GF2_TRY(c->W2_64.ensure(n4 * 8));
    hipLaunchKernelGGL(k_build_w2<double>, dim3(blocks), dim3(256), 0, c->stream, (int)n,
                       c->v.as<double>(), c->W2_64.as<double>());
    GF2_HIP(hipGetLastError());
    if (want_f32) {
        GF2_TRY(c->v_32.ensure(n4 * 4));
        GF2_TRY(c->W2_32.ensure(n4 * 4));
        hipLaunchKernelGGL(k_to_f32, dim3(blocks), dim3(256), 0, c->stream, n4,
                           c->v.as<double>(), c->v_32.as<float>());
        GF2_HIP(hipGetLastError());
        hipLaunchKernelGGL(k_build_w2<float>, dim3(blocks), dim3(256), 0, c->stream, (int)n,
                           c->v.as<double>(), c->W2_32.as<float>());
        GF2_HIP(hipGetLastError());
        c->have_f32_layouts = true;
    }
    return GF2_OK;
}

// ---------------------------------------------------------------------------
// per-batch staging
//
// Gs[t] = G(tau_{k0+t}), Gbs[t] = G(-tau_{k0+t}) = -G(tau_{M-k0-t})   ([nb][n][n])
template <class T>
__global__ void k_stage_g(int n, int M, int k0, int nb, const double *__restrict__ Gt,
                          T *__restrict__ Gs, T *__restrict__ Gbs) {
    const size_t n2 = (size_t)n * n;
    const size_t total = n2 * nb;
    for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < total;
         idx += (size_t)gridDim.x * blockDim.x) {
        const size_t t = idx / n2, e = idx % n2;
        const size_t k = k0 + t;
        Gs[idx] = (T)Gt[k * n2 + e];
        Gbs[idx] = (T)(-Gt[(M - k) * n2 + e]);
    }
}

// Operand copy of G(tau) for the third transform: Gp[t][l][col], l < 16*KT,
// col < SL, zero outside l, k < n.  Column col holds k = col below perm_from;
// from there on, within each 16-block, col = 4a + b holds k = a + 4b: the
// order in which the FP64 MFMA result tile hands out its rows (perm_from = 0),
// and the order the FP32 form gives the rows of its last k tile (see k_s23).
template <class T>
__global__ void k_stage_gp(int n, int kt_tiles, int sl, int perm_from, int M, int k0, int nb,
                           const double *__restrict__ Gt, T *__restrict__ Gp) {
    const int p16 = 16 * kt_tiles;
    const size_t per = (size_t)p16 * sl;
    const size_t n2 = (size_t)n * n;
    const size_t total = per * nb;
    for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < total;
         idx += (size_t)gridDim.x * blockDim.x) {
        const size_t t = idx / per;
        const int rem = (int)(idx % per);
        const int l = rem / sl, col = rem % sl;
        const int k = col < perm_from ? col : (col & ~15) + ((col & 15) >> 2) + 4 * (col & 3);
        double val = 0.0;
        if (col < p16 && l < n && k < n) val = Gt[(size_t)(k0 + t) * n2 + (size_t)l * n + k];
        Gp[idx] = (T)val;
    }
}

// ---------------------------------------------------------------------------
// Fused second and third transforms.
//
// For one tau point t and one (i, n) pair the first transform left the
// N x N slab T1[q][k] (= sum_m v_imqk G_mn).  Per slab
//     X[p][l] = sum_{q,k} Gb[q][p] T1[q][k] G[k][l],
// computed as Y^T = T1^T Gb (contract q) and X^T = G^T Y^T (contract k).
// A wave owns one 16-wide p tile of one slab: Y^T[:, p tile] stays in MFMA
// accumulators and is fed back unchanged as the B operand of the second
// product.  That works because an MFMA result tile holds, per lane, the rows
// of one K group of the next product's B operand (rows 4a..4a+3 for FP32,
// a, a+4, a+8, a+12 for FP64, a = lane/16); the A operand (G) is read in the
// matching row order.  In its last k tile the FP32 form loads the first
// product's A rows in the order m = 4a + b <-> k = a + 4b, so that there, as
// in every FP64 tile, the e-th result register carries k = 4e + a: the second
// product's e-th MFMA of the last tile contracts k = 16 (KT - 1) + 4e ..
// + 4e + 3 and is skipped when all of them are >= N (N % 16 in 1..12).  Workgroup = (t, n, p tile); its waves take the slabs
// i = w, w + nw, ...; G(tau) sits in LDS (or is read from the staged copy
// when it does not fit), the p-tile columns of G(-tau) too.
//
// Layouts: T1[i][t][n][q][k] (one contiguous slab per (i, t, n));
//          X[n][p][r][l] with r = t*N + i (the final contraction reads,
//          for each (n, p), a contiguous block of rows).
struct S23Args {
    const void *T1;
    const void *Gp;   // [nb][16*KT][SL]
    const void *Gb;   // [nb][n][n]
    void *X;
    int n, nb;
};

template <int MODE> struct S23Geom {
    static constexpr int pad = (MODE == MODE_F64) ? 2 : 4;   // conflict-free 16-B row reads
};

// Workgroup size bound: the grouped FP32 form keeps 100-200 registers live
// (at most 8 waves); the FP64 form fits in 128 registers up to 7 tiles and
// then runs 16 waves per workgroup, which is what one workgroup per CU
// (G(tau) in LDS takes ~100 KB) needs to fill the SIMDs.
template <int MODE, int KT> struct S23Threads {
    static constexpr int value = (MODE == MODE_F64 && KT <= 7) ? 1024 : 512;
};

// p tiles per workgroup: the FP32 form up to KT = 7 takes two adjacent p tiles
// per wave (each T1 operand load and each G(tau) read from LDS then feeds two
// MFMAs; 206 registers at KT = 7).  Above KT = 7 the doubled G(-tau) columns
// would leave one workgroup per CU, and the FP64 form has 128 registers.
template <int MODE, int KT> struct S23Pt {
    static constexpr int value = (MODE == MODE_F32 && KT <= 7) ? 2 : 1;
};
static int s23_pt(int mode, int kt) { return (mode == MODE_F32 && kt <= 7) ? 2 : 1; }
// workgroups per (tau, n): one per group of S23Pt p tiles
static int s23_groups(int mode, int kt) { return (kt + s23_pt(mode, kt) - 1) / s23_pt(mode, kt); }

template <int MODE, int KT, bool GLDS>
__global__ __launch_bounds__((S23Threads<MODE, KT>::value)) void k_s23(KRef<S23Args> ref) {
    using T = typename ModeT<MODE>::in_t;
    using acc_t = typename ModeT<MODE>::acc_t;
    constexpr int P16 = 16 * KT;
    constexpr int SL = P16 + S23Geom<MODE>::pad;
    constexpr int PT = S23Pt<MODE, KT>::value;
    constexpr int KTP = (KT + PT - 1) / PT;
    extern __shared__ __attribute__((aligned(16))) unsigned char s23_smem[];

    S23Args a;
    int L;
    if (!kresolve(ref, ref.one.nb * ref.one.n * KTP, a, L)) return;
    const int N = a.n;
    const int pt = (L % KTP) * PT;                 // first p tile of the workgroup
    const int nn = (L / KTP) % N;
    const int t = L / (KTP * N);
    const int S = (N + 3) >> 2;                    // q steps of 4
    const bool two = PT == 2 && pt + 1 < KT;       // wave-uniform

    T *Gl = reinterpret_cast<T *>(s23_smem);
    T *Bl = Gl + (GLDS ? P16 * SL : 0);            // [4S][16 PT]: G(-tau)[q][16 pt + c]
    const T *Gsrc = static_cast<const T *>(a.Gp) + (size_t)t * P16 * SL;
    const T *Gb = static_cast<const T *>(a.Gb) + (size_t)t * N * N;
    const int tid = threadIdx.x, nth = blockDim.x;
    if constexpr (GLDS) {
        const int n16 = P16 * SL * (int)sizeof(T) / 16;
        const float4 *src = reinterpret_cast<const float4 *>(Gsrc);
        float4 *dst = reinterpret_cast<float4 *>(Gl);
        for (int e = tid; e < n16; e += nth) dst[e] = src[e];
    }
    // q order of the first product: with GW = 16 B / element (4 FP32, 2 FP64)
    // and N % GW == 0 the first U = N / (4 GW) groups of 4 GW q are taken as
    // step GW u + j <-> q = 4 GW u + GW a + j (a = lane/16), so that a lane
    // reads GW consecutive q of one slab row with one 16-B load; the
    // remaining q (and every q when N % GW != 0) as step s <-> q = 4s + a.
    // Bl[step][a][c] = G(-tau)[q(step, a)][16 pt + c], c < 16 PT.
    constexpr int GW = 16 / (int)sizeof(T);      // q per 16-B load: 4 (FP32), 2 (FP64)
    // (FP64 keeps one q per load: its grouped form needs too many registers)
    const bool vq = (MODE != MODE_F64) && (N % GW == 0);
    const int U = vq ? N / (4 * GW) : 0;
    for (int e = tid; e < 4 * S * 16 * PT; e += nth) {
        const int st = e / (64 * PT), ga = (e / (16 * PT)) & 3, p = 16 * pt + e % (16 * PT);
        const int q = (st < GW * U) ? 4 * GW * (st / GW) + GW * ga + (st % GW) : 4 * st + ga;
        Bl[e] = (q < N && p < N) ? Gb[(size_t)q * N + p] : T(0);
    }
    __syncthreads();

    const T *Gop = GLDS ? Gl : Gsrc;
    const int lane = tid & 63, g = lane >> 4, c = lane & 15;
    const int nw = nth >> 6;
    const size_t N2 = (size_t)N * N;
    const size_t R = (size_t)a.nb * N;
    const GF2_GLOBAL T *T1 = (const GF2_GLOBAL T *)a.T1;
    GF2_GLOBAL T *X = (GF2_GLOBAL T *)a.X;
    const int p = 16 * pt + c;
    const bool vec4 = (MODE != MODE_F64) && (N % 4 == 0);

    // Operand loads use clamped addresses instead of masks: a row q >= N meets
    // a zero row of Gb, a column k >= N gives a row of Y^T that meets a zero
    // row of G in the second product, so the (finite) values read there add
    // exact zeros.  This keeps the loads free of value selects, which would
    // force a wait right after they are issued.
    //
    // The slab is symmetric (v_imqk = v_imkq), so T1[q][k] is read as
    // T1[k][q]: in the grouped q order a lane's 4 consecutive q of row k are
    // one 16-B load.
    // first-product A row c of the last k tile holds k = 16 (KT - 1) + kperm
    // (see above; the FP32 form keeps k = 16 kt + c in the other tiles)
    const int kperm = (MODE == MODE_F64) ? c : 4 * (c & 3) + (c >> 2);
    const int kc_last = min(16 * (KT - 1) + kperm, N - 1);
    // MFMAs of the second product's last k tile that meet some k < N
    const int elast = __builtin_amdgcn_readfirstlane((N - 16 * (KT - 1) + 3) >> 2);
    auto slab_of = [&](int i) { return T1 + (((size_t)i * a.nb + t) * N + nn) * N2; };
    typedef T qv_t __attribute__((ext_vector_type(GW)));
    qv_t ga_[KT], gb_[KT];                      // grouped operands (GW steps each), double-buffered
    T ta[KT];                                   // one step of the remaining q
    auto loadg = [&](qv_t(&r)[KT], const GF2_GLOBAL T *slab, int u) {
        const GF2_GLOBAL T *col = slab + 4 * GW * u + GW * g;
#pragma unroll
        for (int kt = 0; kt < KT; ++kt) {
            const int k = (kt < KT - 1) ? 16 * kt + c : kc_last;
            r[kt] = *(const GF2_GLOBAL qv_t *)(col + (size_t)k * N);
        }
    };
    auto load1 = [&](T(&r)[KT], const GF2_GLOBAL T *slab, int st) {
        const GF2_GLOBAL T *row = slab + (size_t)min(4 * st + g, N - 1) * N;
#pragma unroll
        for (int kt = 0; kt < KT - 1; ++kt) r[kt] = row[16 * kt + c];
        r[KT - 1] = row[kc_last];
    };

    int i = tid >> 6;
    if (i < N) {
        if (U > 0) loadg(ga_, slab_of(i), 0);
        else load1(ta, slab_of(i), 0);
    }
    for (; i < N; i += nw) {
        const GF2_GLOBAL T *slab = slab_of(i);
        acc_t acc1[KT], acc1b[PT == 2 ? KT : 1];   // p tiles pt, pt + 1
#pragma unroll
        for (int kt = 0; kt < KT; ++kt) acc1[kt] = acc_t{0, 0, 0, 0};
#pragma unroll
        for (int kt = 0; kt < (PT == 2 ? KT : 1); ++kt) acc1b[kt] = acc_t{0, 0, 0, 0};

        // ---- Y^T[k][p] = sum_q T1[q][k] Gb[q][p]
        auto mma = [&](acc_t &ac, T av, T bv) {
            if constexpr (MODE == MODE_F64)
                ac = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, ac, 0, 0, 0);
            else
                ac = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, ac, 0, 0, 0);
        };
        const int bl_off = 16 * PT * g + c;
        auto step = [&](auto av_of, int st) {
            const T bv = Bl[st * 64 * PT + bl_off];
#pragma unroll
            for (int kt = 0; kt < KT; ++kt) mma(acc1[kt], av_of(kt), bv);
            if constexpr (PT == 2) {
                if (two) {
                    const T bw = Bl[st * 64 * PT + bl_off + 16];
#pragma unroll
                    for (int kt = 0; kt < KT; ++kt) mma(acc1b[kt], av_of(kt), bw);
                }
            }
        };
        auto stepg = [&](const qv_t(&r)[KT], int u) {
#pragma unroll
            for (int j = 0; j < GW; ++j) step([&](int kt) { return r[kt][j]; }, GW * u + j);
        };
        auto step1 = [&](const T(&r)[KT], int st) {
            step([&](int kt) { return r[kt]; }, st);
        };
        if (U > 0) {
            // the first ungrouped step is loaded now; it is used last
            if (GW * U < S) load1(ta, slab, GW * U);
            int u = 0;
            for (; u + 1 < U; u += 2) {
                loadg(gb_, slab, u + 1);
                stepg(ga_, u);
                if (u + 2 < U) loadg(ga_, slab, u + 2);
                stepg(gb_, u + 1);
            }
            if (u < U) stepg(ga_, u);
        }
        // remaining steps: the first was loaded ahead, later ones (N % 16 >= 8
        // or N % 4 != 0) are loaded just before use
        for (int st = GW * U; st < S; ++st) {
            if (st > GW * U) load1(ta, slab, st);
            step1(ta, st);
        }
        // first operands of the next slab, in flight during the second product
        if (i + nw < N) {
            if (U > 0) loadg(ga_, slab_of(i + nw), 0);
            else load1(ta, slab_of(i + nw), 0);
        }

        // ---- X^T[l][p] = sum_k G[k][l] Y^T[k][p], one 16-row l tile at a time
        GF2_GLOBAL T *xbase = X + ((size_t)(nn * N + p) * R + (size_t)t * N + i) * N;
        auto store = [&](GF2_GLOBAL T *xb, const acc_t &v, int lt) {
            if constexpr (MODE == MODE_F64) {
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int l = 16 * lt + g + 4 * e;
                    if (l < N) xb[l] = v[e];
                }
            } else {
                const int l0 = 16 * lt + 4 * g;
                if (vec4 && l0 < N) {
                    *(GF2_GLOBAL v4f *)(xb + l0) = v4f{v[0], v[1], v[2], v[3]};
                } else if (!vec4) {
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        if (l0 + e < N) xb[l0 + e] = v[e];
                }
            }
        };
        // the e-th MFMA of k tile kt contracts k = 16 kt + 4e + a; the last tile
        // goes first and runs only its MFMAs with e < elast
        auto gop = [&](const T *grow, int kt, T (&gv)[4]) {
            if constexpr (MODE == MODE_F64) {
                const double2 g0 = *reinterpret_cast<const double2 *>(grow + 16 * kt);
                const double2 g1 = *reinterpret_cast<const double2 *>(grow + 16 * kt + 2);
                gv[0] = g0.x; gv[1] = g0.y; gv[2] = g1.x; gv[3] = g1.y;
            } else {
                const float4 g4 = *reinterpret_cast<const float4 *>(grow + 16 * kt);
                gv[0] = g4.x; gv[1] = g4.y; gv[2] = g4.z; gv[3] = g4.w;
            }
        };
#pragma unroll 1
        for (int lt = 0; lt < KT; ++lt) {
            const T *grow = Gop + (16 * lt + c) * SL + 4 * g;
            if constexpr (PT == 2) {
                // per p tile two chains (even / odd k tiles, added at the end,
                // as in the one-tile form); the G(tau) operand is shared
                acc_t acc2 = acc_t{0, 0, 0, 0}, acc2b = acc_t{0, 0, 0, 0};
                acc_t acc3 = acc_t{0, 0, 0, 0}, acc3b = acc_t{0, 0, 0, 0};
                auto ktile = [&](int kt, bool last) {
                    T gv[4];
                    gop(grow, kt, gv);
                    acc_t &a0 = (kt & 1) ? acc2b : acc2;
                    acc_t &a1 = (kt & 1) ? acc3b : acc3;
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        if (e > 0 && last && elast <= e) break;
                        mma(a0, gv[e], acc1[kt][e]);
                        if (two) mma(a1, gv[e], acc1b[kt][e]);
                    }
                };
                ktile(KT - 1, true);
#pragma unroll
                for (int kt = 0; kt < KT - 1; ++kt) ktile(kt, false);
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    acc2[e] += acc2b[e];
                    acc3[e] += acc3b[e];
                }
                if (p < N) store(xbase, acc2, lt);
                if (two && p + 16 < N) store(xbase + (size_t)16 * R * N, acc3, lt);
            } else {
                // two accumulation chains (even / odd k tiles), added at the end
                acc_t acc2 = acc_t{0, 0, 0, 0}, acc2b = acc_t{0, 0, 0, 0};
                auto ktile = [&](acc_t &ac, int kt, bool last) {
                    T gv[4];
                    gop(grow, kt, gv);
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        if (e > 0 && last && elast <= e) break;
                        mma(ac, gv[e], acc1[kt][e]);
                    }
                };
                ktile(((KT - 1) & 1) ? acc2b : acc2, KT - 1, true);
#pragma unroll
                for (int kt = 0; kt < KT - 1; ++kt) ktile((kt & 1) ? acc2b : acc2, kt, false);
#pragma unroll
                for (int e = 0; e < 4; ++e) acc2[e] += acc2b[e];
                if (p < N) store(xbase, acc2, lt);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Final contraction: part[z][r][j] = - sum_{k in slice z} X(k, r) W2[k][j],
// k = (n, p, l) flattened, X(k, r) = X[k / N][r][k % N] (layout above), so
// for each (n, p) a block's rows are one contiguous piece of memory.
// Split-K over slices of kz; FP32 accumulators are flushed into FP64 every
// 512 K.  Workgroup = (row block, slice), XCD-ordered so that the row
// blocks of one slice (which share the W2 slice) run on one XCD.
struct S4Args {
    const void *X;
    const void *W;
    double *part;
    long long K, kz;
    int n, R, nrb, nsplit;
    int vec;            // n divisible by the vector width
    int ncb;            // column blocks of 16 * NT columns per row block (1 or 2)
};

// The final contraction orders its rows i-major: row r = i nb + t is X row
// t n + i.  First 16-column tile (columns col0 + 16 cc) that a workgroup
// needs: its smallest i is r0 / nb, and the reduction reads only the entries
// j >= i, so tiles wholly below that i are skipped.  Workgroup-uniform.
__device__ __forceinline__ int s4_first_tile(int r0, int nb, int col0) {
    return max(0, (r0 / nb - col0) >> 4);
}
#define GF2_FIRST_TILE_SWITCH(first, run)                                                   \
    switch (first) {                                                                        \
        case 0: run(std::integral_constant<int, 0>{}); break;                               \
        case 1: run(std::integral_constant<int, 1>{}); break;                               \
        case 2: run(std::integral_constant<int, 2>{}); break;                               \
        case 3: run(std::integral_constant<int, 3>{}); break;                               \
        case 4: run(std::integral_constant<int, 4>{}); break;                               \
        case 5: run(std::integral_constant<int, 5>{}); break;                               \
        case 6: run(std::integral_constant<int, 6>{}); break;                               \
        case 7: run(std::integral_constant<int, 7>{}); break;                               \
        case 8: run(std::integral_constant<int, 8>{}); break;                               \
        default: run(std::integral_constant<int, 9>{}); break;                              \
    }

constexpr int S4_WAVES = 8;               // one 16-row tile per wave
constexpr int S4_THREADS = 64 * S4_WAVES;
constexpr int S4_BM = 16 * S4_WAVES;

template <int MODE, int NT>
__global__ __launch_bounds__(S4_THREADS) void k_s4(KRef<S4Args> ref) {
    using T = typename ModeT<MODE>::in_t;
    using acc_t = typename ModeT<MODE>::acc_t;
    constexpr bool F64 = (MODE == MODE_F64);
    constexpr int VEC = 16 / (int)sizeof(T);          // elements per 16-B load
    constexpr int BK = 8 * VEC;                       // 32 (FP32) / 16 (FP64)
    constexpr int BMR = S4_BM;                        // rows per block
    constexpr int BN = 16 * NT;
    constexpr int SK = BK + (F64 ? 2 : 4);
    constexpr int SB = BN + ((16 - BN % 32) + 32) % 32;
    constexpr int A_IT = BMR * 8 / S4_THREADS;        // 16-B A loads per thread
    constexpr int BC = BN / VEC;                      // vector loads per B row
    constexpr int B_IT = (BK * BC + S4_THREADS - 1) / S4_THREADS;
    constexpr int AROWS = S4_THREADS / 8;             // rows covered per A load round
    constexpr int FLUSH = 512 / BK;
    typedef T vec_t __attribute__((ext_vector_type(VEC)));

    __shared__ __attribute__((aligned(16))) T As[BMR][SK];
    __shared__ __attribute__((aligned(16))) T Bs[BK][SB];

    S4Args a;
    int L;
    if (!kresolve(ref, ref.one.nrb * ref.one.nsplit * ref.one.ncb, a, L)) return;
    // rows fastest, then column blocks, then slices: the blocks of one W2 slice are adjacent
    const int rb = L % a.nrb, cbk = (L / a.nrb) % a.ncb, z = L / (a.nrb * a.ncb);
    const int col0 = cbk * BN;
    const int N = a.n;
    const long long k0 = (long long)z * a.kz;
    const long long kend = std::min<long long>(a.K, k0 + a.kz);
    const int r0 = rb * BMR;
    const GF2_GLOBAL T *X = (const GF2_GLOBAL T *)a.X;
    const GF2_GLOBAL T *W = (const GF2_GLOBAL T *)a.W;
    const size_t RN = (size_t)a.R * N;

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int kq = tid & 7, arow = tid >> 3;

    acc_t acc[NT];
    double accd[NT][4];
#pragma unroll
    for (int cc = 0; cc < NT; ++cc) {
        acc[cc] = acc_t{0, 0, 0, 0};
#pragma unroll
        for (int e = 0; e < 4; ++e) accd[cc][e] = 0.0;
    }

    const float inv_n = 1.0f / (float)N;
    // X row of each staged logical row (i-major r = i nb + t -> X row t n + i)
    const int nbt = a.R / N;
    int xrow[A_IT];
#pragma unroll
    for (int j = 0; j < A_IT; ++j) {
        const int r = min(r0 + arow + AROWS * j, a.R - 1);
        xrow[j] = (r % nbt) * N + r / nbt;
    }
    vec_t ra[A_IT], rbv[B_IT];
    auto load_chunk = [&](long long kb) {
        const long long k = kb + VEC * kq;
        const unsigned np = udiv22((unsigned)k, (unsigned)N, inv_n);
        const int l = (int)(k - (long long)np * N);
#pragma unroll
        for (int j = 0; j < A_IT; ++j) {
            const int r = r0 + arow + AROWS * j;
            const int rp = xrow[j];
            vec_t v;
            if (a.vec) {
                if (k < kend && r < a.R) {
                    v = *(const GF2_GLOBAL vec_t *)(X + (size_t)np * RN + (size_t)rp * N + l);
                } else {
#pragma unroll
                    for (int e = 0; e < VEC; ++e) v[e] = T(0);
                }
            } else {
#pragma unroll
                for (int e = 0; e < VEC; ++e) {
                    const long long ke = k + e;
                    T x = T(0);
                    if (ke < kend && r < a.R) {
                        const unsigned npe = udiv22((unsigned)ke, (unsigned)N, inv_n);
                        const int le = (int)(ke - (long long)npe * N);
                        x = X[(size_t)npe * RN + (size_t)rp * N + le];
                    }
                    v[e] = x;
                }
            }
            ra[j] = v;
        }
        // B chunk: rows kb .. kb + BK - 1 of W2, columns col0 .. col0 + BN - 1
#pragma unroll
        for (int j = 0; j < B_IT; ++j) {
            const int u = tid + j * S4_THREADS;
            const int kr = u / BC, c = (u % BC) * VEC;
            const long long gk = kb + kr;
            const int gc = col0 + c;
            const bool ok = u < BK * BC && gk < kend;
            vec_t v;
            if (a.vec) {
                // Clamped addresses, no value select (a select would wait for the load
                // here): rows past the slice meet zero A columns, columns past N only
                // reach outputs j >= N, and both read finite W2 values.
                const long long gkc = gk < a.K ? gk : a.K - 1;
                const int gcc = gc < N ? gc : N - VEC;
                v = *(const GF2_GLOBAL vec_t *)(W + (size_t)gkc * N + gcc);
            } else {
                const GF2_GLOBAL T *src = W + (size_t)gk * N + gc;
#pragma unroll
                for (int e = 0; e < VEC; ++e) v[e] = (ok && gc + e < N) ? src[e] : T(0);
            }
            rbv[j] = v;
        }
    };
    auto store_chunk = [&]() {
#pragma unroll
        for (int j = 0; j < A_IT; ++j)
            *reinterpret_cast<vec_t *>(&As[arow + AROWS * j][VEC * kq]) = ra[j];
#pragma unroll
        for (int j = 0; j < B_IT; ++j) {
            const int u = tid + j * S4_THREADS;
            if (u < BK * BC) *reinterpret_cast<vec_t *>(&Bs[u / BC][(u % BC) * VEC]) = rbv[j];
        }
    };

    const int nchunks = (int)((kend - k0 + BK - 1) / BK);
    const int first = s4_first_tile(r0, a.R / N, col0);
    if (first >= NT) return;   // workgroup-uniform: every entry here has j < i
    auto run = [&](auto cf) {
        constexpr int CF = decltype(cf)::value < NT ? decltype(cf)::value : NT;
        load_chunk(k0);
        for (int ch = 0; ch < nchunks; ++ch) {
            __syncthreads();
            store_chunk();
            __syncthreads();
            if (ch + 1 < nchunks) load_chunk(k0 + (long long)(ch + 1) * BK);
#pragma unroll
            for (int s4 = 0; s4 < BK; s4 += 4) {
                const int kr = s4 + (lane >> 4);
                const T af = As[wave * 16 + (lane & 15)][kr];
#pragma unroll
                for (int cc = CF; cc < NT; ++cc) {
                    const T bf = Bs[kr][cc * 16 + (lane & 15)];
                    if constexpr (F64)
                        acc[cc] = __builtin_amdgcn_mfma_f64_16x16x4f64(af, bf, acc[cc], 0, 0, 0);
                    else
                        acc[cc] = __builtin_amdgcn_mfma_f32_16x16x4f32(af, bf, acc[cc], 0, 0, 0);
                }
            }
            if constexpr (!F64) {
                if ((ch + 1) % FLUSH == 0 || ch + 1 == nchunks) {
#pragma unroll
                    for (int cc = CF; cc < NT; ++cc) {
#pragma unroll
                        for (int e = 0; e < 4; ++e) accd[cc][e] += (double)acc[cc][e];
                        acc[cc] = acc_t{0, 0, 0, 0};
                    }
                }
            }
        }
    };
    GF2_FIRST_TILE_SWITCH(first, run)

    GF2_GLOBAL double *out = (GF2_GLOBAL double *)a.part + (size_t)z * RN;
#pragma unroll
    for (int cc = 0; cc < NT; ++cc)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int row = F64 ? ((lane >> 4) + 4 * e) : (4 * (lane >> 4) + e);
            const int m = r0 + wave * 16 + row;
            const int j = col0 + cc * 16 + (lane & 15);
            if (m < a.R && j < N) {
                double val;
                if constexpr (F64) val = acc[cc][e];
                else val = accd[cc][e];
                out[(size_t)m * N + j] = -val;
            }
        }
}


// Sigma[k0 + t][i][j] = sum_z part[z][t*n + i][j]   (part already carries the minus sign)
// The partial sums hold row i nb + t for (tau_t, i) (the final contraction's
// i-major row order) and only the entries j >= i: Sigma_ij = Sigma_ji (symmetric G and integrals), so
// (i, j) with j < i is the computed (j, i).
__global__ void k_reduce_split(int n, int nb, int nsplit, const double *__restrict__ part,
                               double *__restrict__ Sig, int k0) {
    const size_t n2 = (size_t)n * n;
    const size_t total = n2 * nb;
    for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < total;
         idx += (size_t)gridDim.x * blockDim.x) {
        const size_t t = idx / n2, e = idx % n2;
        const int i = (int)(e / n), j = (int)(e % n);
        const size_t src = ((size_t)min(i, j) * nb + t) * n + max(i, j);
        double s = 0.0;
        for (int z = 0; z < nsplit; ++z) s += part[z * total + src];
        Sig[(size_t)k0 * n2 + idx] = s;
    }
}

// ---------------------------------------------------------------------------
// Split-BF16 forms (BF16x3: NP = 2 planes, BF16x6: NP = 3) of S23 and S4.
//
// Operands are pre-split into NP bf16 planes where they are produced or
// staged, so the kernels issue loads and MFMAs only:
//   T1  planes [i][t][n][q][k] with rows padded to LQ = roundup(n, 8)
//       (written by the first transform; padding is zero);
//   Gq  planes of G(tau) [t][l][col] for the third transform, col in the K
//       order of a 32-deep MFMA fed by two FP32 result tiles (below);
//   W2b planes of W2 [k / 64][j][64] with k in the K order of the A operand
//       of the final contraction (below), built once per system with three
//       planes (the two-term forms read the first two).
// v_mfma_f32_16x16x32_bf16: lane (a = lane/16, c = lane%16) holds A[c][8a..8a+7]
// and B[8a..8a+7][c]; the result tile is laid out like the FP32 MFMA's.
typedef __bf16 v8bf_t __attribute__((ext_vector_type(8)));

__device__ __forceinline__ v8bf_t as_bf8(v8us x) { return __builtin_bit_cast(v8bf_t, x); }


template <int NP>
__device__ __forceinline__ v4f mma3(const v8us (&a)[NP], const v8us (&b)[NP], v4f acc) {
    // same products and order as mma_split
    if constexpr (NP == 3) {
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf8(a[1]), as_bf8(b[1]), acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf8(a[0]), as_bf8(b[2]), acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf8(a[2]), as_bf8(b[0]), acc, 0, 0, 0);
    }
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf8(a[0]), as_bf8(b[1]), acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf8(a[1]), as_bf8(b[0]), acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf8(a[0]), as_bf8(b[0]), acc, 0, 0, 0);
    return acc;
}

// K order of a 32-deep product whose B operand is two FP32 16x16 result
// tiles (rows 0-15 of tile 0, rows 0-15 of tile 1): slot 8a + j holds row
// 4a + j of tile 0 for j < 4 and row 4a + j - 4 of tile 1 for j >= 4.
__device__ __forceinline__ int pair_row(int slot) {
    const int a = slot >> 3, j = slot & 7;
    return (j < 4) ? 4 * a + j : 16 + 4 * a + (j - 4);
}

// Gq[t][l][col], col < 32 * KP: G(tau_{k0+t})[l][k], k = 32 (col / 32) + pair_row(col % 32);
// np planes (2 or 3)
__global__ void k_stage_gq(int n, int KP, int sl, int p16, int k0, int nb, size_t plane, int np,
                           const double *__restrict__ Gt, unsigned short *__restrict__ Gq) {
    const size_t per = (size_t)p16 * sl;
    const size_t n2 = (size_t)n * n;
    const size_t total = per * nb;
    for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < total;
         idx += (size_t)gridDim.x * blockDim.x) {
        const size_t t = idx / per;
        const int rem = (int)(idx % per);
        const int l = rem / sl, col = rem % sl;
        const int k = 32 * (col >> 5) + pair_row(col & 31);
        float x = 0.0f;
        if (col < 32 * KP && l < n && k < n) x = (float)Gt[(size_t)(k0 + t) * n2 + (size_t)l * n + k];
        unsigned short o[3];
        split_bf16n<3>(x, o);
        Gq[idx] = o[0];
        Gq[idx + plane] = o[1];
        if (np == 3) Gq[idx + 2 * plane] = o[2];
    }
}

struct S23b3Args {
    const unsigned short *T1;   // plane 0; plane i at + i * t1_plane (FP32 T1: the FP32 array)
    long long t1_plane;
    int lq;                     // slab row (padded for planes; n for an FP32 T1)
    const unsigned short *Gq;   // plane 0; plane i at + i * gq_plane
    long long gq_plane;
    const float *Gb;            // G(-tau) [nb][n][n] FP32
    float *X;                   // [n][n][R][n] FP32
    int n, nb;
};

// p tiles per wave of the split S23 kernel: two for KT <= 7 (the T1 operands
// of the first product and the G(tau) operands of the second are loaded once
// for both tiles), one above (registers).  Each tile's products and their
// order do not depend on this.
template <int KT> struct S23bPt { static constexpr int value = (KT >= 2 && KT <= 7) ? 2 : 1; };
static int s23b_pt(int kt) { return (kt >= 2 && kt <= 7) ? 2 : 1; }
// workgroups per (tau, n)
static int s23b_groups(int kt) { return (kt + s23b_pt(kt) - 1) / s23b_pt(kt); }

// F32IN: T1 is FP32 (written by the FP32 first transform) and is split into
// NP planes in registers as each step's operands are used.
template <int KT, int NP, bool F32IN>
__global__ __launch_bounds__(512) void k_s23_bf3(KRef<S23b3Args> ref) {
    constexpr int KP = (KT + 1) / 2;          // 32-deep k steps of the second product
    constexpr int P16 = 16 * KT;
    constexpr int SLG = 32 * KP + 8;          // LDS row of Gq (bf16)
    constexpr int PT = S23bPt<KT>::value;
    constexpr int GR = (KT + PT - 1) / PT;    // workgroups per (t, nn)
    extern __shared__ __attribute__((aligned(16))) unsigned char s23b_smem[];

    S23b3Args a;
    int L;
    if (!kresolve(ref, ref.one.nb * ref.one.n * GR, a, L)) return;
    const int N = a.n;
    const int pt = (L % GR) * PT;             // first p tile of the workgroup
    const int nn = (L / GR) % N;
    const int t = L / (GR * N);
    const bool two = PT == 2 && pt + 1 < KT;  // workgroup-uniform
    const int S32 = (N + 31) >> 5;            // 32-deep q steps of the first product
    const int SQ = 32 * S32 + 8;              // LDS row of the G(-tau) slice (bf16)

    // NP planes of the Gq slice, then NP planes of [16 PT][SQ]:
    // G(-tau)[q][16 pt + cc] at [cc][q]
    unsigned short *GS = reinterpret_cast<unsigned short *>(s23b_smem);
    unsigned short *BS = GS + NP * P16 * SLG;
    const int tid = threadIdx.x, nth = blockDim.x;
    {
        const size_t off = (size_t)t * P16 * SLG;
        const int n16 = P16 * SLG / 8;
#pragma unroll
        for (int pl = 0; pl < NP; ++pl) {
            const float4 *src = reinterpret_cast<const float4 *>(a.Gq + pl * a.gq_plane + off);
            float4 *dst = reinterpret_cast<float4 *>(GS + pl * P16 * SLG);
            for (int e = tid; e < n16; e += nth) dst[e] = src[e];
        }
        const float *Gb = a.Gb + (size_t)t * N * N;
        for (int e = tid; e < 16 * PT * SQ; e += nth) {
            const int cc = e / SQ, q = e - cc * SQ, p = 16 * pt + cc;
            const float x = (q < N && p < N) ? Gb[(size_t)q * N + p] : 0.0f;
            unsigned short o[NP];
            split_bf16n<NP>(x, o);
#pragma unroll
            for (int pl = 0; pl < NP; ++pl) BS[pl * 16 * PT * SQ + e] = o[pl];
        }
    }
    __syncthreads();

    const int lane = tid & 63, g = lane >> 4, c = lane & 15;
    const int nw = nth >> 6;
    const size_t slab_sz = (size_t)N * a.lq;
    const size_t R = (size_t)a.nb * N;
    const int p = 16 * pt + c;
    const bool vec4 = (N % 4 == 0);
    // rows k >= N read row N - 1 (finite; they meet zero rows of G); q
    // blocks past the padded row read q = 0 (they meet zero rows of G(-tau))
    const int kc_last = min(16 * (KT - 1) + c, N - 1);
    const GF2_GLOBAL unsigned short *T1p[NP];
    const unsigned short *GSp[NP];
    const unsigned short *BSp[NP];
#pragma unroll
    for (int pl = 0; pl < NP; ++pl) {
        T1p[pl] = (const GF2_GLOBAL unsigned short *)a.T1 + pl * a.t1_plane;
        GSp[pl] = GS + pl * P16 * SLG;
        BSp[pl] = BS + pl * 16 * PT * SQ + c * SQ + 8 * g;
    }

    for (int i = tid >> 6; i < N; i += nw) {
        const size_t soff = (((size_t)i * a.nb + t) * N + nn) * slab_sz;
        v4f acc1[2 * KP], acc1b[PT == 2 ? 2 * KP : 1];   // p tiles pt, pt + 1
#pragma unroll
        for (int kt = 0; kt < 2 * KP; ++kt) acc1[kt] = v4f{0, 0, 0, 0};
#pragma unroll
        for (int kt = 0; kt < (PT == 2 ? 2 * KP : 1); ++kt) acc1b[kt] = v4f{0, 0, 0, 0};

        // ---- Y^T[k][p] = sum_q T1[k][q] Gb[q][p]  (slab symmetric)
        if constexpr (F32IN) {
            // FP32 slab rows of n: 8 q of row k as two 4-wide pieces; a piece
            // at or past q = n reads q = 0.. of the same row instead (finite;
            // it meets zero rows of G(-tau)), so no load leaves the slab.
            const GF2_GLOBAL float *T1f = (const GF2_GLOBAL float *)a.T1;
            float raw[KT][8];
            auto loadf = [&](int s) {
                const int q0 = 32 * s + 8 * g;
#pragma unroll
                for (int kt = 0; kt < KT; ++kt) {
                    const int k = (kt < KT - 1) ? 16 * kt + c : kc_last;
                    const GF2_GLOBAL float *row = T1f + soff + (size_t)k * N;
                    if (vec4) {
                        const v4f lo = *(const GF2_GLOBAL v4f *)(row + (q0 < N ? q0 : 0));
                        const v4f hi = *(const GF2_GLOBAL v4f *)(row + (q0 + 4 < N ? q0 + 4 : 0));
#pragma unroll
                        for (int e = 0; e < 4; ++e) {
                            raw[kt][e] = lo[e];
                            raw[kt][4 + e] = hi[e];
                        }
                    } else {
#pragma unroll
                        for (int e = 0; e < 8; ++e) raw[kt][e] = row[q0 + e < N ? q0 + e : 0];
                    }
                }
            };
            loadf(0);
            for (int s = 0; s < S32; ++s) {
                v8us bv[NP], bw[NP];
#pragma unroll
                for (int pl = 0; pl < NP; ++pl) {
                    bv[pl] = *reinterpret_cast<const v8us *>(BSp[pl] + 32 * s);
                    if constexpr (PT == 2) bw[pl] = *reinterpret_cast<const v8us *>(BSp[pl] + 16 * SQ + 32 * s);
                }
                const int q1 = 32 * (s + 1) + 8 * g;
#pragma unroll
                for (int kt = 0; kt < KT; ++kt) {
                    v8us av[NP];
                    split8<NP>(raw[kt], av);
                    acc1[kt] = mma3<NP>(av, bv, acc1[kt]);
                    if constexpr (PT == 2)
                        if (two) acc1b[kt] = mma3<NP>(av, bw, acc1b[kt]);
                    if (s + 1 < S32) {
                        // next step's operands of this k tile, in flight during the step
                        const int k = (kt < KT - 1) ? 16 * kt + c : kc_last;
                        const GF2_GLOBAL float *row = T1f + soff + (size_t)k * N;
                        if (vec4) {
                            const v4f lo = *(const GF2_GLOBAL v4f *)(row + (q1 < N ? q1 : 0));
                            const v4f hi = *(const GF2_GLOBAL v4f *)(row + (q1 + 4 < N ? q1 + 4 : 0));
#pragma unroll
                            for (int e = 0; e < 4; ++e) {
                                raw[kt][e] = lo[e];
                                raw[kt][4 + e] = hi[e];
                            }
                        } else {
#pragma unroll
                            for (int e = 0; e < 8; ++e) raw[kt][e] = row[q1 + e < N ? q1 + e : 0];
                        }
                    }
                }
            }
        } else {
        v8us av[KT][NP];
        auto load = [&](int s) {
            int q0 = 32 * s + 8 * g;
            if (q0 + 8 > a.lq) q0 = 0;
#pragma unroll
            for (int kt = 0; kt < KT; ++kt) {
                const int k = (kt < KT - 1) ? 16 * kt + c : kc_last;
                const size_t o = soff + (size_t)k * a.lq + q0;
#pragma unroll
                for (int pl = 0; pl < NP; ++pl) av[kt][pl] = *(const GF2_GLOBAL v8us *)(T1p[pl] + o);
            }
        };
        load(0);
        for (int s = 0; s < S32; ++s) {
            v8us bv[NP], bw[NP];
#pragma unroll
            for (int pl = 0; pl < NP; ++pl) {
                bv[pl] = *reinterpret_cast<const v8us *>(BSp[pl] + 32 * s);
                if constexpr (PT == 2) bw[pl] = *reinterpret_cast<const v8us *>(BSp[pl] + 16 * SQ + 32 * s);
            }
            if constexpr (NP == 2 && PT == 1 && KT < 10) {
                // whole next step prefetched into a second register set
                v8us cv[KT][NP];
#pragma unroll
                for (int kt = 0; kt < KT; ++kt)
#pragma unroll
                    for (int pl = 0; pl < NP; ++pl) cv[kt][pl] = av[kt][pl];
                if (s + 1 < S32) load(s + 1);
#pragma unroll
                for (int kt = 0; kt < KT; ++kt) acc1[kt] = mma3<NP>(cv[kt], bv, acc1[kt]);
            } else {
                // no room for a second set: each k tile's next operands are
                // loaded into its registers once its products issue
                int q1 = 32 * (s + 1) + 8 * g;
                if (q1 + 8 > a.lq) q1 = 0;
#pragma unroll
                for (int kt = 0; kt < KT; ++kt) {
                    acc1[kt] = mma3<NP>(av[kt], bv, acc1[kt]);
                    if constexpr (PT == 2)
                        if (two) acc1b[kt] = mma3<NP>(av[kt], bw, acc1b[kt]);
                    if (s + 1 < S32) {
                        const int k = (kt < KT - 1) ? 16 * kt + c : kc_last;
                        const size_t o = soff + (size_t)k * a.lq + q1;
#pragma unroll
                        for (int pl = 0; pl < NP; ++pl) av[kt][pl] = *(const GF2_GLOBAL v8us *)(T1p[pl] + o);
                    }
                }
            }
        }
        }

        // ---- X^T[l][p] = sum_k G[k][l] Y^T[k][p]; B operand = two result tiles
        v8us yv[KP][NP], yw[PT == 2 ? KP : 1][NP];
#pragma unroll
        for (int u = 0; u < KP; ++u) {
            float y[8];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                y[e] = acc1[2 * u][e];
                y[4 + e] = acc1[2 * u + 1][e];
            }
            split8<NP>(y, yv[u]);
            if constexpr (PT == 2) {
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    y[e] = acc1b[2 * u][e];
                    y[4 + e] = acc1b[2 * u + 1][e];
                }
                split8<NP>(y, yw[u]);
            }
        }
        GF2_GLOBAL float *xbase = (GF2_GLOBAL float *)a.X + ((size_t)(nn * N + p) * R + (size_t)t * N + i) * N;
        auto store = [&](GF2_GLOBAL float *xb, const v4f &v, int lt) {
            const int l0 = 16 * lt + 4 * g;
            if (vec4 && l0 < N) {
                *(GF2_GLOBAL v4f *)(xb + l0) = v4f{v[0], v[1], v[2], v[3]};
            } else if (!vec4) {
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    if (l0 + e < N) xb[l0 + e] = v[e];
            }
        };
#pragma unroll 1
        for (int lt = 0; lt < KT; ++lt) {
            v4f acc2 = v4f{0, 0, 0, 0}, acc3 = v4f{0, 0, 0, 0};
            const int row = (16 * lt + c) * SLG + 8 * g;
#pragma unroll
            for (int u = 0; u < KP; ++u) {
                v8us gv[NP];
#pragma unroll
                for (int pl = 0; pl < NP; ++pl) gv[pl] = *reinterpret_cast<const v8us *>(GSp[pl] + row + 32 * u);
                acc2 = mma3<NP>(gv, yv[u], acc2);
                if constexpr (PT == 2)
                    if (two) acc3 = mma3<NP>(gv, yw[u], acc3);
            }
            if (p < N) store(xbase, acc2, lt);
            if (two && p + 16 < N) store(xbase + (size_t)16 * R * N, acc3, lt);
        }
    }
}

// W2b[kc][j][w] (three planes, plane i at + i * plane), w < 64: W2[k][j] with
// k = 64 kc + 32 (w / 32) + pair_row(w % 32); zero for k >= n^3 or j >= n.
__global__ void k_build_w2b(int n, int bn, long long nkc, size_t plane, const double *__restrict__ v,
                            unsigned short *__restrict__ W2b) {
    const size_t n2 = (size_t)n * n, n3 = n2 * n;
    const size_t total = (size_t)nkc * bn * 64;
    for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < total;
         idx += (size_t)gridDim.x * blockDim.x) {
        const size_t kc = idx / ((size_t)bn * 64);
        const int rem = (int)(idx % ((size_t)bn * 64));
        const int j = rem >> 6, w = rem & 63;
        const size_t k = 64 * kc + 32 * (w >> 5) + pair_row(w & 31);
        float x = 0.0f;
        if (k < n3 && j < n) {
            // k = (nn, p, l): W2[nn][p][l][j] = 2 v_l p nn j - v_nn p l j
            const size_t nn = k / n2, pp = (k / n) % n, l = k % n;
            x = (float)(2.0 * v[((l * n + pp) * n + nn) * n + j] - v[((nn * n + pp) * n + l) * n + j]);
        }
        unsigned short o[3];
        split_bf16n<3>(x, o);
        W2b[idx] = o[0];
        W2b[idx + plane] = o[1];
        W2b[idx + 2 * plane] = o[2];
    }
}

// Final contraction in split BF16.  Each wave owns 16 rows and reads its A
// operand (X, FP32) straight from memory, splitting it in registers; the W2b
// chunk (shared by the 8 waves) goes through LDS.  K order within a 32-deep
// step: slot 8a + j <-> k = pair_row(8a + j), i.e. two runs of 4 consecutive k.
struct S4b3Args {
    const float *X;
    const unsigned short *W2b;   // plane i at + i * plane
    long long plane;
    double *part;
    long long K, kz;
    int n, R, nrb, nsplit, vec;
};

template <int NT, int NP>
__global__ __launch_bounds__(S4_THREADS) void k_s4_bf3(KRef<S4b3Args> ref) {
    constexpr int BK = 64;
    constexpr int BN = 16 * NT;
    constexpr int SKB = BK + 8;                       // LDS row (bf16)
    constexpr int FLUSH = 512 / BK;
    constexpr int B16 = BN * BK / 8;                  // 16-B units per plane per chunk
    constexpr int B_IT = (B16 + S4_THREADS - 1) / S4_THREADS;
    __shared__ __attribute__((aligned(16))) unsigned short Bs[NP][BN][SKB];

    S4b3Args a;
    int L;
    if (!kresolve(ref, ref.one.nrb * ref.one.nsplit, a, L)) return;
    const int rb = L % a.nrb, z = L / a.nrb;
    const int N = a.n;
    const long long k0 = (long long)z * a.kz;
    const long long kend = std::min<long long>(a.K, k0 + a.kz);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int g = lane >> 4, c = lane & 15;
    const size_t RN = (size_t)a.R * N;
    const int r = std::min(rb * S4_BM + wave * 16 + c, a.R - 1);
    const int nbt = a.R / N;
    const int xr = (r % nbt) * N + r / nbt;   // X row of the i-major row r = i nb + t

    v4f acc[NT];
    double accd[NT][4];
#pragma unroll
    for (int cc = 0; cc < NT; ++cc) {
        acc[cc] = v4f{0, 0, 0, 0};
#pragma unroll
        for (int e = 0; e < 4; ++e) accd[cc][e] = 0.0;
    }

    // A: per 32-deep step two runs of 4 k (k = kb + 32 h + 4g .. and + 16)
    const float inv_n = 1.0f / (float)N;
    v4f ra[4];
    auto load_a = [&](long long kb) {
#pragma unroll
        for (int h = 0; h < 4; ++h) {
            long long k = kb + 32 * (h >> 1) + 16 * (h & 1) + 4 * g;
            if (k >= a.K) k = 0;                          // meets zero rows of W2b
            if (a.vec) {
                const unsigned np = udiv22((unsigned)k, (unsigned)N, inv_n);
                const int l = (int)(k - (long long)np * N);
                ra[h] = *(const GF2_GLOBAL v4f *)((const GF2_GLOBAL float *)a.X + (size_t)np * RN + (size_t)xr * N + l);
            } else {
                float x[4];
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    long long ke = k + e;
                    if (ke >= a.K) ke = 0;
                    const unsigned np = udiv22((unsigned)ke, (unsigned)N, inv_n);
                    const int l = (int)(ke - (long long)np * N);
                    x[e] = ((const GF2_GLOBAL float *)a.X)[(size_t)np * RN + (size_t)xr * N + l];
                }
                ra[h] = v4f{x[0], x[1], x[2], x[3]};
            }
        }
    };
    v8us rbv[B_IT][NP];
    auto load_b = [&](long long kb) {
        const size_t base = (size_t)(kb / BK) * BN * BK;
#pragma unroll
        for (int j = 0; j < B_IT; ++j) {
            // threads past the chunk reload its last unit (not stored): no
            // conditional writes, which would put the staging arrays in scratch
            const int u = min(tid + j * S4_THREADS, B16 - 1);
#pragma unroll
            for (int pl = 0; pl < NP; ++pl)
                rbv[j][pl] = *(const GF2_GLOBAL v8us *)((const GF2_GLOBAL unsigned short *)a.W2b + pl * a.plane +
                                                        base + (size_t)u * 8);
        }
    };
    auto store_b = [&]() {
#pragma unroll
        for (int j = 0; j < B_IT; ++j) {
            // (clamped threads rewrite the last unit with the value it already has)
            const int u = min(tid + j * S4_THREADS, B16 - 1);
            const int jn = u / (BK / 8), w8 = u % (BK / 8);
#pragma unroll
            for (int pl = 0; pl < NP; ++pl) *reinterpret_cast<v8us *>(&Bs[pl][jn][8 * w8]) = rbv[j][pl];
        }
    };

    const int nchunks = (int)((kend - k0 + BK - 1) / BK);
    const int first = s4_first_tile(rb * S4_BM, a.R / N, 0);
    if (first >= NT) return;   // workgroup-uniform: every entry here has j < i
    auto run = [&](auto cf) {
        constexpr int CF = decltype(cf)::value < NT ? decltype(cf)::value : NT;
        load_a(k0);
        load_b(k0);
        for (int ch = 0; ch < nchunks; ++ch) {
            __syncthreads();
            store_b();
            __syncthreads();
            v4f cur[4];
#pragma unroll
            for (int h = 0; h < 4; ++h) cur[h] = ra[h];
            if (ch + 1 < nchunks) {
                load_a(k0 + (long long)(ch + 1) * BK);
                load_b(k0 + (long long)(ch + 1) * BK);
            }
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                float x[8] = {cur[2 * s][0], cur[2 * s][1], cur[2 * s][2], cur[2 * s][3],
                              cur[2 * s + 1][0], cur[2 * s + 1][1], cur[2 * s + 1][2], cur[2 * s + 1][3]};
                v8us xv[NP];
                split8<NP>(x, xv);
#pragma unroll
                for (int cc = CF; cc < NT; ++cc) {
                    v8us bv[NP];
#pragma unroll
                    for (int pl = 0; pl < NP; ++pl)
                        bv[pl] = *reinterpret_cast<const v8us *>(&Bs[pl][16 * cc + c][32 * s + 8 * g]);
                    acc[cc] = mma3<NP>(xv, bv, acc[cc]);
                }
            }
            if ((ch + 1) % FLUSH == 0 || ch + 1 == nchunks) {
#pragma unroll
                for (int cc = CF; cc < NT; ++cc) {
#pragma unroll
                    for (int e = 0; e < 4; ++e) accd[cc][e] += (double)acc[cc][e];
                    acc[cc] = v4f{0, 0, 0, 0};
                }
            }
        }
    };
    GF2_FIRST_TILE_SWITCH(first, run)

    GF2_GLOBAL double *out = (GF2_GLOBAL double *)a.part + (size_t)z * RN;
#pragma unroll
    for (int cc = 0; cc < NT; ++cc)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int m = rb * S4_BM + wave * 16 + 4 * g + e;
            const int j = cc * 16 + c;
            if (m < a.R && j < N) out[(size_t)m * N + j] = -accd[cc][e];
        }
}

// ---------------------------------------------------------------------------
// host side: launches of one problem or of a table of problems

template <int MODE, int KT>
static constexpr size_t s23_lds_g() {
    using T = typename ModeT<MODE>::in_t;
    return (size_t)16 * KT * (16 * KT + S23Geom<MODE>::pad) * sizeof(T);
}
static size_t s23_lds_b(int mode, int n) {
    return (size_t)4 * ((n + 3) / 4) * 16 * (mode == MODE_F64 ? 8 : 4);
}

template <int MODE, int KT>
static bool s23_glds() {
    return s23_lds_g<MODE, KT>() + S23Pt<MODE, KT>::value * s23_lds_b(MODE, 16 * KT) <=
           (size_t)120 * 1024;
}

// default waves per S23 workgroup: ~16 resident waves per CU
template <int MODE, int KT>
static int s23_default_waves(int n) {
    const size_t lds = (s23_glds<MODE, KT>() ? s23_lds_g<MODE, KT>() : 0) +
                       S23Pt<MODE, KT>::value * s23_lds_b(MODE, n);
    const int per_cu = std::max<int>(1, (int)((160 * 1024) / lds));
    return std::min(S23Threads<MODE, KT>::value / 64, std::max(4, 16 / per_cu));
}

template <int MODE, int KT>
static int launch_s23_kt(hipStream_t st, dim3 grid, int waves, size_t lds_b, const KRef<S23Args> &r,
                         bool attr_only) {
    // lds_b: the G(-tau) columns of one p tile; S23Pt tiles per workgroup
    constexpr int PT = S23Pt<MODE, KT>::value;
    const bool glds = s23_glds<MODE, KT>();
    const size_t lds = (glds ? s23_lds_g<MODE, KT>() : 0) + PT * lds_b;
    waves = std::min(waves, S23Threads<MODE, KT>::value / 64);
    const void *fn = glds ? (const void *)k_s23<MODE, KT, true> : (const void *)k_s23<MODE, KT, false>;
    // the same limit (the largest any n of this KT needs) on every path
    const size_t lds_max = (glds ? s23_lds_g<MODE, KT>() : 0) + PT * s23_lds_b(MODE, 16 * KT);
    GF2_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_max));
    if (attr_only) return GF2_OK;
    if (glds) hipLaunchKernelGGL((k_s23<MODE, KT, true>), grid, dim3(64 * waves), lds, st, r);
    else hipLaunchKernelGGL((k_s23<MODE, KT, false>), grid, dim3(64 * waves), lds, st, r);
    GF2_HIP(hipGetLastError());
    return GF2_OK;
}

template <int MODE>
static int launch_s23(hipStream_t st, int kt, dim3 grid, int waves, size_t lds_b,
                      const KRef<S23Args> &r, bool attr_only = false) {
    switch (kt) {
#define GF2_S23_CASE(K_) case K_: return launch_s23_kt<MODE, K_>(st, grid, waves, lds_b, r, attr_only);
        GF2_S23_CASE(1) GF2_S23_CASE(2) GF2_S23_CASE(3) GF2_S23_CASE(4) GF2_S23_CASE(5)
        GF2_S23_CASE(6) GF2_S23_CASE(7) GF2_S23_CASE(8) GF2_S23_CASE(9) GF2_S23_CASE(10)
#undef GF2_S23_CASE
        default: return fail(GF2_EINVAL, "gf2_sigma_tau: n > 160 is not supported");
    }
}

template <int MODE>
static int default_waves(int kt, int n) {
    switch (kt) {
#define GF2_W_CASE(K_) case K_: return s23_default_waves<MODE, K_>(n);
        GF2_W_CASE(1) GF2_W_CASE(2) GF2_W_CASE(3) GF2_W_CASE(4) GF2_W_CASE(5)
        GF2_W_CASE(6) GF2_W_CASE(7) GF2_W_CASE(8) GF2_W_CASE(9) GF2_W_CASE(10)
#undef GF2_W_CASE
        default: return 4;
    }
}

template <int MODE>
static int max_waves(int kt) {
    switch (kt) {
#define GF2_M_CASE(K_) case K_: return S23Threads<MODE, K_>::value / 64;
        GF2_M_CASE(1) GF2_M_CASE(2) GF2_M_CASE(3) GF2_M_CASE(4) GF2_M_CASE(5)
        GF2_M_CASE(6) GF2_M_CASE(7) GF2_M_CASE(8) GF2_M_CASE(9) GF2_M_CASE(10)
#undef GF2_M_CASE
        default: return 4;
    }
}

template <int MODE>
static int launch_s4(hipStream_t st, int nt, dim3 grid, const KRef<S4Args> &r) {
    switch (nt) {
#define GF2_S4_CASE(T_) case T_: hipLaunchKernelGGL((k_s4<MODE, T_>), grid, dim3(S4_THREADS), 0, st, r); break;
        GF2_S4_CASE(1) GF2_S4_CASE(2) GF2_S4_CASE(3) GF2_S4_CASE(4) GF2_S4_CASE(5)
        GF2_S4_CASE(6) GF2_S4_CASE(7) GF2_S4_CASE(8) GF2_S4_CASE(9) GF2_S4_CASE(10)
#undef GF2_S4_CASE
        default: return fail(GF2_EINVAL, "gf2_sigma_tau: n > 160 is not supported");
    }
    GF2_HIP(hipGetLastError());
    return GF2_OK;
}

// Largest column-tile count of the split forms: BF16x3 runs n <= 160, BF16x6
// (three planes of the G slices in LDS) n <= 144.
static int split_max_kt(int np) { return np == 3 ? 9 : 10; }

template <int KT>
static size_t s23b3_lds(int n, int np) {
    constexpr int KP = (KT + 1) / 2;
    constexpr int P16 = 16 * KT;
    constexpr int SLG = 32 * KP + 8;
    const int SQ = 32 * ((n + 31) / 32) + 8;
    return 2 * (size_t)np * ((size_t)P16 * SLG + (size_t)16 * S23bPt<KT>::value * SQ);
}

template <int KT, int NP, bool F32IN>
static int launch_s23_bf3_kt(hipStream_t st, dim3 grid, int waves, size_t lds,
                             const KRef<S23b3Args> &r, bool attr_only) {
    GF2_HIP(hipFuncSetAttribute((const void *)k_s23_bf3<KT, NP, F32IN>,
                                hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)s23b3_lds<KT>(16 * KT, NP)));
    if (attr_only) return GF2_OK;
    hipLaunchKernelGGL((k_s23_bf3<KT, NP, F32IN>), grid, dim3(64 * std::min(waves, 8)), lds, st, r);
    GF2_HIP(hipGetLastError());
    return GF2_OK;
}

static size_t s23_bf3_lds(int kt, int n, int np) {
    switch (kt) {
#define GF2_L_CASE(K_) case K_: return s23b3_lds<K_>(n, np);
        GF2_L_CASE(1) GF2_L_CASE(2) GF2_L_CASE(3) GF2_L_CASE(4) GF2_L_CASE(5)
        GF2_L_CASE(6) GF2_L_CASE(7) GF2_L_CASE(8) GF2_L_CASE(9) GF2_L_CASE(10)
#undef GF2_L_CASE
        default: return 0;
    }
}

// f32in: T1 is FP32 (mixed mode: three planes only)
static int launch_s23_bf3(hipStream_t st, int np, bool f32in, int kt, dim3 grid, int waves, size_t lds,
                          const KRef<S23b3Args> &r, bool attr_only = false) {
    if (kt > split_max_kt(np)) return fail(GF2_EINVAL, "gf2_sigma_tau: n too large for this precision");
    if (f32in) {
        if (np != 3) return fail(GF2_EINVAL, "gf2_sigma_tau: FP32 T1 needs the three-term split");
        switch (kt) {
#define GF2_B_CASE(K_) case K_: return launch_s23_bf3_kt<K_, 3, true>(st, grid, waves, lds, r, attr_only);
            GF2_B_CASE(1) GF2_B_CASE(2) GF2_B_CASE(3) GF2_B_CASE(4) GF2_B_CASE(5)
            GF2_B_CASE(6) GF2_B_CASE(7) GF2_B_CASE(8) GF2_B_CASE(9)
#undef GF2_B_CASE
            default: break;
        }
    } else if (np == 3) {
        switch (kt) {
#define GF2_B_CASE(K_) case K_: return launch_s23_bf3_kt<K_, 3, false>(st, grid, waves, lds, r, attr_only);
            GF2_B_CASE(1) GF2_B_CASE(2) GF2_B_CASE(3) GF2_B_CASE(4) GF2_B_CASE(5)
            GF2_B_CASE(6) GF2_B_CASE(7) GF2_B_CASE(8) GF2_B_CASE(9)
#undef GF2_B_CASE
            default: break;
        }
    } else {
        switch (kt) {
#define GF2_B_CASE(K_) case K_: return launch_s23_bf3_kt<K_, 2, false>(st, grid, waves, lds, r, attr_only);
            GF2_B_CASE(1) GF2_B_CASE(2) GF2_B_CASE(3) GF2_B_CASE(4) GF2_B_CASE(5)
            GF2_B_CASE(6) GF2_B_CASE(7) GF2_B_CASE(8) GF2_B_CASE(9) GF2_B_CASE(10)
#undef GF2_B_CASE
            default: break;
        }
    }
    return fail(GF2_EINVAL, "gf2_sigma_tau: n > 160 is not supported");
}

static int launch_s4_bf3(hipStream_t st, int np, int nt, dim3 grid, const KRef<S4b3Args> &r) {
    if (nt > split_max_kt(np)) return fail(GF2_EINVAL, "gf2_sigma_tau: n too large for this precision");
    if (np == 3) {
        switch (nt) {
#define GF2_S4B_CASE(T_) case T_: hipLaunchKernelGGL((k_s4_bf3<T_, 3>), grid, dim3(S4_THREADS), 0, st, r); break;
            GF2_S4B_CASE(1) GF2_S4B_CASE(2) GF2_S4B_CASE(3) GF2_S4B_CASE(4) GF2_S4B_CASE(5)
            GF2_S4B_CASE(6) GF2_S4B_CASE(7) GF2_S4B_CASE(8) GF2_S4B_CASE(9)
#undef GF2_S4B_CASE
            default: return fail(GF2_EINVAL, "gf2_sigma_tau: n > 160 is not supported");
        }
    } else {
        switch (nt) {
#define GF2_S4B_CASE(T_) case T_: hipLaunchKernelGGL((k_s4_bf3<T_, 2>), grid, dim3(S4_THREADS), 0, st, r); break;
            GF2_S4B_CASE(1) GF2_S4B_CASE(2) GF2_S4B_CASE(3) GF2_S4B_CASE(4) GF2_S4B_CASE(5)
            GF2_S4B_CASE(6) GF2_S4B_CASE(7) GF2_S4B_CASE(8) GF2_S4B_CASE(9) GF2_S4B_CASE(10)
#undef GF2_S4B_CASE
            default: return fail(GF2_EINVAL, "gf2_sigma_tau: n > 160 is not supported");
        }
    }
    GF2_HIP(hipGetLastError());
    return GF2_OK;
}

// W2 planes for the split-BF16 final contraction (once per system; three
// planes, of which BF16x3 reads the first two)
static int build_bf3_layouts(gf2_ctx *c) {
    const long long n = c->n, n3 = n * n * n;
    const int bn = 16 * (int)((n + 15) / 16);
    const long long nkc = (n3 + 63) / 64;
    const size_t plane = (size_t)nkc * bn * 64;
    GF2_TRY(c->W2_b3.ensure(3 * plane * 2));
    const unsigned blocks = (unsigned)std::min<size_t>((plane + 255) / 256, 65536);
    hipLaunchKernelGGL(k_build_w2b, dim3(blocks), dim3(256), 0, c->stream, (int)n, bn, nkc, plane,
                       c->v.as<double>(), c->W2_b3.as<unsigned short>());
    GF2_HIP(hipGetLastError());
    c->have_bf3_layouts = true;
    return GF2_OK;
}

// ---------------------------------------------------------------------------
// One system's Sigma(tau): sizes, workspaces and launch shapes.  The tau batch
// b, the waves per S23 workgroup and the tile shapes change only which
// workgroup computes which independent result, never the arithmetic of a result
// (the first transform's K chunks are added in the same k order whatever their
// depth), so the autotuner below may pick them freely.
struct SigShape {
    int b = 0;
    int waves = 0;
    int s4cb = 0;    // FP64/FP32 final contraction: column blocks per row block (1 or 2)
    int s1_bk = 0;   // first transform, FP32 kernel: K chunk (16 or 20; 0 = by n)
    int s1_nt = 0;   // first transform: 16-column tiles per workgroup (0 = fewest blocks of <= 8)
};

struct SigPlan {
    gf2_ctx *c = nullptr;
    int mode = 0, n = 0, ntau = 0, M = 0;
    const double *G = nullptr;
    double *Sig = nullptr;
    int KT = 0, SL = 0, lq = 0, KP = 0, SLG = 0, nsplit = 0, s1_bk = 16, s1_nt = 0;
    int s4_nt = 0;   // 16-column tiles per S4 workgroup (KT split over sh.s4cb blocks)
    long long kz = 0;
    size_t t1_plane = 0, gq_plane = 0;
    SigShape sh;
    const void *V = nullptr, *W2 = nullptr;
};

// Largest tau batch.  T1 and X of b tau points take b (esz + t1sz) n^4 bytes;
// the batch gets up to 48 GiB of them (at n = 100 in FP32, 64 tau points: then
// b n = 6400 rows fill whole 128-row blocks of the first transform and the
// final contraction), and at most half of the device memory that is free or
// already held by these two buffers.  Every batch size gives bitwise the same
// Sigma(tau), so the choice only moves time.
static int sigma_bmax(const gf2_ctx *c, int mode) {
    const size_t n = (size_t)c->n;
    const size_t esz = (mode == MODE_F64) ? 8 : 4;
    const size_t t1sz = split_planes(mode) ? 2 * (size_t)split_planes(mode) : esz;   // T1 element
    const size_t N4 = n * n * n * n;
    size_t budget = (size_t)48 << 30;
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) == hipSuccess)
        budget = std::min(budget, (fr + c->sig_T1.bytes + c->sig_X.bytes) / 2);
    return (int)std::min<size_t>(std::max<size_t>(1, budget / (N4 * (esz + t1sz))), 64);
}

static int plan_init(gf2_ctx *c, int ntau, int prec, const double *G, double *Sig, SigShape sh,
                     SigPlan &p) {
    const int n = c->n;
    if (n > 160) return fail(GF2_EINVAL, "gf2_sigma_tau: n > 160 is not supported");
    const int np = split_planes(prec), np23 = s23_planes(prec), np4 = s4_planes(prec);
    if (np23 && (n + 15) / 16 > split_max_kt(np23))
        return fail(GF2_EINVAL, "gf2_sigma_tau: the three-term split forms support n <= 144");
    p = SigPlan();
    p.c = c;
    p.mode = prec;
    p.n = n;
    p.ntau = ntau;
    p.M = ntau - 1;
    p.G = G;
    p.Sig = Sig;
    const long long N = n, N2 = N * N, N3 = N2 * N, N4 = N3 * N;
    const size_t esz = (p.mode == MODE_F64) ? 8 : 4;
    if (p.mode != MODE_F64 && !c->have_f32_layouts) GF2_TRY(sigma_build_layouts(c, true));
    if (np4 && !c->have_bf3_layouts) GF2_TRY(build_bf3_layouts(c));
    p.V = (p.mode == MODE_F64) ? c->v.ptr : c->v_32.ptr;
    p.W2 = (p.mode == MODE_F64) ? c->W2_64.ptr : c->W2_32.ptr;
    p.KT = (n + 15) / 16;
    p.SL = 16 * p.KT + ((p.mode == MODE_F64) ? S23Geom<MODE_F64>::pad : S23Geom<MODE_F32>::pad);
    p.lq = (n + 7) / 8 * 8;
    p.KP = (p.KT + 1) / 2;
    p.SLG = 32 * p.KP + 8;
    p.kz = 4096;
    if (N3 < 8 * 4096) p.kz = std::max<long long>(512, ((N3 / 8) + 511) / 512 * 512);
    p.nsplit = (int)((N3 + p.kz - 1) / p.kz);
    p.s1_bk = (s1_mode(p.mode) == MODE_F32 && n % 16 != 0 && n % 20 == 0) ? 20 : 16;
    if (s1_mode(p.mode) == MODE_F32 && (sh.s1_bk == 16 || sh.s1_bk == 20)) p.s1_bk = sh.s1_bk;
    p.s1_nt = (sh.s1_nt >= 1 && sh.s1_nt <= 8) ? sh.s1_nt : 0;
    const int bmax = sigma_bmax(c, p.mode);
    p.sh.b = std::max(1, std::min(sh.b > 0 ? sh.b : bmax, std::min(bmax, ntau)));
    const int wmax = (p.mode == MODE_F64) ? max_waves<MODE_F64>(p.KT)
                     : (p.mode == MODE_F32) ? max_waves<MODE_F32>(p.KT) : 8;
    if (sh.waves > 0) {
        p.sh.waves = std::min(sh.waves, wmax);
    } else if (np23) {
        const int per_cu = std::max<int>(1, (int)((160 * 1024) / s23_bf3_lds(p.KT, n, np23)));
        p.sh.waves = std::min(8, std::max(4, 16 / per_cu));
    } else {
        p.sh.waves = (p.mode == MODE_F64) ? default_waves<MODE_F64>(p.KT, n)
                                          : default_waves<MODE_F32>(p.KT, n);
    }
    p.sh.s4cb = np4 ? 1 : (sh.s4cb > 0 ? std::min(sh.s4cb, 2) : 1);
    p.s4_nt = (p.KT + p.sh.s4cb - 1) / p.sh.s4cb;
    const size_t b = (size_t)p.sh.b;
    p.t1_plane = b * N2 * N * p.lq;
    p.gq_plane = b * 16 * p.KT * p.SLG;
    if (np) GF2_TRY(c->sig_T1.ensure(np * p.t1_plane * 2));
    if (np23) GF2_TRY(c->sig_Gq.ensure(np23 * p.gq_plane * 2));
    GF2_TRY(c->sig_T1.ensure(b * N4 * esz));
    GF2_TRY(c->sig_X.ensure(b * N4 * esz));
    GF2_TRY(c->sig_G.ensure(b * N2 * esz));
    GF2_TRY(c->sig_Gb.ensure(b * N2 * esz));
    GF2_TRY(c->sig_Gp.ensure(b * 16 * p.KT * p.SL * esz));
    GF2_TRY(c->sig_part.ensure((size_t)p.nsplit * b * N2 * 8));
    return GF2_OK;
}

// staging of G(tau), G(-tau) for tau points k0 .. k0 + nb - 1
static int plan_stage(const SigPlan &p, hipStream_t st, int k0, int nb) {
    gf2_ctx *c = p.c;
    const int n = p.n;
    const size_t N2 = (size_t)n * n;
    const size_t tot = (size_t)nb * N2;
    const unsigned blocks = (unsigned)std::min<size_t>((tot + 255) / 256, 4096);
    const size_t totp = (size_t)nb * 16 * p.KT * p.SL;
    const unsigned blocksp = (unsigned)std::min<size_t>((totp + 255) / 256, 4096);
    if (p.mode == MODE_F64) {
        hipLaunchKernelGGL(k_stage_g<double>, dim3(blocks), dim3(256), 0, st, n, p.M, k0, nb, p.G,
                           c->sig_G.as<double>(), c->sig_Gb.as<double>());
        hipLaunchKernelGGL(k_stage_gp<double>, dim3(blocksp), dim3(256), 0, st, n, p.KT, p.SL, 0,
                           p.M, k0, nb, p.G, c->sig_Gp.as<double>());
    } else {
        hipLaunchKernelGGL(k_stage_g<float>, dim3(blocks), dim3(256), 0, st, n, p.M, k0, nb, p.G,
                           c->sig_G.as<float>(), c->sig_Gb.as<float>());
        if (s23_planes(p.mode) == 0) {
            hipLaunchKernelGGL(k_stage_gp<float>, dim3(blocksp), dim3(256), 0, st, n, p.KT,
                               p.SL, 16 * (p.KT - 1), p.M, k0, nb, p.G, c->sig_Gp.as<float>());
        } else {
            const size_t totq = (size_t)nb * 16 * p.KT * p.SLG;
            const unsigned blocksq = (unsigned)std::min<size_t>((totq + 255) / 256, 4096);
            hipLaunchKernelGGL(k_stage_gq, dim3(blocksq), dim3(256), 0, st, n, p.KP, p.SLG, 16 * p.KT,
                               k0, nb, p.gq_plane, s23_planes(p.mode), p.G,
                               c->sig_Gq.as<unsigned short>());
        }
    }
    GF2_HIP(hipGetLastError());
    return GF2_OK;
}

static int plan_reduce(const SigPlan &p, hipStream_t st, int k0, int nb) {
    const size_t tot = (size_t)nb * p.n * p.n;
    const unsigned blocks = (unsigned)std::min<size_t>((tot + 255) / 256, 4096);
    hipLaunchKernelGGL(k_reduce_split, dim3(blocks), dim3(256), 0, st, p.n, nb, p.nsplit,
                       p.c->sig_part.as<double>(), p.Sig, k0);
    GF2_HIP(hipGetLastError());
    return GF2_OK;
}

// arguments of the three contraction stages for a batch of nb tau points
static GemmArgs plan_s1(const SigPlan &p, int nb, int &nt) {
    const long long N = p.n, N2 = N * N, N3 = N2 * N;
    const long long R = (long long)nb * N;
    GemmArgs g{};
    g.A = p.c->sig_G.ptr; g.lda = N; g.sA = 0;
    g.B = p.V; g.ldb = N2; g.sB = N3;
    g.C = p.c->sig_T1.ptr; g.ldc = N2; g.sC = R * N2;
    g.M = (int)R; g.N = (int)N2; g.K = p.n; g.kz = p.n; g.split = 0;
    g.alpha = 1.0;
    g.vecA = 0;
    if (split_planes(p.mode)) {
        g.vecA = (p.n % 4 == 0) ? 1 : 0;
        g.pn = p.n;
        g.pld = p.lq;
        g.ldc = N * p.lq;
        g.sC = R * N * p.lq;
        g.plane = (long long)p.t1_plane;
    }
    dim3 grid = gemm_grid(g, p.n, nt);
    if (p.s1_nt > 0) {   // tuned column tile
        nt = p.s1_nt;
        grid.y = (unsigned)(((g.N + 15) / 16 + nt - 1) / nt);
    }
    g.gx = (int)grid.x;
    g.gy = (int)grid.y;
    g.gz = (int)grid.z;
    return g;
}

static S23Args plan_s23(const SigPlan &p, int nb) {
    return S23Args{p.c->sig_T1.ptr, p.c->sig_Gp.ptr, p.c->sig_Gb.ptr, p.c->sig_X.ptr, p.n, nb};
}

static S23b3Args plan_s23b3(const SigPlan &p, int nb) {
    S23b3Args a{};
    a.T1 = p.c->sig_T1.as<unsigned short>();
    a.t1_plane = (long long)p.t1_plane;
    a.lq = split_planes(p.mode) ? p.lq : p.n;
    a.Gq = p.c->sig_Gq.as<unsigned short>();
    a.gq_plane = (long long)p.gq_plane;
    a.Gb = p.c->sig_Gb.as<float>();
    a.X = p.c->sig_X.as<float>();
    a.n = p.n;
    a.nb = nb;
    return a;
}

static S4Args plan_s4(const SigPlan &p, int nb) {
    const long long N = p.n, N3 = N * N * N;
    const long long R = (long long)nb * N;
    S4Args a{};
    a.X = p.c->sig_X.ptr;
    a.W = p.W2;
    a.part = p.c->sig_part.as<double>();
    a.K = N3;
    a.kz = p.kz;
    a.n = p.n;
    a.R = (int)R;
    a.nrb = (int)((R + S4_BM - 1) / S4_BM);
    a.nsplit = p.nsplit;
    a.vec = (p.mode == MODE_F64) ? (p.n % 2 == 0) : (p.n % 4 == 0);
    a.ncb = p.sh.s4cb;
    return a;
}

static S4b3Args plan_s4b3(const SigPlan &p, int nb) {
    const S4Args a = plan_s4(p, nb);
    const long long nkc = (a.K + 63) / 64;
    S4b3Args b{};
    b.X = p.c->sig_X.as<float>();
    b.W2b = p.c->W2_b3.as<unsigned short>();
    b.plane = nkc * 16 * p.KT * 64;
    b.part = a.part;
    b.K = a.K;
    b.kz = a.kz;
    b.n = a.n;
    b.R = a.R;
    b.nrb = a.nrb;
    b.nsplit = a.nsplit;
    b.vec = (p.n % 4 == 0);
    return b;
}

static int launch_s1(int mode_, int bk, int nt, dim3 grid, hipStream_t st, const KRef<GemmArgs> &r) {
    const int mode = s1_mode(mode_);
    if (mode == MODE_F64) launch_nt<MODE_F64, false, true, 16>(nt, grid, st, r);
    else if (mode == MODE_BF3) launch_nt<MODE_BF3, false, true, 0>(nt, grid, st, r);
    else if (mode == MODE_BF6) launch_nt<MODE_BF6, false, true, 0>(nt, grid, st, r);
    else if (bk == 20) launch_nt<MODE_F32, false, false, 20>(nt, grid, st, r);
    else launch_nt<MODE_F32, false, false, 16>(nt, grid, st, r);
    GF2_HIP(hipGetLastError());
    return GF2_OK;
}

// One tau batch of one system, arguments by value (no table).
static int plan_run_batch(const SigPlan &p, hipStream_t st, int k0, int nb, bool prof) {
    gf2_ctx *c = p.c;
    const double fl = 2.0 * std::pow((double)p.n, 5) * nb;
    GF2_TRY(plan_stage(p, st, k0, nb));
    {
        int nt;
        KRef<GemmArgs> r{};
        r.one = plan_s1(p, nb, nt);
        const dim3 grid(xcd_grid((long long)r.one.gx * r.one.gy * r.one.gz));
        const int ph = prof ? prof_begin(c, GF2_KC_SIGMA_GEMM) : -1;
        GF2_TRY(launch_s1(p.mode, p.s1_bk, nt, grid, st, r));
        if (prof) prof_end(c, ph, fl);
    }
    {
        const int np = s23_planes(p.mode);
        const int groups = np ? s23b_groups(p.KT) : s23_groups(p.mode, p.KT);
        const dim3 grid(xcd_grid((long long)nb * p.n * groups));
        const int ph = prof ? prof_begin(c, GF2_KC_SIGMA_S23) : -1;
        if (np) {
            KRef<S23b3Args> r{};
            r.one = plan_s23b3(p, nb);
            GF2_TRY(launch_s23_bf3(st, np, split_planes(p.mode) == 0, p.KT, grid, p.sh.waves,
                                   s23_bf3_lds(p.KT, p.n, np), r));
        } else {
            KRef<S23Args> r{};
            r.one = plan_s23(p, nb);
            if (p.mode == MODE_F64)
                GF2_TRY(launch_s23<MODE_F64>(st, p.KT, grid, p.sh.waves, s23_lds_b(p.mode, p.n), r));
            else
                GF2_TRY(launch_s23<MODE_F32>(st, p.KT, grid, p.sh.waves, s23_lds_b(p.mode, p.n), r));
        }
        if (prof) prof_end(c, ph, 2.0 * fl);
    }
    {
        const int ph = prof ? prof_begin(c, GF2_KC_SIGMA_SPLITK) : -1;
        if (s4_planes(p.mode)) {
            KRef<S4b3Args> r{};
            r.one = plan_s4b3(p, nb);
            const dim3 grid(xcd_grid((long long)r.one.nrb * r.one.nsplit));
            GF2_TRY(launch_s4_bf3(st, s4_planes(p.mode), p.KT, grid, r));
        } else {
            KRef<S4Args> r{};
            r.one = plan_s4(p, nb);
            const dim3 grid(xcd_grid((long long)r.one.nrb * r.one.nsplit * r.one.ncb));
            if (p.mode == MODE_F64) GF2_TRY(launch_s4<MODE_F64>(st, p.s4_nt, grid, r));
            else GF2_TRY(launch_s4<MODE_F32>(st, p.s4_nt, grid, r));
        }
        if (prof) prof_end(c, ph, fl);
    }
    return plan_reduce(p, st, k0, nb);
}

static int plan_run(SigPlan &p, bool prof) {
    if (split_planes(p.mode))   // the first transform never writes the padding of the T1 rows
        GF2_TRY(fill_zero(p.c, p.c->sig_T1.ptr, split_planes(p.mode) * p.t1_plane * 2));
    for (int k0 = 0; k0 < p.ntau; k0 += p.sh.b)
        GF2_TRY(plan_run_batch(p, p.c->stream, k0, std::min(p.sh.b, p.ntau - k0), prof));
    return GF2_OK;
}

// ---------------------------------------------------------------------------
// Autotuner: on the first Sigma(tau) of an (n, ntau, precision) class, time
// each candidate shape on the first tau batch of the real input and keep the
// fastest per tau point (process-wide cache).  GF2_SIGMA_TUNE=0 in the
// environment skips tuning (default shape).
struct TuneKey {
    int n, ntau, mode;
    bool operator<(const TuneKey &o) const {
        return n != o.n ? n < o.n : ntau != o.ntau ? ntau < o.ntau : mode < o.mode;
    }
};
static std::mutex g_tune_mu;
static std::map<TuneKey, SigShape> g_tune;
// Candidates are timed in order of preference (larger tau batches, fewer
// waves, the rule's first-transform shape first); a later one replaces the
// best so far only when it is faster by more than 2%, so shapes within the
// timing noise of each other do not swap from one process to the next.
constexpr double kTuneMargin = 0.98;

static int tuned_shape(gf2_ctx *c, int ntau, int prec, const double *G, double *Sig, SigShape &out) {
    // GF2_SIGMA_SHAPE="b,waves[,s4cb[,s1_bk,s1_nt]]" forces a shape (read on every
    // call; for tests of the invariance and for sweeps)
    if (const char *fs = std::getenv("GF2_SIGMA_SHAPE")) {
        int b = 0, w = 0, cb = 0, bk = 0, nt = 0;
        const int got = std::sscanf(fs, "%d,%d,%d,%d,%d", &b, &w, &cb, &bk, &nt);
        if (got >= 2 && b > 0 && w > 0) {
            out = SigShape{b, w, got >= 3 ? cb : 0, got >= 5 ? bk : 0, got >= 5 ? nt : 0};
            return GF2_OK;
        }
    }
    const TuneKey key{c->n, ntau, prec};
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune.find(key);
        if (it != g_tune.end()) {
            out = it->second;
            return GF2_OK;
        }
    }
    const char *env = std::getenv("GF2_SIGMA_TUNE");
    SigShape best{};
    if (!(env && env[0] == '0')) {
        const int bmax = std::min(sigma_bmax(c, prec), ntau);
        std::vector<int> bs;
        for (int b : {bmax, (bmax + 1) / 2, (bmax + 3) / 4})
            if (b >= 1 && std::find(bs.begin(), bs.end(), b) == bs.end()) bs.push_back(b);
        std::vector<int> ws = s23_planes(prec) ? std::vector<int>{4, 8} : std::vector<int>{4, 8, 16};
        hipEvent_t e0, e1;
        GF2_HIP(hipEventCreate(&e0));
        GF2_HIP(hipEventCreate(&e1));
        double best_t = 1e300;
        int rc = GF2_OK;
        std::vector<int> cbs = s4_planes(prec) ? std::vector<int>{1} : std::vector<int>{1, 2};
        for (int b : bs) {
          for (int cb : cbs) {
            for (int w : ws) {
                SigPlan p;
                rc = plan_init(c, ntau, prec, G, Sig, SigShape{b, w, cb}, p);
                if (rc != GF2_OK) break;
                if (p.sh.waves != w || p.sh.s4cb != cb) continue;   // not a distinct shape
                if (split_planes(prec)) rc = fill_zero(c, c->sig_T1.ptr, split_planes(prec) * p.t1_plane * 2);
                if (rc != GF2_OK) break;
                const int nb = std::min(b, ntau);
                (void)hipEventRecord(e0, c->stream);
                rc = plan_run_batch(p, c->stream, 0, nb, false);
                (void)hipEventRecord(e1, c->stream);
                if (rc != GF2_OK) break;
                if (hipEventSynchronize(e1) != hipSuccess) { rc = fail(GF2_EHIP, "autotuner: event"); break; }
                float ms = 0.0f;
                (void)hipEventElapsedTime(&ms, e0, e1);
                const double per_tau = ms / nb;
                if (per_tau < best_t * kTuneMargin) {
                    best_t = per_tau;
                    best = SigShape{b, p.sh.waves, p.sh.s4cb};
                }
            }
            if (rc != GF2_OK) break;
          }
          if (rc != GF2_OK) break;
        }
        // the first transform's tile shape, timed alone on the best tau batch
        // (its output, and so the later stages, do not depend on it)
        if (rc == GF2_OK) {
            std::vector<std::pair<int, int>> s1c{{0, 0}, {16, 4}, {16, 8}};
            if (s1_mode(prec) == MODE_F32 && c->n % 20 == 0) s1c.push_back({20, 4});
            double best_s1 = 1e300;
            for (auto bn : s1c) {
                SigShape sh = best;
                sh.s1_bk = bn.first;
                sh.s1_nt = bn.second;
                SigPlan p;
                rc = plan_init(c, ntau, prec, G, Sig, sh, p);
                if (rc != GF2_OK) break;
                const int nb = std::min(p.sh.b, ntau);
                rc = plan_stage(p, c->stream, 0, nb);
                if (rc != GF2_OK) break;
                int nt;
                KRef<GemmArgs> r{};
                r.one = plan_s1(p, nb, nt);
                const dim3 grid(xcd_grid((long long)r.one.gx * r.one.gy * r.one.gz));
                (void)hipEventRecord(e0, c->stream);
                rc = launch_s1(p.mode, p.s1_bk, nt, grid, c->stream, r);
                (void)hipEventRecord(e1, c->stream);
                if (rc != GF2_OK) break;
                if (hipEventSynchronize(e1) != hipSuccess) { rc = fail(GF2_EHIP, "autotuner: event"); break; }
                float ms = 0.0f;
                (void)hipEventElapsedTime(&ms, e0, e1);
                if (ms < best_s1 * kTuneMargin) {
                    best_s1 = ms;
                    best.s1_bk = bn.first;
                    best.s1_nt = bn.second;
                }
            }
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        GF2_TRY(rc);
    }
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[key] = best;
    out = best;
    return GF2_OK;
}

int sigma_run(gf2_ctx *c, const gf2_dims *d, int prec, const double *G_tau, double *Sigma_tau) {
    SigShape sh;
    GF2_TRY(tuned_shape(c, d->ntau, prec, G_tau, Sigma_tau, sh));
    SigPlan p;
    GF2_TRY(plan_init(c, d->ntau, prec, G_tau, Sigma_tau, sh, p));
    return plan_run(p, true);
}

// ---------------------------------------------------------------------------
// Many systems: every tau batch of every system in shared launches (one per
// kernel class and stage), captured once per batch shape into a HIP graph on
// the lead context's capture stream and replayed on its stream.  The argument
// tables of all launches are uploaded once with the capture.

struct GroupLaunch {
    int stage;      // 1 = S1, 2 = S23, 4 = S4
    int cls_a, cls_b, cls_c;   // S1: bk, nt, -; S23: KT, waves, -; S4: NT
    size_t tab_off, boff_off;  // byte offsets into the table buffer
    int nsys, total;
    size_t lds;
};

template <class A>
static void push_table(std::vector<unsigned char> &buf, const std::vector<A> &tab,
                       const std::vector<int> &boff, GroupLaunch &gl) {
    auto align = [&](size_t a) { while (buf.size() % a) buf.push_back(0); };
    align(16);
    gl.tab_off = buf.size();
    const unsigned char *t = reinterpret_cast<const unsigned char *>(tab.data());
    buf.insert(buf.end(), t, t + tab.size() * sizeof(A));
    align(16);
    gl.boff_off = buf.size();
    const unsigned char *b = reinterpret_cast<const unsigned char *>(boff.data());
    buf.insert(buf.end(), b, b + boff.size() * sizeof(int));
}

int sigma_run_batched(gf2_ctx *lead, const std::vector<gf2_ctx *> &cs, const std::vector<int> &ntau,
                      int prec, const std::vector<const double *> &G,
                      const std::vector<double *> &Sig) {
    const int ns = (int)cs.size();
    std::vector<SigPlan> plans(ns);
    for (int s = 0; s < ns; ++s) {
        SigShape sh;
        GF2_TRY(tuned_shape(cs[s], ntau[s], prec, G[s], Sig[s], sh));
        GF2_TRY(plan_init(cs[s], ntau[s], prec, G[s], Sig[s], sh, plans[s]));
    }
    const int np = split_planes(prec), np23 = s23_planes(prec), np4 = s4_planes(prec);
    const bool f32in = np == 0;
    if (np)
        for (auto &p : plans) GF2_TRY(fill_zero(p.c, p.c->sig_T1.ptr, np * p.t1_plane * 2));
    // shape key: everything the captured launches depend on
    long long key = 1469598103934665603LL ^ prec;
    auto mix = [&](long long v) { key = (key ^ v) * 1099511628211LL; };
    for (auto &p : plans) {
        mix(p.n); mix(p.ntau); mix(p.sh.b); mix(p.sh.waves); mix(p.sh.s4cb); mix(p.s1_bk); mix(p.s1_nt);
        mix((long long)(uintptr_t)p.G); mix((long long)(uintptr_t)p.Sig);
        mix((long long)(uintptr_t)p.c->sig_T1.ptr); mix((long long)(uintptr_t)p.c->sig_X.ptr);
        mix((long long)(uintptr_t)p.c->sig_part.ptr); mix((long long)(uintptr_t)p.c->sig_Gp.ptr);
        mix((long long)(uintptr_t)p.c->sig_Gq.ptr); mix((long long)(uintptr_t)p.V);
        mix((long long)(uintptr_t)p.W2); mix((long long)(uintptr_t)p.c->W2_b3.ptr);
    }
    if (lead->sig_graph && lead->sig_key == key) {
        GF2_HIP(hipGraphLaunch(static_cast<hipGraphExec_t>(lead->sig_graph), lead->stream));
        return GF2_OK;
    }
    if (lead->sig_graph) {
        (void)hipGraphExecDestroy(static_cast<hipGraphExec_t>(lead->sig_graph));
        lead->sig_graph = nullptr;
        lead->sig_key = 0;
    }
    // rounds: round r = tau batch r of every system that has one
    int rounds = 0;
    for (auto &p : plans) rounds = std::max(rounds, (p.ntau + p.sh.b - 1) / p.sh.b);
    std::vector<unsigned char> buf;
    std::vector<std::vector<GroupLaunch>> per_round(rounds);
    for (int r = 0; r < rounds; ++r) {
        std::vector<int> act;
        for (int s = 0; s < ns; ++s)
            if (r * plans[s].sh.b < plans[s].ntau) act.push_back(s);
        auto nb_of = [&](int s) { return std::min(plans[s].sh.b, plans[s].ntau - r * plans[s].sh.b); };
        // S1 classes (bk, nt)
        std::map<std::pair<int, int>, std::vector<int>> c1;
        for (int s : act) {
            int nt;
            (void)plan_s1(plans[s], nb_of(s), nt);
            c1[{plans[s].s1_bk, nt}].push_back(s);
        }
        for (auto &kv : c1) {
            std::vector<GemmArgs> tab;
            std::vector<int> boff{0};
            for (int s : kv.second) {
                int nt;
                tab.push_back(plan_s1(plans[s], nb_of(s), nt));
                boff.push_back(boff.back() + tab.back().gx * tab.back().gy * tab.back().gz);
            }
            GroupLaunch gl{1, kv.first.first, kv.first.second, 0, 0, 0, (int)tab.size(), boff.back(), 0};
            push_table(buf, tab, boff, gl);
            per_round[r].push_back(gl);
        }
        // S23 classes (KT, waves)
        std::map<std::pair<int, int>, std::vector<int>> c2;
        for (int s : act) c2[{plans[s].KT, plans[s].sh.waves}].push_back(s);
        for (auto &kv : c2) {
            std::vector<int> boff{0};
            size_t lds = 0;
            GroupLaunch gl{2, kv.first.first, kv.first.second, 0, 0, 0, (int)kv.second.size(), 0, 0};
            if (np23) {
                std::vector<S23b3Args> tab;
                for (int s : kv.second) {
                    tab.push_back(plan_s23b3(plans[s], nb_of(s)));
                    boff.push_back(boff.back() + nb_of(s) * plans[s].n * s23b_groups(plans[s].KT));
                    lds = std::max(lds, s23_bf3_lds(plans[s].KT, plans[s].n, np23));
                }
                push_table(buf, tab, boff, gl);
            } else {
                std::vector<S23Args> tab;
                for (int s : kv.second) {
                    tab.push_back(plan_s23(plans[s], nb_of(s)));
                    boff.push_back(boff.back() +
                                   nb_of(s) * plans[s].n * s23_groups(prec, plans[s].KT));
                    lds = std::max(lds, s23_lds_b(prec, plans[s].n));
                }
                push_table(buf, tab, boff, gl);
            }
            gl.total = boff.back();
            gl.lds = lds;
            per_round[r].push_back(gl);
        }
        // S4 classes (NT)
        std::map<int, std::vector<int>> c4;
        for (int s : act) c4[np4 ? plans[s].KT : plans[s].s4_nt].push_back(s);
        for (auto &kv : c4) {
            std::vector<int> boff{0};
            GroupLaunch gl{4, kv.first, 0, 0, 0, 0, (int)kv.second.size(), 0, 0};
            if (np4) {
                std::vector<S4b3Args> tab;
                for (int s : kv.second) {
                    tab.push_back(plan_s4b3(plans[s], nb_of(s)));
                    boff.push_back(boff.back() + tab.back().nrb * tab.back().nsplit);
                }
                push_table(buf, tab, boff, gl);
            } else {
                std::vector<S4Args> tab;
                for (int s : kv.second) {
                    tab.push_back(plan_s4(plans[s], nb_of(s)));
                    boff.push_back(boff.back() + tab.back().nrb * tab.back().nsplit * tab.back().ncb);
                }
                push_table(buf, tab, boff, gl);
            }
            gl.total = boff.back();
            per_round[r].push_back(gl);
        }
    }
    GF2_TRY(lead->sig_tab.ensure(std::max<size_t>(buf.size(), 16)));
    GF2_HIP(hipMemcpyAsync(lead->sig_tab.ptr, buf.data(), buf.size(), hipMemcpyHostToDevice,
                           lead->stream));
    // dynamic-LDS limits are set outside the capture
    for (auto &v : per_round)
        for (auto &gl : v)
            if (gl.stage == 2) {
                KRef<S23Args> r0{};
                KRef<S23b3Args> r1{};
                if (np23) GF2_TRY(launch_s23_bf3(lead->stream, np23, f32in, gl.cls_a, dim3(1), gl.cls_b, gl.lds, r1, true));
                else if (prec == MODE_F64) GF2_TRY(launch_s23<MODE_F64>(lead->stream, gl.cls_a, dim3(1), gl.cls_b, gl.lds, r0, true));
                else GF2_TRY(launch_s23<MODE_F32>(lead->stream, gl.cls_a, dim3(1), gl.cls_b, gl.lds, r0, true));
            }
    GF2_HIP(hipStreamSynchronize(lead->stream));
    if (!lead->bat_cap) GF2_HIP(hipStreamCreateWithFlags(&lead->bat_cap, hipStreamNonBlocking));
    hipStream_t st = lead->bat_cap;
    unsigned char *tb = lead->sig_tab.as<unsigned char>();
    hipGraph_t graph = nullptr;
    GF2_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    int rc = GF2_OK;
    for (int r = 0; r < rounds && rc == GF2_OK; ++r) {
        for (int s = 0; s < ns && rc == GF2_OK; ++s) {
            auto &p = plans[s];
            if (r * p.sh.b < p.ntau) rc = plan_stage(p, st, r * p.sh.b, std::min(p.sh.b, p.ntau - r * p.sh.b));
        }
        for (auto &gl : per_round[r]) {
            if (rc != GF2_OK) break;
            const dim3 grid(xcd_grid(gl.total));
            if (gl.stage == 1) {
                KRef<GemmArgs> ref{};
                ref.tab = reinterpret_cast<const GemmArgs *>(tb + gl.tab_off);
                ref.boff = reinterpret_cast<const int *>(tb + gl.boff_off);
                ref.nsys = gl.nsys;
                ref.total = gl.total;
                rc = launch_s1(prec, gl.cls_a, gl.cls_b, grid, st, ref);
            } else if (gl.stage == 2) {
                if (np23) {
                    KRef<S23b3Args> ref{};
                    ref.tab = reinterpret_cast<const S23b3Args *>(tb + gl.tab_off);
                    ref.boff = reinterpret_cast<const int *>(tb + gl.boff_off);
                    ref.nsys = gl.nsys;
                    ref.total = gl.total;
                    rc = launch_s23_bf3(st, np23, f32in, gl.cls_a, grid, gl.cls_b, gl.lds, ref);
                } else {
                    KRef<S23Args> ref{};
                    ref.tab = reinterpret_cast<const S23Args *>(tb + gl.tab_off);
                    ref.boff = reinterpret_cast<const int *>(tb + gl.boff_off);
                    ref.nsys = gl.nsys;
                    ref.total = gl.total;
                    if (prec == MODE_F64) rc = launch_s23<MODE_F64>(st, gl.cls_a, grid, gl.cls_b, gl.lds, ref);
                    else rc = launch_s23<MODE_F32>(st, gl.cls_a, grid, gl.cls_b, gl.lds, ref);
                }
            } else {
                if (np4) {
                    KRef<S4b3Args> ref{};
                    ref.tab = reinterpret_cast<const S4b3Args *>(tb + gl.tab_off);
                    ref.boff = reinterpret_cast<const int *>(tb + gl.boff_off);
                    ref.nsys = gl.nsys;
                    ref.total = gl.total;
                    rc = launch_s4_bf3(st, np4, gl.cls_a, grid, ref);
                } else {
                    KRef<S4Args> ref{};
                    ref.tab = reinterpret_cast<const S4Args *>(tb + gl.tab_off);
                    ref.boff = reinterpret_cast<const int *>(tb + gl.boff_off);
                    ref.nsys = gl.nsys;
                    ref.total = gl.total;
                    if (prec == MODE_F64) rc = launch_s4<MODE_F64>(st, gl.cls_a, grid, ref);
                    else rc = launch_s4<MODE_F32>(st, gl.cls_a, grid, ref);
                }
            }
        }
        for (int s = 0; s < ns && rc == GF2_OK; ++s) {
            auto &p = plans[s];
            if (r * p.sh.b < p.ntau) rc = plan_reduce(p, st, r * p.sh.b, std::min(p.sh.b, p.ntau - r * p.sh.b));
        }
    }
    const hipError_t ec = hipStreamEndCapture(st, &graph);
    if (rc != GF2_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc;
    }
    GF2_HIP(ec);
    hipGraphExec_t exec = nullptr;
    const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    GF2_HIP(ei);
    lead->sig_graph = exec;
    lead->sig_key = key;
    GF2_HIP(hipGraphLaunch(exec, lead->stream));
    return GF2_OK;
}

void sigma_release(gf2_ctx *c) {
    if (c->sig_graph) {
        (void)hipGraphExecDestroy(static_cast<hipGraphExec_t>(c->sig_graph));
        c->sig_graph = nullptr;
        c->sig_key = 0;
    }
}

}  // namespace gf2

using namespace gf2;

extern "C" int gf2_sigma_tau(gf2_ctx *c, const gf2_dims *d, int prec, const double *G_tau,
                             double *Sigma_tau) {
    if (!c || !d || !G_tau || !Sigma_tau) return fail(GF2_EINVAL, "gf2_sigma_tau: NULL argument");
    if (!c->has_system) return fail(GF2_ESTATE, "gf2_sigma_tau: no system set");
    if (d->n != c->n) return fail(GF2_EINVAL, "gf2_sigma_tau: dims->n differs from the system");
    if (d->ntau < 4) return fail(GF2_EINVAL, "gf2_sigma_tau: ntau must be >= 4");
    if (prec < GF2_PREC_FP64 || prec > GF2_PREC_BF16MIX)
        return fail(GF2_EINVAL, "gf2_sigma_tau: bad precision");
    if ((const void *)G_tau == (const void *)Sigma_tau)
        return fail(GF2_EINVAL, "gf2_sigma_tau: Sigma_tau aliases G_tau");
    GF2_HIP(hipSetDevice(c->device));
    GF2_TRY(sigma_run(c, d, prec, G_tau, Sigma_tau));
    int bad = 0;
    GF2_TRY(any_nonfinite(c, (size_t)d->ntau * d->n * d->n, Sigma_tau, &bad));
    if (bad) return fail(GF2_ENONFINITE, "gf2_sigma_tau: non-finite self-energy");
    return GF2_OK;
}
