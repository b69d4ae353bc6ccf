// Eq. (Sigma): the second-order self-energy in imaginary time on MFMA.
//
// For every tau point (A = G(tau), B = G(-tau) = -G(beta - tau)) the six-index
// sum is evaluated as four index transforms, each a GEMM with one large
// dimension (cost 2 N^5 each, 8 N^5 per tau):
//
//   S1  T1[q][k][i][n] = sum_m V1[m][q][k][i] A[m][n]       V1[m][q][k][i] = v_imqk
//   S2  T2[k][i][n][p] = sum_q T1[q][k][i][n] B[q][p]
//   S3  X [i][n][p][l] = sum_k T2[k][i][n][p] A[k][l]
//   S4  Sigma[i][j]    = - sum_{n,p,l} X[i][n][p][l] W2[n][p][l][j]
//                                                           W2[n][p][l][j] = 2 v_lpnj - v_nplj
//
// S1-S3 have the form C[r][c] = sum_a T[a][r] M[a][c] with r running over
// N^3 rows; S4 is a split-K GEMM with K = N^3 whose partial sums are added
// in FP64 in a fixed order.  Several tau points run in one launch (grid z,
// and stacked rows in S4).  G is symmetric, so A and B are used as stored.
//
// Arithmetic: FP64 MFMA (v_mfma_f64_16x16x4f64), FP32 MFMA
// (v_mfma_f32_16x16x4f32), or BF16x3: each FP32 operand x is split into
// hi = bf16(x), lo = bf16(x - hi) when it is staged into LDS, and
// a*b ~ hi_a*lo_b + lo_a*hi_b + hi_a*hi_b on v_mfma_f32_16x16x32_bf16 with
// FP32 accumulation.  In S4 the FP32 accumulators are flushed into FP64
// registers every 512 K elements.
#include "gf2_internal.h"

#include <algorithm>
#include <cstring>

namespace gf2 {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef double v4d __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef unsigned short v8us __attribute__((ext_vector_type(8)));

template <int MODE> struct ModeT;
template <> struct ModeT<MODE_F64> { using in_t = double; using acc_t = v4d; static constexpr int BK = 16; };
template <> struct ModeT<MODE_F32> { using in_t = float;  using acc_t = v4f; static constexpr int BK = 16; };
template <> struct ModeT<MODE_BF3> { using in_t = float;  using acc_t = v4f; static constexpr int BK = 32; };

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
};

constexpr int NTHREADS = 256;
constexpr int BM = 128;  // 4 waves x 2 row tiles x 16
constexpr int RT = 2;    // row tiles per wave

__device__ __forceinline__ unsigned short bf16_rne(float x) {
    unsigned int u = __float_as_uint(x);
    unsigned int r = u + 0x7FFFu + ((u >> 16) & 1u);
    return (unsigned short)(r >> 16);
}
__device__ __forceinline__ float bf16_to_f(unsigned short h) {
    return __uint_as_float(((unsigned int)h) << 16);
}
__device__ __forceinline__ void split_bf16(float x, unsigned short &hi, unsigned short &lo) {
    hi = bf16_rne(x);
    lo = bf16_rne(x - bf16_to_f(hi));
}

template <class T> __device__ __forceinline__ T ldg(const T *p) { return *p; }

// ---------------------------------------------------------------------------
// FP64 / FP32 kernel: LDS tiles As[k][m], Bs[k][n]
template <int MODE, bool AK, int NT>
__global__ __launch_bounds__(NTHREADS) void gemm_fp(GemmArgs g) {
    using in_t = typename ModeT<MODE>::in_t;
    using acc_t = typename ModeT<MODE>::acc_t;
    constexpr int BK = ModeT<MODE>::BK;
    constexpr int BN = 16 * NT;
    constexpr int SA = BM + 16;                       // padded row strides
    constexpr int SB = BN + ((16 - BN % 32) + 32) % 32;
    constexpr bool OUT64 = !AK || MODE == MODE_F64;   // S4 writes FP64 partials
    constexpr int FLUSH = 512 / BK;                   // chunks between FP64 flushes

    __shared__ in_t As[BK][SA];
    __shared__ in_t Bs[BK][SB];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int z = blockIdx.z;
    const long long mb = (long long)blockIdx.x * BM;
    const int nb = blockIdx.y * BN;

    const in_t *A = static_cast<const in_t *>(g.A) + (long long)z * g.sA;
    const in_t *B = static_cast<const in_t *>(g.B) + (long long)z * g.sB;
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
            const in_t *p = A + gk * g.lda + gm;
            if (gk < Kz && gm + A_PER <= g.M && g.vecA) {
                if constexpr (MODE == MODE_F64) {
#pragma unroll
                    for (int e = 0; e < A_PER; e += 2) {
                        double2 t = *reinterpret_cast<const double2 *>(p + e);
                        ra[e] = t.x;
                        ra[e + 1] = t.y;
                    }
                } else {
#pragma unroll
                    for (int e = 0; e < A_PER; e += 4) {
                        float4 t = *reinterpret_cast<const float4 *>(p + e);
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
                        static_cast<double *>(g.C)[(long long)z * g.sC + m * g.ldc + n] = g.alpha * val;
                    } else {
                        static_cast<in_t *>(g.C)[(long long)z * g.sC + m * g.ldc + n] =
                            (in_t)(g.alpha * (double)acc[r][c][e]);
                    }
                }
            }
}

// ---------------------------------------------------------------------------
// BF16x3 kernel: FP32 operands split into hi/lo BF16 in LDS, tiles As[m][k], Bs[n][k]
template <bool AK, int NT>
__global__ __launch_bounds__(NTHREADS) void gemm_bf3(GemmArgs g) {
    constexpr int BK = 32;
    constexpr int BN = 16 * NT;
    constexpr int SK = BK + 8;       // padded k stride (bf16 elements)
    constexpr bool OUT64 = !AK;
    constexpr int FLUSH = 512 / BK;

    __shared__ __attribute__((aligned(16))) unsigned short Ah[BM][SK];
    __shared__ __attribute__((aligned(16))) unsigned short Al[BM][SK];
    __shared__ __attribute__((aligned(16))) unsigned short Bh[BN][SK];
    __shared__ __attribute__((aligned(16))) unsigned short Bl[BN][SK];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int z = blockIdx.z;
    const long long mb = (long long)blockIdx.x * BM;
    const int nb = blockIdx.y * BN;

    const float *A = static_cast<const float *>(g.A) + (long long)z * g.sA;
    const float *B = static_cast<const float *>(g.B) + (long long)z * g.sB;
    const int Kz = g.split ? min(g.kz, g.K - z * g.kz) : g.K;
    if (Kz <= 0) return;

    v4f acc[RT][NT];
    double accd[RT][NT][4];
#pragma unroll
    for (int r = 0; r < RT; ++r)
#pragma unroll
        for (int c = 0; c < NT; ++c) {
            acc[r][c] = v4f{0, 0, 0, 0};
#pragma unroll
            for (int e = 0; e < 4; ++e) accd[r][c][e] = 0.0;
        }

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
            const float *p = A + gm * g.lda + gk;
            if (gm < g.M && gk + 16 <= Kz && g.vecA) {
#pragma unroll
                for (int e = 0; e < 16; e += 4) {
                    float4 t = *reinterpret_cast<const float4 *>(p + e);
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
            v8us hi, lo;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                unsigned short a, b;
                split_bf16(ra[h * 8 + e], a, b);
                hi[e] = a;
                lo[e] = b;
            }
            *reinterpret_cast<v8us *>(&Ah[a_m][a_k0 + h * 8]) = hi;
            *reinterpret_cast<v8us *>(&Al[a_m][a_k0 + h * 8]) = lo;
        }
#pragma unroll
        for (int it = 0; it < B_ITERS; ++it) {
            const int grp = tid + it * NTHREADS;
            if (grp < BG) {
                const int n = grp % BN, kg = grp / BN;
                v8us hi, lo;
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    unsigned short a, b;
                    split_bf16(rb[it][e], a, b);
                    hi[e] = a;
                    lo[e] = b;
                }
                *reinterpret_cast<v8us *>(&Bh[n][kg * 8]) = hi;
                *reinterpret_cast<v8us *>(&Bl[n][kg * 8]) = lo;
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
        v8bf ah[RT], al[RT];
#pragma unroll
        for (int r = 0; r < RT; ++r) {
            const int m = wave * (16 * RT) + r * 16 + (lane & 15);
            ah[r] = __builtin_bit_cast(v8bf, *reinterpret_cast<const v8us *>(&Ah[m][kq]));
            al[r] = __builtin_bit_cast(v8bf, *reinterpret_cast<const v8us *>(&Al[m][kq]));
        }
#pragma unroll
        for (int c = 0; c < NT; ++c) {
            const int n = c * 16 + (lane & 15);
            v8bf bh = __builtin_bit_cast(v8bf, *reinterpret_cast<const v8us *>(&Bh[n][kq]));
            v8bf bl = __builtin_bit_cast(v8bf, *reinterpret_cast<const v8us *>(&Bl[n][kq]));
#pragma unroll
            for (int r = 0; r < RT; ++r) {
                acc[r][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[r], bl, acc[r][c], 0, 0, 0);
                acc[r][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[r], bh, acc[r][c], 0, 0, 0);
                acc[r][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[r], bh, acc[r][c], 0, 0, 0);
            }
        }
        if constexpr (OUT64) {
            if ((ch + 1) % FLUSH == 0 || ch + 1 == nchunks) {
#pragma unroll
                for (int r = 0; r < RT; ++r)
#pragma unroll
                    for (int c = 0; c < NT; ++c) {
#pragma unroll
                        for (int e = 0; e < 4; ++e) accd[r][c][e] += (double)acc[r][c][e];
                        acc[r][c] = v4f{0, 0, 0, 0};
                    }
            }
        }
    }

#pragma unroll
    for (int r = 0; r < RT; ++r)
#pragma unroll
        for (int c = 0; c < NT; ++c)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const long long m = mb + wave * (16 * RT) + r * 16 + 4 * (lane >> 4) + e;
                const int n = nb + c * 16 + (lane & 15);
                if (m < g.M && n < g.N) {
                    if constexpr (OUT64)
                        static_cast<double *>(g.C)[(long long)z * g.sC + m * g.ldc + n] =
                            g.alpha * accd[r][c][e];
                    else
                        static_cast<float *>(g.C)[(long long)z * g.sC + m * g.ldc + n] =
                            (float)(g.alpha * (double)acc[r][c][e]);
                }
            }
}

// ---------------------------------------------------------------------------
// host-side dispatch

template <int MODE, bool AK>
static void launch_nt(int nt, dim3 grid, hipStream_t s, const GemmArgs &g) {
#define GF2_NT_CASE(T)                                                              \
    case T:                                                                         \
        if constexpr (MODE == MODE_BF3)                                             \
            hipLaunchKernelGGL((gemm_bf3<AK, T>), grid, dim3(NTHREADS), 0, s, g);  \
        else                                                                        \
            hipLaunchKernelGGL((gemm_fp<MODE, AK, T>), grid, dim3(NTHREADS), 0, s, g); \
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

static int gemm(gf2_ctx *c, int mode, bool ak, GemmArgs g, int zcount) {
    int nt, nblk;
    col_blocking(g.N, nt, nblk);
    dim3 grid((unsigned)((g.M + BM - 1) / BM), (unsigned)nblk, (unsigned)zcount);
    if (mode == MODE_F64) {
        if (ak) launch_nt<MODE_F64, true>(nt, grid, c->stream, g);
        else launch_nt<MODE_F64, false>(nt, grid, c->stream, g);
    } else if (mode == MODE_F32) {
        if (ak) launch_nt<MODE_F32, true>(nt, grid, c->stream, g);
        else launch_nt<MODE_F32, false>(nt, grid, c->stream, g);
    } else {
        if (ak) launch_nt<MODE_BF3, true>(nt, grid, c->stream, g);
        else launch_nt<MODE_BF3, false>(nt, grid, c->stream, g);
    }
    GF2_HIP(hipGetLastError());
    return GF2_OK;
}

int gemm_f64_kmajor(gf2_ctx *c, const GemmArgsF64 &a) {
    GemmArgs g{};
    g.A = a.A; g.lda = a.lda; g.sA = 0;
    g.B = a.B; g.ldb = a.ldb; g.sB = 0;
    g.C = a.C; g.ldc = a.ldc; g.sC = 0;
    g.M = a.M; g.N = a.N; g.K = a.K; g.kz = a.K; g.split = 0;
    g.alpha = a.alpha;
    g.vecA = (a.lda % 2 == 0) ? 1 : 0;
    return gemm(c, MODE_F64, true, g, 1);
}

// ---------------------------------------------------------------------------
// layouts of v (built once per system)

template <class T>
__global__ void k_build_layouts(int n, const double *__restrict__ v, T *__restrict__ V1,
                                T *__restrict__ W2) {
    const size_t n2 = (size_t)n * n, n3 = n2 * n, n4 = n3 * n;
    for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < n4;
         idx += (size_t)gridDim.x * blockDim.x) {
        // idx = ((a*n + b)*n + c)*n + d
        const size_t a = idx / n3, b = (idx / n2) % n, cc = (idx / n) % n, d = idx % n;
        // V1[m=a][q=b][k=cc][i=d] = v[i][m][q][k]
        V1[idx] = (T)v[((d * n + a) * n + b) * n + cc];
        // W2[n=a][p=b][l=cc][j=d] = 2 v[l][p][n][j] - v[n][p][l][j]
        W2[idx] = (T)(2.0 * v[((cc * n + b) * n + a) * n + d] - v[((a * n + b) * n + cc) * n + d]);
    }
}

int sigma_build_layouts(gf2_ctx *c, bool want_f32) {
    const size_t n = c->n, n4 = n * n * n * n;
    const unsigned blocks = (unsigned)std::min<size_t>((n4 + 255) / 256, 65536);
    GF2_TRY(c->V1_64.ensure(n4 * 8));
    GF2_TRY(c->W2_64.ensure(n4 * 8));
    hipLaunchKernelGGL(k_build_layouts<double>, dim3(blocks), dim3(256), 0, c->stream, (int)n,
                       c->v.as<double>(), c->V1_64.as<double>(), c->W2_64.as<double>());
    GF2_HIP(hipGetLastError());
    if (want_f32) {
        GF2_TRY(c->V1_32.ensure(n4 * 4));
        GF2_TRY(c->W2_32.ensure(n4 * 4));
        hipLaunchKernelGGL(k_build_layouts<float>, dim3(blocks), dim3(256), 0, c->stream, (int)n,
                           c->v.as<double>(), c->V1_32.as<float>(), c->W2_32.as<float>());
        GF2_HIP(hipGetLastError());
        c->have_f32_layouts = true;
    }
    return GF2_OK;
}

// ---------------------------------------------------------------------------
// per-batch staging and reduction

// Gs[t] = G(tau_{k0+t}), Gbs[t] = G(-tau_{k0+t}) = -G(tau_{M-k0-t})
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

// Sigma[k0 + t][i][j] = sum_z part[z][t*n + i][j]   (part already carries the minus sign)
__global__ void k_reduce_split(int n, int nb, int nsplit, const double *__restrict__ part,
                               double *__restrict__ Sig, int k0) {
    const size_t n2 = (size_t)n * n;
    const size_t total = n2 * nb;
    const size_t zs = total;  // partial stride: (nb*n) x n
    for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < total;
         idx += (size_t)gridDim.x * blockDim.x) {
        double s = 0.0;
        for (int z = 0; z < nsplit; ++z) s += part[z * zs + idx];
        Sig[(size_t)k0 * n2 + idx] = s;
    }
}

int sigma_run(gf2_ctx *c, const gf2_dims *d, int prec, const double *G_tau, double *Sigma_tau) {
    const int n = c->n;
    const int ntau = d->ntau;
    const int M = ntau - 1;
    const long long N = n, N2 = N * N, N3 = N2 * N, N4 = N3 * N;
    const int mode = prec;
    const size_t esz = (mode == MODE_F64) ? 8 : 4;
    if (mode != MODE_F64 && !c->have_f32_layouts) GF2_TRY(sigma_build_layouts(c, true));
    const void *V1 = (mode == MODE_F64) ? c->V1_64.ptr : c->V1_32.ptr;
    const void *W2 = (mode == MODE_F64) ? c->W2_64.ptr : c->W2_32.ptr;

    // tau batch: two intermediates of b*N^4 elements, capped at ~16 GB
    const size_t budget = (size_t)16 << 30;
    const size_t bmax = std::max<size_t>(1, budget / (2 * (size_t)N4 * esz));
    const int b = (int)std::min<size_t>(bmax, (size_t)std::min(ntau, 64));

    // split-K for S4: K = N^3 split into slices of kz (multiple of 512)
    long long kz = 4096;
    if (N3 < 8 * 4096) kz = std::max<long long>(512, ((N3 / 8) + 511) / 512 * 512);
    const int nsplit = (int)((N3 + kz - 1) / kz);

    GF2_TRY(c->sig_T1.ensure((size_t)b * N4 * esz));
    GF2_TRY(c->sig_T2.ensure((size_t)b * N4 * esz));
    GF2_TRY(c->sig_G.ensure((size_t)b * N2 * esz));
    GF2_TRY(c->sig_Gb.ensure((size_t)b * N2 * esz));
    GF2_TRY(c->sig_part.ensure((size_t)nsplit * b * N2 * 8));

    const bool vec = (N3 % 4 == 0);
    for (int k0 = 0; k0 < ntau; k0 += b) {
        const int nb = std::min(b, ntau - k0);
        {
            const size_t tot = (size_t)nb * N2;
            const unsigned blocks = (unsigned)std::min<size_t>((tot + 255) / 256, 4096);
            if (mode == MODE_F64)
                hipLaunchKernelGGL(k_stage_g<double>, dim3(blocks), dim3(256), 0, c->stream, n, M,
                                   k0, nb, G_tau, c->sig_G.as<double>(), c->sig_Gb.as<double>());
            else
                hipLaunchKernelGGL(k_stage_g<float>, dim3(blocks), dim3(256), 0, c->stream, n, M,
                                   k0, nb, G_tau, c->sig_G.as<float>(), c->sig_Gb.as<float>());
            GF2_HIP(hipGetLastError());
        }
        GemmArgs g{};
        g.M = (int)N3;
        g.N = n;
        g.K = n;
        g.kz = n;
        g.split = 0;
        g.alpha = 1.0;
        g.vecA = vec ? 1 : 0;
        g.lda = N3;
        g.ldb = N;
        g.ldc = N;
        g.sB = N2;
        g.sC = N4;
        const double stage_flops = 2.0 * (double)N4 * (double)N * nb;
        // S1: T1 = V1^T A   (A = G(tau))
        g.A = V1; g.sA = 0;
        g.B = c->sig_G.ptr;
        g.C = c->sig_T1.ptr;
        int ph = prof_begin(c, GF2_KC_SIGMA_GEMM);
        GF2_TRY(gemm(c, mode, true, g, nb));
        prof_end(c, ph, stage_flops);
        // S2: T2 = T1 x_q B   (B = G(-tau))
        g.A = c->sig_T1.ptr; g.sA = N4;
        g.B = c->sig_Gb.ptr;
        g.C = c->sig_T2.ptr;
        ph = prof_begin(c, GF2_KC_SIGMA_GEMM);
        GF2_TRY(gemm(c, mode, true, g, nb));
        prof_end(c, ph, stage_flops);
        // S3: X = T2 x_k A  (into T1)
        g.A = c->sig_T2.ptr; g.sA = N4;
        g.B = c->sig_G.ptr;
        g.C = c->sig_T1.ptr;
        ph = prof_begin(c, GF2_KC_SIGMA_GEMM);
        GF2_TRY(gemm(c, mode, true, g, nb));
        prof_end(c, ph, stage_flops);
        // S4: partial[z] = -X[(t,i)][K-slice z] W2[K-slice z][j]
        GemmArgs h{};
        h.A = c->sig_T1.ptr;
        h.lda = N3;
        h.sA = kz;
        h.B = W2;
        h.ldb = N;
        h.sB = kz * N;
        h.C = c->sig_part.ptr;
        h.ldc = N;
        h.sC = (long long)nb * N2;
        h.M = (int)(nb * N);
        h.N = n;
        h.K = (int)N3;
        h.kz = (int)kz;
        h.split = 1;
        h.alpha = -1.0;
        h.vecA = vec ? 1 : 0;
        ph = prof_begin(c, GF2_KC_SIGMA_SPLITK);
        GF2_TRY(gemm(c, mode, false, h, nsplit));
        prof_end(c, ph, stage_flops);
        {
            const size_t tot = (size_t)nb * N2;
            const unsigned blocks = (unsigned)std::min<size_t>((tot + 255) / 256, 4096);
            hipLaunchKernelGGL(k_reduce_split, dim3(blocks), dim3(256), 0, c->stream, n, nb,
                               nsplit, c->sig_part.as<double>(), Sigma_tau, k0);
            GF2_HIP(hipGetLastError());
        }
    }
    return GF2_OK;
}

}  // namespace gf2

using namespace gf2;

extern "C" int gf2_sigma_tau(gf2_ctx *c, const gf2_dims *d, int prec, const double *G_tau,
                             double *Sigma_tau) {
    if (!c || !d || !G_tau || !Sigma_tau) return fail(GF2_EINVAL, "gf2_sigma_tau: NULL argument");
    if (!c->has_system) return fail(GF2_ESTATE, "gf2_sigma_tau: no system set");
    if (d->n != c->n) return fail(GF2_EINVAL, "gf2_sigma_tau: dims->n differs from the system");
    if (d->ntau < 4) return fail(GF2_EINVAL, "gf2_sigma_tau: ntau must be >= 4");
    if (prec < GF2_PREC_FP64 || prec > GF2_PREC_BF16X3)
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
