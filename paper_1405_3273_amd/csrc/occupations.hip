// Natural occupation numbers of the correlated density.
//
// The paper reports the natural occupation numbers (NONs) of the
// self-consistent density (Results: the H32 lattice and its figure of NONs
// against the lattice parameter; Supplementary Material, NON plots) without
// a formula.  Here they are the eigenvalues of the spin-summed density in the
// symmetrically orthonormalised basis, S^{1/2} P S^{1/2}, which has the same
// spectrum as P S and as L^T P L for the Cholesky factor S = L L^T.
//
// Three steps, all FP64 on the device:
//   1. S = L L^T (one workgroup, column by column; one wave per row dot);
//   2. A = L^T (P L) (two small products);
//   3. the eigenvalues of the symmetric A by the two-sided cyclic Jacobi
//      method in parallel round-robin order: each round rotates n/2 disjoint
//      index pairs at once (columns, barrier, rows, barrier), a sweep is
//      n - 1 rounds and every pair meets once per sweep.  A pair is rotated
//      when |a_pq| > max(n eps sqrt|a_pp a_qq|, eps ||A||_F); the method stops
//      after a sweep without rotations.  One workgroup; A sits in LDS up to
//      n = OC_LDS_MAXN, else in the workspace (global memory, through L2).
// The eigenvalues are written largest first.

#include "gf2_internal.h"

namespace gf2 {

constexpr int OC_THREADS = 1024;
constexpr int OC_MAXN = 1024;
constexpr int OC_LDS_MAXN = 136;       // n^2 doubles in LDS next to the static arrays
constexpr int OC_MAX_SWEEPS = 60;

// status bits
enum { OC_NOT_PD = 1, OC_NOCONV = 2, OC_NONFINITE = 4 };

__device__ __forceinline__ double wave_sum_d(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

// S = L L^T with L lower triangular; L and Lt = L^T are written in full
// (zeros outside the triangle).  status[0] is cleared here and gets
// OC_NOT_PD when a pivot is not positive (S not positive definite).
__global__ __launch_bounds__(OC_THREADS) void k_cholesky(int n, const double *__restrict__ S,
                                                          double *__restrict__ L,
                                                          double *__restrict__ Lt,
                                                          int *__restrict__ status) {
    __shared__ double col[OC_MAXN];
    const int tid = threadIdx.x, nth = blockDim.x;
    const int lane = tid & 63, wv = tid >> 6, nw = nth >> 6;
    const size_t n2 = (size_t)n * n;
    if (tid == 0) status[0] = 0;
    for (size_t e = tid; e < n2; e += nth) {
        L[e] = 0.0;
        Lt[e] = 0.0;
    }
    __syncthreads();
    for (int j = 0; j < n; ++j) {
        // col[i] = S_ij - sum_{k<j} L_ik L_jk   (i >= j)
        for (int i = j + wv; i < n; i += nw) {
            double acc = 0.0;
            for (int k = lane; k < j; k += 64) acc += L[(size_t)i * n + k] * L[(size_t)j * n + k];
            acc = wave_sum_d(acc);
            if (lane == 0) col[i] = S[(size_t)i * n + j] - acc;
        }
        __syncthreads();
        const double d2 = col[j];
        if (!(d2 > 0.0)) {          // uniform: every thread reads the same value
            if (tid == 0) status[0] = OC_NOT_PD;
            return;
        }
        const double d = sqrt(d2);
        for (int i = j + tid; i < n; i += nth) {
            const double v = (i == j) ? d : col[i] / d;
            L[(size_t)i * n + j] = v;
            Lt[(size_t)j * n + i] = v;
        }
        __syncthreads();
    }
}

// Index pair t of round r of the round-robin order over m (even) indices:
// index m - 1 stays, the others turn one place per round.
__device__ __forceinline__ void rr_pair(int r, int t, int m, int &p, int &q) {
    if (t == 0) {
        p = r;
        q = m - 1;
    } else {
        p = (r + t) % (m - 1);
        q = (r - t + (m - 1)) % (m - 1);
    }
}

__device__ double block_sum(double v, double *red) {
    v = wave_sum_d(v);
    const int tid = threadIdx.x;
    if ((tid & 63) == 0) red[tid >> 6] = v;
    __syncthreads();
    double s = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += red[w];
    __syncthreads();
    return s;
}

// Eigenvalues of the symmetric A (n x n, row-major, overwritten when it is
// not copied to LDS), largest first, into occ[n]; status bits OC_NOCONV,
// OC_NONFINITE are added to status[0].
__global__ __launch_bounds__(OC_THREADS) void k_jacobi(int n, double *__restrict__ Ag, int use_lds,
                                                        double *__restrict__ occ,
                                                        int *__restrict__ status) {
    extern __shared__ double shA[];
    __shared__ double sc[OC_MAXN / 2], ss[OC_MAXN / 2];
    __shared__ double red[OC_THREADS / 64];
    __shared__ int nrot;
    const int tid = threadIdx.x, nth = blockDim.x;
    const size_t n2 = (size_t)n * n;
    double *A = use_lds ? shA : Ag;
    if (use_lds)
        for (size_t e = tid; e < n2; e += nth) shA[e] = Ag[e];
    __syncthreads();

    double f = 0.0;
    for (size_t e = tid; e < n2; e += nth) f += A[e] * A[e];
    const double eps = 0x1p-52;
    const double anorm = sqrt(block_sum(f, red));
    const double rel = (double)n * eps, absthr = eps * anorm;

    const int m = n + (n & 1), np = m / 2;
    int sweep = 0;
    for (; sweep < OC_MAX_SWEEPS; ++sweep) {
        if (tid == 0) nrot = 0;
        __syncthreads();
        int mine = 0;
        for (int r = 0; r < m - 1; ++r) {
            for (int t = tid; t < np; t += nth) {
                int p, q;
                rr_pair(r, t, m, p, q);
                double c = 1.0, s = 0.0;
                if (p < n && q < n) {
                    const double apq = A[(size_t)p * n + q];
                    const double app = A[(size_t)p * n + p], aqq = A[(size_t)q * n + q];
                    if (fabs(apq) > fmax(rel * sqrt(fabs(app * aqq)), absthr)) {
                        // tan of the angle that zeroes a_pq, the root of
                        // t^2 + 2 theta t - 1 = 0 of modulus <= 1
                        const double th = (app - aqq) / (2.0 * apq);
                        const double tn = -copysign(1.0, th) / (fabs(th) + sqrt(fma(th, th, 1.0)));
                        c = 1.0 / sqrt(fma(tn, tn, 1.0));
                        s = tn * c;
                        ++mine;
                    }
                }
                sc[t] = c;
                ss[t] = s;
            }
            __syncthreads();
            // A <- A J: columns p, q of every row k
            for (int idx = tid; idx < np * n; idx += nth) {
                const int t = idx / n, k = idx - t * n;
                const double s = ss[t];
                if (s == 0.0) continue;
                const double c = sc[t];
                int p, q;
                rr_pair(r, t, m, p, q);
                double *row = A + (size_t)k * n;
                const double akp = row[p], akq = row[q];
                row[p] = c * akp - s * akq;
                row[q] = s * akp + c * akq;
            }
            __syncthreads();
            // A <- J^T A: rows p, q of every column k
            for (int idx = tid; idx < np * n; idx += nth) {
                const int t = idx / n, k = idx - t * n;
                const double s = ss[t];
                if (s == 0.0) continue;
                const double c = sc[t];
                int p, q;
                rr_pair(r, t, m, p, q);
                const double apk = A[(size_t)p * n + k], aqk = A[(size_t)q * n + k];
                A[(size_t)p * n + k] = c * apk - s * aqk;
                A[(size_t)q * n + k] = s * apk + c * aqk;
            }
            __syncthreads();
        }
        if (mine) atomicAdd(&nrot, mine);
        __syncthreads();
        const int done = (nrot == 0);
        __syncthreads();            // every thread has read nrot before it is cleared
        if (done) break;
    }
    if (tid == 0 && sweep == OC_MAX_SWEEPS) atomicOr(status, (int)OC_NOCONV);

    // largest first: rank = #{larger} + #{equal with a smaller index}
    for (int i = tid; i < n; i += nth) {
        const double di = A[(size_t)i * n + i];
        if (!isfinite(di)) atomicOr(status, (int)OC_NONFINITE);
        int rank = 0;
        for (int j = 0; j < n; ++j) {
            const double dj = A[(size_t)j * n + j];
            rank += (dj > di) | ((dj == di) & (j < i));
        }
        occ[min(rank, n - 1)] = di;
    }
}

int occupations_run(gf2_ctx *c, const double *P, double *occ) {
    const int n = c->n;
    const size_t n2 = (size_t)n * n;
    GF2_TRY(c->occ_ws.ensure(4 * n2 * sizeof(double) + 256));
    double *L = c->occ_ws.as<double>();
    double *Lt = L + n2, *T = Lt + n2, *A = T + n2;
    int *status = reinterpret_cast<int *>(A + n2);
    const int ph = prof_begin(c, GF2_KC_OCCUPATIONS);
    hipLaunchKernelGGL(k_cholesky, dim3(1), dim3(OC_THREADS), 0, c->stream, n, c->S.as<double>(), L,
                       Lt, status);
    GF2_HIP(hipGetLastError());
    GF2_TRY(matmul_nn(c, n, P, L, T));
    GF2_TRY(matmul_nn(c, n, Lt, T, A));
    const int use_lds = n <= OC_LDS_MAXN;
    const size_t shm = use_lds ? n2 * sizeof(double) : 0;
    if (shm > 0)
        GF2_HIP(hipFuncSetAttribute((const void *)k_jacobi,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm));
    hipLaunchKernelGGL(k_jacobi, dim3(1), dim3(OC_THREADS), shm, c->stream, n, A, use_lds, occ,
                       status);
    GF2_HIP(hipGetLastError());
    prof_end(c, ph, (double)n);
    int st = 0;
    GF2_HIP(hipMemcpyAsync(&st, status, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    GF2_HIP(hipStreamSynchronize(c->stream));
    if (st & OC_NOT_PD)
        return fail(GF2_EINVAL, "gf2_natural_occupations: the overlap S is not positive definite");
    if (st & OC_NONFINITE)
        return fail(GF2_ENONFINITE, "gf2_natural_occupations: non-finite eigenvalue (NaN/Inf in P?)");
    if (st & OC_NOCONV)
        return fail(GF2_ENOCONV, "gf2_natural_occupations: Jacobi sweeps did not converge");
    return GF2_OK;
}

}  // namespace gf2

using namespace gf2;

extern "C" int gf2_natural_occupations(gf2_ctx *c, const double *P, double *occ) {
    if (!c || !P || !occ) return fail(GF2_EINVAL, "gf2_natural_occupations: NULL argument");
    if (!c->has_system) return fail(GF2_ESTATE, "gf2_natural_occupations: no system set");
    if (c->n > OC_MAXN)
        return fail(GF2_EINVAL, "gf2_natural_occupations: n above " + std::to_string(OC_MAXN));
    GF2_HIP(hipSetDevice(c->device));
    return occupations_run(c, P, occ);
}
