// Internal declarations of libgf2 (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "gf2.h"

namespace gf2 {

// ---- errors ---------------------------------------------------------------
void set_error(const std::string &msg);
int fail(int code, const std::string &msg);
int hip_fail(hipError_t e, const char *what, const char *file, int line);

#define GF2_HIP(call)                                                        \
    do {                                                                     \
        hipError_t e_ = (call);                                              \
        if (e_ != hipSuccess) return ::gf2::hip_fail(e_, #call, __FILE__, __LINE__); \
    } while (0)

#define GF2_TRY(call)                                                        \
    do {                                                                     \
        int rc_ = (call);                                                    \
        if (rc_ != GF2_OK) return rc_;                                       \
    } while (0)

// ---- device buffers ---------------------------------------------------------
// Grow-only device allocation owned by the context.
struct DevBuf {
    void *ptr = nullptr;
    size_t bytes = 0;
    int ensure(size_t need);
    void release();
    template <class T> T *as() const { return static_cast<T *>(ptr); }
};

// Sigma(tau) arithmetic modes (match GF2_PREC_*).
enum { MODE_F64 = 0, MODE_F32 = 1, MODE_BF3 = 2, MODE_BF6 = 3, MODE_BFM = 4 };
// Global-memory pointers in kernels.  Pointers read from argument structs are
// generic, for which the compiler emits flat loads and stores; flat accesses
// also count against the LDS wait counter, so every wait for an LDS access
// would wait for the global loads and stores in flight too.  The hot operand
// streams are therefore addressed through address-space-1 pointers.
#define GF2_GLOBAL __attribute__((address_space(1)))

// Per-stage arithmetic of the Sigma(tau) contraction.  split_planes: bf16
// planes of the first transform's output T1 (0: T1 is FP32/FP64);
// s23_planes: planes per operand in the fused second and third transforms
// (0: the FP32/FP64 MFMA kernel); s4_planes: the same for the final
// contraction; s1_mode: the mode of the first transform's kernel.  The mixed
// mode runs the first transform in FP32 MFMA (T1 stays FP32 and is split in
// registers where it is read), the second and third in the three-term split
// and the final contraction in the two-term split.
constexpr int split_planes(int mode) { return mode == MODE_BF3 ? 2 : mode == MODE_BF6 ? 3 : 0; }
constexpr int s23_planes(int mode) { return mode == MODE_BFM ? 3 : split_planes(mode); }
constexpr int s4_planes(int mode) { return mode == MODE_BFM ? 2 : split_planes(mode); }
constexpr int s1_mode(int mode) { return mode == MODE_BFM ? MODE_F32 : mode; }

}  // namespace gf2

struct gf2_prof_pending {
    int cls;
    hipEvent_t start, stop;
    double work;
};

struct gf2_ctx {
    int device = 0;
    hipStream_t stream = nullptr;

    // ---- opt-in kernel timing ----
    bool prof = false;
    double prof_ms[GF2_KC_COUNT] = {0};
    long long prof_n[GF2_KC_COUNT] = {0};
    double prof_work[GF2_KC_COUNT] = {0};
    std::vector<gf2_prof_pending> prof_pending;
    std::vector<hipEvent_t> prof_pool;

    // ---- system (gf2_set_system) ----
    int n = 0;
    bool has_system = false;
    gf2::DevBuf S, Sinv, h, v;            // FP64
    std::vector<double> S_host, Sinv_host, h_host;

    // Layouts for the Sigma contraction, built once per system:
    //   v_32           FP32 copy of v (first index transform, FP32 and BF16x3)
    //   W2[n][p][l][j] = 2 v_lpnj - v_nplj   (final contraction; FP64 and FP32)
    //   W2_b3          W2 as bf16 hi/lo planes in the final contraction's K order
    gf2::DevBuf v_32, W2_64, W2_32, W2_b3;
    bool have_f32_layouts = false;
    bool have_bf3_layouts = false;

    // ---- workspaces (grow-only) ----
    gf2::DevBuf sig_T1, sig_X, sig_G, sig_Gb, sig_Gp, sig_Gq, sig_part;
    gf2::DevBuf four_c, four_C, four_fold, four_twid;
    gf2::DevBuf dys_part, dys_X, dys_aux, dys_out;
    gf2::DevBuf fock_part;
    gf2::DevBuf occ_ws;                   // natural occupations: L, L^T, P L, A, status
    // non-equidistant tau grid (gf2_set_tau_grid); grid_ntau == 0: uniform grid
    int grid_ntau = 0;
    std::vector<double> grid_host;
    gf2::DevBuf grid_tau, grid_thom;      // tau_k; Thomas factors of the spline system
    gf2::DevBuf grid_W, grid_T;           // tau->iw weights, iw->tau cos/sin table
    int grid_w_niw = 0, grid_t_niw = 0;   // niw the tables were built for
    double grid_w_beta = 0.0, grid_t_beta = 0.0;
    gf2::DevBuf grid_coef, grid_plan;     // spline coefficients; planar [2 niw][n n] work
    gf2::DevBuf it_Sig_iw, it_G_iw, it_Sig1, it_mom, it_Sig_new, it_Pout, it_Pin, it_F, it_tmp;
    gf2::DevBuf it_hist;                  // Pulay history on the device: [2*depth][n][n]
    gf2::DevBuf it_red;                   // inner-loop reduction results
    gf2::DevBuf bat_red;                  // the same for every system of a batch
    void *bat_red_h = nullptr;            // pinned copy of bat_red
    size_t bat_red_h_bytes = 0;
    // batched sweeps (gf2_iterate_batched, owned by the first context of the batch)
    gf2::DevBuf bat_tab, bat_boff, bat_out;
    void *bat_host = nullptr;             // pinned staging (hipHostMalloc)
    size_t bat_host_bytes = 0;
    void *bat_graph = nullptr;            // hipGraphExec_t of the Dyson round
    hipStream_t bat_cap = nullptr;        // private stream the round is captured on
    gf2::DevBuf sig_tab;                  // argument tables of the batched Sigma launches
    void *sig_graph = nullptr;            // hipGraphExec_t of the batched Sigma
    long long sig_key = 0;
    long long bat_key = 0;                // shape the graph was captured for

    // ---- density-fitting factors (gf2_set_df_factors) ----
    int df_m = 0;                         // auxiliary functions (0: none set)
    gf2::DevBuf df_B64, df_Bt64;          // B[P][a][b], Bt[a][P][b] (FP64)
    gf2::DevBuf df_B32, df_Bt32;          // the same in FP32
    gf2::DevBuf df_ws, df_T, df_part;     // chain intermediates, exchange products, split-K partials
};

namespace gf2 {

// ---- opt-in kernel timing (common.hip) ----------------------------------------
// prof_begin records a start event for class cls (returns a handle, -1 when
// profiling is off); prof_end records the stop event and the launch's work.
int prof_begin(gf2_ctx *c, int cls);
void prof_end(gf2_ctx *c, int handle, double work);
void prof_release(gf2_ctx *c);

// ---- small shared kernels (common.hip) ---------------------------------------
int copy_d2d(gf2_ctx *c, void *dst, const void *src, size_t bytes);
int fill_zero(gf2_ctx *c, void *dst, size_t bytes);
// y = a*x + b*y, n doubles
int axpby(gf2_ctx *c, size_t n, double a, const double *x, double b, double *y);
// max |a - b| over n doubles (host result; synchronises)
int max_abs_diff(gf2_ctx *c, size_t n, const double *a, const double *b, double *out);
// 1 if any element of x[n] is not finite (host result; synchronises)
int any_nonfinite(gf2_ctx *c, size_t n, const double *x, int *out);
// out = sum_i a_i * b_i (host result; synchronises)
int dot(gf2_ctx *c, size_t n, const double *a, const double *b, double *out);
// small dense matmul on the device: C = A * B (n x n FP64)
int matmul_nn(gf2_ctx *c, int n, const double *A, const double *B, double *C);

// Plain FP64 GEMM on MFMA: C[m*ldc + n] = alpha * sum_k A[k*lda + m] B[k*ldb + n]
struct GemmArgsF64 {
    const double *A; long long lda;
    const double *B; long long ldb;
    double *C; long long ldc;
    int M, N, K;
    double alpha;
};
int gemm_f64_kmajor(gf2_ctx *c, const GemmArgsF64 &a);

// ---- stages ---------------------------------------------------------------------
int sigma_build_layouts(gf2_ctx *c, bool want_f32);
int sigma_run(gf2_ctx *c, const gf2_dims *d, int prec, const double *G_tau, double *Sigma_tau);
// Sigma(tau) of many systems (one lead context runs the captured graph)
int sigma_run_batched(gf2_ctx *lead, const std::vector<gf2_ctx *> &cs, const std::vector<int> &ntau,
                      int prec, const std::vector<const double *> &G,
                      const std::vector<double *> &Sig);
void sigma_release(gf2_ctx *c);
// density-fitted Sigma(tau) from the context's factors (prec FP64 or FP32)
int sigma_df_run(gf2_ctx *c, const gf2_dims *d, int prec, const double *G_tau, double *Sigma_tau);

int fourier_tau2iw(gf2_ctx *c, const gf2_dims *d, const double *Sig_tau, double2 *Sig_iw,
                   double *Sig1);
int fourier_iw2tau(gf2_ctx *c, const gf2_dims *d, const double2 *G_iw, const double *mom,
                   double *G_tau);

// Dyson over all frequencies.  mode = GF2_DYSON_*.  out[0] = tr(PS),
// out[1] = E_2b (ENERGY).  If mom_out != NULL the tail moments G1,G2,G3
// of this (mu, F, Sigma_1) are written there ([3][n][n]).  trace_n (may be
// NULL): tr(PS) by the formula of the TRACE mode, bitwise what a TRACE solve
// at the same mu returns, in every mode.
int dyson_run(gf2_ctx *c, const gf2_dims *d, int mode, double mu, const double *F,
              const double2 *Sig_iw, const double *Sig1, double2 *G_iw, double *P,
              double *mom_out, double *out, double *trace_n = nullptr);

int fock_run(gf2_ctx *c, const double *P, double *F);

// One round of Dyson solves for several systems (batched driver).  Job s:
// mode (GF2_DYSON_*, or -1 to skip), mu, F, Sigma(i w), Sigma_1, and for
// FULL/ENERGY the outputs G(i w), P and the tail moments.  res[3 s + 0..1] as
// the out[] of dyson_run, res[3 s + 2] as its trace_n.  All systems run on lead->stream.
struct DysonReq {
    gf2_ctx *c;
    const gf2_dims *d;
    int mode;
    double mu;
    const double *F;
    const double2 *Sig;
    const double *Sig1;
    double2 *G_iw;
    double *P;
    double *mom;        // FULL/ENERGY: tail moments written here ([3][n][n])
};
int dyson_round(gf2_ctx *lead, const std::vector<DysonReq> &req, std::vector<double> &res);
void dyson_round_release(gf2_ctx *lead);

// trigamma(x) for x > 0 (host)
double trigamma(double x);

}  // namespace gf2
