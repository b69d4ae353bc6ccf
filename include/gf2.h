/*
 * gf2.h -- C ABI of libgf2, an MI355X (gfx950) implementation of the
 * data-parallel hot path of self-consistent second-order Green's function
 * theory (GF2) of Phillips & Zgid, arXiv:1405.3273.
 *
 * The method (Implementation section and Supplementary Material):
 *
 *   Eq. (GF)         G(i w_n) = [ (mu + i w_n) S - F - Sigma(i w_n) ]^-1
 *   Eq. (FockMatrix) F_ij = h_ij + sum_kl P_kl ( v_ijlk - v_iklj / 2 )
 *   Eq. (Sigma)      Sigma_ij(tau) = - sum_{klmnpq} G_kl(tau) G_mn(tau) G_pq(-tau)
 *                                    * v_imqk ( 2 v_lpnj - v_nplj )
 *
 * iterated as steps 1-3 of the Supplementary Material: a reference, an
 * inner loop (2.a mu search, 2.b Fock rebuild) at fixed Sigma, then a new
 * Sigma(tau) and its transform to the Matsubara axis.
 *
 * Conventions shared by every call
 * --------------------------------
 * - n basis functions (non-orthogonal AO basis, spin restricted).
 * - Real matrices are FP64, row-major, [n][n].  v is FP64 [n][n][n][n],
 *   v[i][j][k][l] = (ij|kl) in chemist notation with the 8-fold symmetry
 *   of real integrals (the library relies on it).
 * - Complex arrays are interleaved (re, im) FP64 pairs, [niw][n][n].
 * - Matsubara grid: w_n = (2n+1) pi / beta, n = 0..niw-1 (only n >= 0 is
 *   stored; X(-i w) = conj X(i w)).
 * - Imaginary-time grid: uniform, tau_k = k beta / (ntau-1), k = 0..ntau-1,
 *   both endpoints included; tau_0 and tau_{ntau-1} stand for 0+ and beta-.
 *   G(-tau_k) = -G(tau_{ntau-1-k}) (antiperiodicity).
 * - P is the spin-summed density (tr(P S) = nelec); G and Sigma are per spin.
 * - Every array argument is a DEVICE pointer owned by the caller unless
 *   the argument says "host".  The library never frees caller memory; it
 *   owns only the workspaces inside a gf2_ctx.
 * - Calls are ordered on the context's stream.  Calls that return host
 *   scalars synchronise that stream before returning.
 * - Every function returns a status code (GF2_OK = 0 or a negative
 *   GF2_E* value).  No exception crosses the ABI.  gf2_last_error() returns
 *   a message for the last failure on the calling thread.
 */
#ifndef GF2_H
#define GF2_H

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------- */
#define GF2_OK          0
#define GF2_EINVAL     -1   /* bad argument (sizes, NULL, enum value)            */
#define GF2_EHIP       -2   /* a HIP runtime call failed                         */
#define GF2_ENOMEM     -3   /* device allocation failed                          */
#define GF2_ENOCONV    -4   /* an iteration hit its step limit                   */
#define GF2_EBRACKET   -5   /* nelec outside [0, 2n] or the mu bracket failed    */
#define GF2_ENONFINITE -6   /* a NaN/Inf appeared in a result                    */
#define GF2_ESTATE     -7   /* call order: no system set on the context          */

/* ---- enums ------------------------------------------------------------ */
/* Arithmetic of the Sigma(tau) contraction (everything else is FP64). */
#define GF2_PREC_FP64    0   /* FP64 MFMA                                        */
#define GF2_PREC_FP32    1   /* FP32 MFMA, FP32 accumulate, FP64 final sums      */
#define GF2_PREC_BF16X3  2   /* operands split hi+lo BF16, hi*hi+hi*lo+lo*hi     */
                             /* on BF16 MFMA, FP32 accumulate, FP64 final sums   */
#define GF2_PREC_BF16X6  3   /* operands split hi+mid+lo BF16; the six products  */
                             /* of order 1, 2^-8 and 2^-16 on BF16 MFMA, FP32    */
                             /* accumulate, FP64 final sums (n <= 144)           */
#define GF2_PREC_BF16MIX 4   /* per stage: first index transform FP32 MFMA; the  */
                             /* second and third as BF16X6 (the FP32 first-      */
                             /* transform result split in registers); the final  */
                             /* contraction as BF16X3 (n <= 144)                  */

#define GF2_TAU2IW 0         /* gf2_fourier: Sigma(tau) -> Sigma(i w), Sigma_1  */
#define GF2_IW2TAU 1         /* gf2_fourier: G(i w) + tail moments -> G(tau)     */

#define GF2_DYSON_TRACE  0   /* tr(P S) only                                     */
#define GF2_DYSON_FULL   1   /* + G(i w) (optional) and P                        */
#define GF2_DYSON_ENERGY 2   /* + the two-body Galitskii-Migdal energy            */

#define GF2_MU_BISECT    0   /* bracket around mu0, midpoints                    */
#define GF2_MU_ILLINOIS  1   /* bracket around mu0, Illinois regula falsi         */
#define GF2_MU_SECANT    2   /* start at mu0, secant step from the previous slope, */
                             /* expand to a bracket, then Illinois                */

typedef struct gf2_ctx gf2_ctx;

typedef struct {
    int    n;       /* basis functions                                     */
    int    nelec;   /* electrons (spin-summed)                             */
    int    ntau;    /* tau points including both endpoints, >= 4           */
    int    niw;     /* Matsubara frequencies (n >= 0), >= 1                */
    double beta;    /* inverse temperature (1/Eh), > 0                     */
} gf2_dims;

typedef struct {
    double tol_mu;       /* mu search: stop when the bracket is narrower      */
    double tol_N;        /* mu search: accept when |tr(PS) - nelec| < tol_N    */
    double tol_P;        /* inner loop: stop when max|P_out - P_in| < tol_P    */
    double tol_E;        /* outer loop: |dE| threshold (reported, see below)   */
    int    max_inner;    /* inner passes per outer iteration                   */
    int    max_bisect;   /* mu evaluations per search                          */
    double mu_halfwidth; /* initial half-width of the mu bracket (Eh)          */
    double damp_P;       /* density damping a_P in the inner loop              */
    int    mix_depth;    /* Pulay history length (1 = plain damping)           */
    double damp_Sigma;   /* Sigma(tau) damping a_S in the outer loop           */
    int    mu_method;    /* GF2_MU_BISECT, GF2_MU_ILLINOIS or GF2_MU_SECANT    */
    int    prec;         /* GF2_PREC_* for Sigma(tau)                          */
    double tol_N_rel;    /* >= 0.  0: every mu search of the inner loop uses    */
                         /* tol_N (the paper's loop as the oracle runs it).     */
                         /* > 0: inexact mu in early passes: pass k accepts     */
                         /* |N - nelec| < max(tol_N, min(1e-6, tol_N_rel *      */
                         /* max|P_out - P_in| of pass k-1)); the inner loop     */
                         /* stops only after a pass that used tol_N.            */
    int    sigma_df;     /* 0: Sigma(tau) from the integrals of gf2_set_system; */
                         /* 1: from the density-fitting factors, as            */
                         /* gf2_sigma_tau_df (prec FP64 or FP32; single-system */
                         /* gf2_iterate only)                                  */
} gf2_params;
/* No outer-iteration limit and no determinism switch: gf2_iterate runs one
 * outer iteration, so the caller owns the outer loop, its limit and its stop
 * test (tol_E is carried for that caller); and every call is deterministic --
 * all floating-point reductions (split-K partial sums, per-frequency partial
 * densities and traces, Fock partials) are added in a fixed order, so equal
 * inputs give bitwise equal results on every run and every launch shape. */

/* Outer-loop state, owned by the caller (device arrays [..][n][n]). */
typedef struct {
    double  mu;          /* in/out: chemical potential (start of the bracket)  */
    double *F;           /* in/out device [n][n]: Fock matrix (h at the start) */
    double *P;           /* in/out device [n][n]: density                      */
    double *G_tau;       /* in/out device [ntau][n][n]                         */
    double *Sigma_tau;   /* in/out device [ntau][n][n] (previous Sigma)        */
    int     iteration;   /* in/out: completed outer iterations (0 = none)      */
    int     has_P;       /* in/out: 0 until P holds a density                  */
    double  energy;      /* in/out: energy of the last iteration               */
} gf2_state;

typedef struct {
    double energy, e1b, e2b;     /* E = e1b + e2b (Eh)                         */
    double dE, dP;               /* change vs the previous outer iteration     */
    double mu;
    int    n_inner;              /* inner passes                               */
    int    n_eval;               /* tr(PS) evaluations in all mu searches      */
    double ms_sigma, ms_fourier, ms_inner, ms_total;   /* wall-clock, ms       */
} gf2_report;

/* ---- context ------------------------------------------------------------
 * gf2_ctx_create: bind a context to HIP device `device` and the stream
 * `stream` (a hipStream_t passed as void*; NULL = the device's null stream).
 * The context owns all workspaces; gf2_ctx_destroy frees them.
 */
int gf2_ctx_create(gf2_ctx **ctx, int device, void *stream);
int gf2_ctx_destroy(gf2_ctx *ctx);

/* Message of the last failure on the calling thread ("" if none).  The
 * message is per thread, not per context: a thread that drives several
 * contexts reads it right after the failing call. */
const char *gf2_last_error(void);

/* gf2_set_system: the one-particle data and integrals of the problem
 * (Implementation section: non-orthogonal AO basis with overlap S, core
 * Hamiltonian h, AO integrals v).  S, h: device [n][n]; v: device
 * [n][n][n][n] (ij|kl).  The data are copied; the context then also holds
 * S^-1, the layouts of v used by the Sigma contraction (for all precisions)
 * and the bracket W_lpnj = 2 v_lpnj - v_nplj of Eq. (Sigma).
 * Errors: GF2_EINVAL for n < 1 or NULL pointers, GF2_EINVAL if S is
 * singular.  Symmetry of S, h, v is assumed, not checked.
 */
int gf2_set_system(gf2_ctx *ctx, int n, const double *S, const double *h, const double *v);

/* gf2_sigma_tau: Eq. (Sigma) at every tau point, G(-tau) from
 * antiperiodicity.  G_tau: device [ntau][n][n] FP64 (symmetric).
 * Sigma_tau: device [ntau][n][n] FP64 output (may not alias G_tau), exactly
 * symmetric: Sigma_ij = Sigma_ji for symmetric G and integrals, so the
 * entries j >= i are computed and (i, j), j < i, is a copy of (j, i).
 * prec: GF2_PREC_*.  dims->n must equal the n of gf2_set_system;
 * nelec, niw are ignored.  Returns GF2_ENONFINITE if the result holds a
 * NaN or Inf, GF2_ENOMEM if the workspace cannot be allocated.
 * Workspace (owned by the context, kept between calls): the first and
 * second transforms' intermediates of a batch of tau points, at most 64
 * points, 48 GiB and half of the device memory free at the call (n = 100,
 * FP32: 64 points, 51 GB).  The first call for an (n, ntau, prec) class in a
 * process also times candidate batch and tile shapes on the input; every
 * shape gives bitwise the same result.
 */
int gf2_sigma_tau(gf2_ctx *ctx, const gf2_dims *dims, int prec,
                  const double *G_tau, double *Sigma_tau);

/* gf2_set_df_factors: density-fitting factors of the integrals, the
 * cheaper route to Eq. (Sigma) that the Implementation section proposes
 * (recalled in the Conclusions): v_ijkl = sum_P B^P_ij B^P_kl over naux
 * auxiliary functions P.  B: device [naux][n][n] FP64, each B^P symmetric
 * (assumed, not checked), n that of gf2_set_system.  The factors are
 * copied (with the layouts gf2_sigma_tau_df reads, FP64 and FP32); the
 * context keeps them until the next gf2_set_df_factors or gf2_set_system,
 * which drops them.  They are used only by gf2_sigma_tau_df and by
 * gf2_iterate with prm->sigma_df = 1; v of gf2_set_system stays the
 * integrals of the Fock build.
 * Errors: GF2_EINVAL for naux < 1 or a NULL B; GF2_ESTATE without a system.
 */
int gf2_set_df_factors(gf2_ctx *ctx, int naux, const double *B);

/* gf2_sigma_tau_df: Eq. (Sigma) with the factored integrals of
 * gf2_set_df_factors.  With Y^P = B^P G(tau), X^PQ = Y^P B^Q and
 * Gb = G(-tau), the two diagrams become
 *   Sigma = -( 2 sum_PQ tr(X^PQ Gb) X^PQ - sum_PQ X^PQ Gb X^PQ ),
 * evaluated on MFMA GEMMs.  The direct term costs O(naux n^3 + naux^2 n^2)
 * flops per tau point; the exchange term is taken either as the products of
 * every factor pair (4 naux^2 n^3 flops) or through the n^4 tensor
 * sum_Q (B^Q Gb) (x) B^Q (4 naux n^4 flops), the latter when naux > n and
 * its n^4 array fits in 16 GiB (GF2_DF_ROUTE=pair|tensor in the
 * environment forces one).  Arguments and output as gf2_sigma_tau (G_tau and Sigma_tau
 * device [ntau][n][n] FP64, G symmetric, Sigma returned exactly symmetric);
 * prec: GF2_PREC_FP64 (FP64 MFMA) or GF2_PREC_FP32 (FP32 MFMA and FP32
 * intermediates, sums over more than 512 terms carried in FP64).
 * Errors: GF2_ESTATE without factors; GF2_EINVAL for another prec, a
 * dims->n that differs from the system, ntau < 4, aliasing, NULL pointers;
 * GF2_ENOMEM if the workspace (5 naux n^2 + 2 n^2 + naux^2 elements, the
 * split-K partial sums, and 1 GiB of pair products or the n^4 array)
 * cannot be allocated;
 * GF2_ENONFINITE for a NaN or Inf in the result.
 */
int gf2_sigma_tau_df(gf2_ctx *ctx, const gf2_dims *dims, int prec,
                     const double *G_tau, double *Sigma_tau);

/* gf2_fourier: transforms between imaginary time and Matsubara frequency
 * (Implementation section: FFT with an analytic high-frequency tail).
 *   dir = GF2_TAU2IW: in = Sigma(tau) device [ntau][n][n] FP64;
 *       out = Sigma(i w_n) device [niw][n][n] complex FP64 -- the Fourier
 *       integral of the not-a-knot cubic spline of Sigma(tau), taken
 *       exactly interval by interval; moment1_out (device [n][n], may be
 *       NULL) = Sigma_1 = -(Sigma(0+) + Sigma(beta-)).  moments unused.
 *   dir = GF2_IW2TAU: in = G(i w_n) device [niw][n][n] complex;
 *       moments = device [3][n][n] = G1, G2, G3 of the tail
 *       G ~ G1/(iw) + G2/(iw)^2 + G3/(iw)^3;
 *       out = G(tau) device [ntau][n][n] FP64: the tail-subtracted
 *       Matsubara sum plus the tail in closed form.  moment1_out unused.
 * The tau grid is uniform, tau_k = k beta/(ntau-1), unless a grid was set
 * with gf2_set_tau_grid; then dims->ntau must equal its length and its last
 * point must equal dims->beta (GF2_EINVAL otherwise).
 * Works on any n (no system needed).
 */
int gf2_fourier(gf2_ctx *ctx, const gf2_dims *dims, int dir, const void *in,
                const double *moments, void *out, double *moment1_out);

/* gf2_set_tau_grid: a non-equidistant imaginary-time grid for this context
 * (Implementation section: the paper uses a non-equidistant grid of a few
 * thousand points).  tau: device [ntau] FP64, copied; tau_0 = 0 < tau_1 <
 * ... < tau_{ntau-1} = beta, symmetric about beta/2 (tau_{M-k} = beta -
 * tau_k, so G(-tau_k) = -G(tau_{M-k}) stays on the grid).  Every later
 * gf2_fourier, gf2_iterate and gf2_iterate_batched call on the context
 * samples G(tau), Sigma(tau) at these points: the spline integral and the
 * Matsubara sum use the actual spacings (FP64 MFMA GEMMs against weight
 * tables built on first use for each (niw, beta)).  ntau = 0 (tau may be
 * NULL) restores the uniform grid.  Synchronises the context's stream.
 * Errors: GF2_EINVAL for ntau < 4, a NULL grid, or a grid that does not
 * start at 0, increase strictly, or mirror about its midpoint.
 */
int gf2_set_tau_grid(gf2_ctx *ctx, int ntau, const double *tau);

/* gf2_dyson: Eq. (GF) at every Matsubara frequency for chemical potential
 * mu, with the system's S and the given F (device [n][n]) and
 * Sigma(i w) (device [niw][n][n] complex, NULL = 0) and Sigma_1 (device
 * [n][n], NULL = 0).  Each inverse is a Gauss-Jordan elimination with
 * partial pivoting in FP64.  The density is P = -2 G(beta-) with the tail
 * summed exactly: P = (4/beta) sum_n Re[G - G1/(iw) - G2/(iw)^2 - G3/(iw)^3]
 * + G1 - (beta/2) G2.
 *   mode TRACE:  host_out[0] = tr(P S).  G_iw, P ignored.
 *   mode FULL:   also writes P (device [n][n]) and, if G_iw != NULL,
 *                G (device [niw][n][n] complex).
 *   mode ENERGY: as FULL, and host_out[1] = E_2b = (1/beta) sum over all n
 *                of tr[G Sigma] (truncated sum + exact 1/w^2 tail).
 * host_out: host double[2].
 */
int gf2_dyson(gf2_ctx *ctx, const gf2_dims *dims, int mode, double mu,
              const double *F, const void *Sigma_iw, const double *Sigma1,
              void *G_iw, double *P, double *host_out);

/* gf2_dyson_noalloc: gf2_dyson for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same arguments, modes, results and errors as
 * gf2_dyson (the same kernels on the same workgroups, so the same bits); the
 * workspace (tail moments, per-workgroup partial sums, reduced results) is a
 * fixed device array of GF2_NOALLOC_SCRATCH_BYTES that the library holds on
 * every GPU it runs on until the process ends, instead of context memory, so
 * the call makes no hipMalloc/hipFree or other allocating call.  The context
 * itself (gf2_ctx_create, gf2_set_system) is set up beforehand as usual.
 * All calls on one GPU share that array: calls that overlap on one GPU
 * (other host threads, other contexts' streams) race and must be serialised
 * by the caller.  Workspace: 48 n^2 bytes of moments plus 32 bytes per
 * partial-sum slot (at most 8 per CU) and, for FULL/ENERGY, n^2 doubles per
 * P partial (one per workgroup: 2 per CU for n > 48); a solve that needs more
 * than GF2_NOALLOC_SCRATCH_BYTES returns GF2_EINVAL and changes nothing (on
 * a 256-CU MI355X: TRACE for every n <= 160, FULL/ENERGY up to n = 127).
 * Synchronises the context's stream (host_out).
 */
#define GF2_NOALLOC_SCRATCH_BYTES (64u << 20)
int gf2_dyson_noalloc(gf2_ctx *ctx, const gf2_dims *dims, int mode, double mu,
                      const double *F, const void *Sigma_iw, const double *Sigma1,
                      void *G_iw, double *P, double *host_out);

/* gf2_fock: Eq. (FockMatrix) F = h + J(P) - K(P)/2 for the system's h and
 * v.  P, F: device [n][n] (may not alias).
 */
int gf2_fock(gf2_ctx *ctx, const double *P, double *F);

/* gf2_natural_occupations: the natural occupation numbers of a density
 * (Results: the NONs of the self-consistent density, plotted for the H32
 * lattice against the lattice parameter; Supplementary Material, NON plots).
 * The paper gives no formula; they are taken as the eigenvalues of the
 * spin-summed density in the symmetrically orthonormalised basis,
 * S^{1/2} P S^{1/2} (the spectrum of P S), with S of gf2_set_system.
 * P: device [n][n] FP64, symmetric (only the whole matrix is read; it is not
 * modified).  occ: device [n] FP64, written largest first; with tr(P S) = N_e
 * the values lie in [0, 2] and sum to N_e.  Runs on the context's stream and
 * synchronises it (the status of the eigensolver is read back).
 * Errors: GF2_EINVAL for NULL arguments, n > 1024 or an overlap that is not
 * positive definite; GF2_ESTATE without a system; GF2_ENOCONV if the Jacobi
 * sweeps do not converge; GF2_ENONFINITE for a NaN/Inf eigenvalue (occ is
 * written in every case except GF2_EINVAL/GF2_ESTATE).
 */
int gf2_natural_occupations(gf2_ctx *ctx, const double *P, double *occ);

/* gf2_density_fock: one pass of steps 2.a-2.b at fixed Sigma: find mu
 * (bracketing search on tr(P(mu) S) = nelec, see gf2_params) starting from
 * *mu_inout (host), then P_out = P(mu) (device [n][n]), F_out = F(P_out)
 * (device [n][n], may be NULL) and, if G_iw_out != NULL, the G(i w) of that
 * Dyson solve.  host_out (host double[4]) = { tr(P_out S), E_1b =
 * tr[P_out (h + F_out)]/2 (0 if F_out is NULL), E_2b (0 if Sigma_iw is
 * NULL), number of tr(PS) evaluations }.
 * Errors: GF2_EBRACKET if nelec is outside [0, 2n] or no bracket is found,
 * GF2_ENOCONV if the search exceeds max_bisect evaluations.
 */
int gf2_density_fock(gf2_ctx *ctx, const gf2_dims *dims, const gf2_params *prm,
                     const double *F_in, const void *Sigma_iw, const double *Sigma1,
                     double *mu_inout, double *P_out, double *F_out, void *G_iw_out,
                     double *host_out);

/* gf2_iterate: one outer iteration of the Supplementary Material's loop.
 * iteration 0 (st->iteration == 0): the reference, step 2 with Sigma = 0
 * from st->F (the core guess h) -- a finite-beta Hartree-Fock solution.
 * iteration >= 1: Sigma(tau) from st->G_tau (step 3; exactly symmetric as
 * gf2_sigma_tau returns it, so the rounding of the reduced-precision forms
 * seeds no antisymmetric part that the loop would amplify), damped against
 * st->Sigma_tau from the second correlated iteration on, transformed to
 * Sigma(i w); then the inner loop: passes of gf2_density_fock with the
 * density mixed by damped Pulay/Anderson mixing of (P_in, P_out - P_in)
 * (mix_depth 1 = the plain damping of the paper) until
 * max|P_out - P_in| < tol_P; then E = E_1b + E_2b and the new G(tau).
 * All state arrays are updated in place.  The report (host) carries the
 * energy, its change, max|dP| against the previous iteration, mu, pass
 * and evaluation counts and stage timings.
 */
int gf2_iterate(gf2_ctx *ctx, const gf2_dims *dims, const gf2_params *prm,
                gf2_state *st, gf2_report *rep);

/* gf2_iterate_batched: one outer iteration (as gf2_iterate) for each of nsys
 * independent systems, e.g. a geometry sweep with uneven n -- the systems of
 * the paper's sweeps are independent problems, so they share launches only.
 * ctxs[s] (host array of nsys distinct contexts on one device) holds system
 * s (gf2_set_system), dims[s] its sizes and states[s] its state (device
 * arrays as for gf2_iterate); prm applies to all.  Everything runs on
 * ctxs[0]'s stream (the other contexts' streams are synchronised first and
 * left untouched).  The inner loops advance in lockstep: each round solves
 * Eq. (GF) at the pending mu of every system's search, or its density pass,
 * as one replay of a captured HIP graph (tail moments, the inversions of all
 * systems grouped by size class, the reductions); every system gets the
 * workgroups and arithmetic of gf2_iterate, so its result is the same.
 * reports[s] as gf2_iterate, except that ms_sigma, ms_fourier, ms_inner and
 * ms_total are the times of the whole batch.  Errors: as gf2_iterate for any
 * system; GF2_EINVAL for nsys < 1, NULL arrays, a repeated context or
 * contexts on different devices.  On error the states of all systems are
 * unspecified.
 */
int gf2_iterate_batched(gf2_ctx *const *ctxs, int nsys, const gf2_dims *dims,
                        const gf2_params *prm, gf2_state *states, gf2_report *reports);

/* ---- opt-in kernel timing -------------------------------------------------
 * With profiling on, the context brackets every launch of the listed kernel
 * classes with a pair of HIP events on its stream and records the
 * algorithmic work of that launch:
 *   GF2_KC_SIGMA_GEMM    first index transform of Eq. (Sigma) (contracts m); work = flops
 *   GF2_KC_SIGMA_SPLITK  final contraction of Eq. (Sigma);    work = flops
 *   GF2_KC_SIGMA_S23     second and third index transforms, fused (contract q, k);
 *                        work = flops (4 n^5 per tau point)
 *   GF2_KC_DYSON         Eq. (GF) inversions (any mode);       work = flops (8 n^3 per frequency)
 *   GF2_KC_T2I_EXPAND    Sigma(i w) expansion;                 work = bytes written (16 n^2 niw)
 *   GF2_KC_I2T_FOLD      G(i w) fold;                          work = bytes read (16 n^2 niw)
 *   GF2_KC_FOCK          Eq. (FockMatrix);                     work = bytes read (8 n^4)
 *   GF2_KC_OCCUPATIONS   natural occupation numbers (gf2_natural_occupations, all
 *                        three steps as one bracket);          work = n (eigenvalues)
 *   GF2_KC_SIGMA_DF      density-fitted Eq. (Sigma), one bracket per tau point;
 *                        work = flops of the route taken (m = naux): pair route
 *                        4 m^2 n^3 + 4 m^2 n^2 + 8 m n^3, tensor route
 *                        4 m n^4 + 4 m^2 n^2 + 10 m n^3
 * gf2_profile_enable(ctx, 1) clears the counters and starts recording;
 * gf2_profile_enable(ctx, 0) stops.  gf2_profile_read synchronises the
 * stream and fills host arrays [nslots] (nslots <= GF2_KC_COUNT) with the
 * summed event time (ms), the number of launches and the summed work.
 */
#define GF2_KC_SIGMA_GEMM   0
#define GF2_KC_SIGMA_SPLITK 1
#define GF2_KC_DYSON        2
#define GF2_KC_T2I_EXPAND   3
#define GF2_KC_I2T_FOLD     4
#define GF2_KC_FOCK         5
#define GF2_KC_SIGMA_S23    6
#define GF2_KC_OCCUPATIONS  7
#define GF2_KC_SIGMA_DF     8
#define GF2_KC_COUNT        9

int gf2_profile_enable(gf2_ctx *ctx, int on);
int gf2_profile_read(gf2_ctx *ctx, int nslots, double *ms, long long *launches, double *work);

#ifdef __cplusplus
}
#endif
#endif /* GF2_H */
