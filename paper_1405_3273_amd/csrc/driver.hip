// The GF2 loop (Supplementary Material, steps 1-3) on top of the stage kernels.
//
// Host-side control only: every array operation runs on the device; the host
// keeps scalars (mu bracket, residual norms, the small Pulay system).
//
// mu search (step 2.a): bracketing search on N(mu) = tr(P(mu) S) - nelec.
//   Bracket [mu0 - hw, mu0 + hw]; while N(lo) > 0 move to [lo - w, lo], while
//   N(hi) < 0 move to [hi, hi + w]; or (secant start) evaluate N(mu0), step by
//   -N(mu0)/slope (slope from the previous search, 1/hw without one; step size
//   clamped to [4 tol_mu, hw]) and double the step until the sign changes.
//   Then evaluate an interior point (midpoint, or the Illinois regula-falsi
//   point when it is strictly inside), accept it when |N| < tol_N, otherwise
//   replace the end with the same sign (Illinois halves the value kept at an
//   end that survives two steps in a row); stop at bracket width < tol_mu with
//   the midpoint.
// Inner loop (2.a-2.b): F = F(P_in) -> mu -> P_out; r = P_out - P_in; stop at
//   max|r| < tol_P; next P_in = sum_a c_a (x_a + (1 - a_P) r_a) with
//   c = argmin |sum c_a r_a|, sum c_a = 1 over the last mix_depth pairs.
// Outer iteration (3): Sigma(tau) from G(tau), damping, Sigma(i w), inner
//   loop, Galitskii-Migdal energy, G(tau).
#include "gf2_internal.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <vector>

namespace gf2 {

static double now_ms() {
    using namespace std::chrono;
    return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

// N(mu) - nelec via the TRACE Dyson solve
static int particle_excess(gf2_ctx *c, const gf2_dims *d, double mu, const double *F,
                           const double2 *Sig, double *out) {
    double r[2];
    GF2_TRY(dyson_run(c, d, GF2_DYSON_TRACE, mu, F, Sig, nullptr, nullptr, nullptr, nullptr, r));
    *out = r[0] - (double)d->nelec;
    return GF2_OK;
}

// The mu search as a resumable state machine: start() sets the first mu to
// evaluate (pending); feed(N(pending) - nelec) either finishes (done, mu) or
// sets the next pending mu.  One search per system; the batched driver runs
// many of them in lockstep, one Dyson launch per round.
struct MuSearch {
    const gf2_params *p = nullptr;
    double hint = 0.0;                // slope dN/dmu from the previous search (<= 0: none)
    double slope = 0.0;               // slope of the final bracket (valid if have_slope)
    bool have_slope = false;
    int evals = 0;
    int stage = 0;                    // 1 secant start, 2 secant expansion, 3 lower end,
                                      // 4 upper end, 5 interior
    double a = 0, fa = 0, b = 0, fb = 0, lo = 0, hi = 0, f_lo = 0, f_hi = 0, t_lo = 0, t_hi = 0;
    int side = 0, istep = 0;
    double pending = 0.0;
    bool done = false;
    double mu = 0.0;
    double tolN = 0.0;                // acceptance |N - nelec| < tolN (params->tol_N or looser)

    void start(const gf2_params *prm, double mu0, double slope_hint, double tol_n) {
        p = prm;
        tolN = tol_n;
        hint = slope_hint;
        have_slope = false;
        evals = 0;
        done = false;
        side = 0;
        istep = 0;
        if (p->mu_method == GF2_MU_SECANT) {
            a = mu0;
            stage = 1;
            pending = a;
        } else {
            lo = mu0 - p->mu_halfwidth;
            hi = mu0 + p->mu_halfwidth;
            stage = 3;
            pending = lo;
        }
    }
    void finish(double m, double l, double fl, double h, double fh, bool have) {
        if (have && h > l && fh > fl) {
            slope = (fh - fl) / (h - l);
            have_slope = true;
        }
        mu = m;
        done = true;
    }
    int next_interior() {
        if (istep >= p->max_bisect) return fail(GF2_ENOCONV, "mu search did not converge");
        double mid = 0.5 * (lo + hi);
        if (p->mu_method != GF2_MU_BISECT && f_hi > f_lo) {
            const double x = (lo * f_hi - hi * f_lo) / (f_hi - f_lo);
            if (lo < x && x < hi) mid = x;
        }
        pending = mid;
        stage = 5;
        return GF2_OK;
    }
    int enter_interior() {
        t_lo = f_lo;
        t_hi = f_hi;
        side = 0;
        istep = 0;
        return next_interior();
    }
    int feed(double f) {
        ++evals;
        switch (stage) {
            case 1: {
                fa = f;
                if (std::fabs(fa) < tolN) {
                    finish(a, 0, 0, 0, 0, false);
                    return GF2_OK;
                }
                const double s_ = (hint > 0.0) ? hint : 1.0 / p->mu_halfwidth;
                double step = -fa / s_;
                const double mag =
                    std::fmin(std::fmax(std::fabs(step), 4.0 * p->tol_mu), p->mu_halfwidth);
                step = step > 0.0 ? mag : -mag;
                b = a + step;
                if (evals > p->max_bisect) return fail(GF2_EBRACKET, "mu search: no bracket found");
                stage = 2;
                pending = b;
                return GF2_OK;
            }
            case 2: {
                fb = f;
                if (std::fabs(fb) < tolN) {
                    if (a < b) finish(b, a, fa, b, fb, true);
                    else finish(b, b, fb, a, fa, true);
                    return GF2_OK;
                }
                if ((fb > 0.0) != (fa > 0.0)) {
                    if (a < b) { lo = a; f_lo = fa; hi = b; f_hi = fb; }
                    else       { lo = b; f_lo = fb; hi = a; f_hi = fa; }
                    return enter_interior();
                }
                const double nb = b + 2.0 * (b - a);
                a = b;
                fa = fb;
                b = nb;
                if (evals > p->max_bisect) return fail(GF2_EBRACKET, "mu search: no bracket found");
                pending = b;
                return GF2_OK;
            }
            case 3: {
                f_lo = f;
                if (f_lo > 0.0) {
                    if (evals > p->max_bisect) return fail(GF2_EBRACKET, "mu search: no lower bracket end");
                    const double w = hi - lo;
                    hi = lo;
                    lo = lo - w;
                    pending = lo;
                    return GF2_OK;
                }
                stage = 4;
                pending = hi;
                return GF2_OK;
            }
            case 4: {
                f_hi = f;
                if (f_hi < 0.0) {
                    if (evals > p->max_bisect) return fail(GF2_EBRACKET, "mu search: no upper bracket end");
                    const double w = hi - lo;
                    lo = hi;
                    hi = hi + w;
                    pending = hi;
                    return GF2_OK;
                }
                return enter_interior();
            }
            case 5: {
                const double mid = pending, fm = f;
                if (std::fabs(fm) < tolN) {
                    if (fm < 0.0) finish(mid, mid, fm, hi, t_hi, true);
                    else finish(mid, lo, t_lo, mid, fm, true);
                    return GF2_OK;
                }
                if (fm < 0.0) {
                    lo = mid;
                    f_lo = fm;
                    t_lo = fm;
                    if (side == -1) f_hi *= 0.5;
                    side = -1;
                } else {
                    hi = mid;
                    f_hi = fm;
                    t_hi = fm;
                    if (side == 1) f_lo *= 0.5;
                    side = 1;
                }
                if (hi - lo < p->tol_mu) {
                    finish(0.5 * (lo + hi), lo, t_lo, hi, t_hi, true);
                    return GF2_OK;
                }
                ++istep;
                return next_interior();
            }
            default:
                return fail(GF2_ESTATE, "mu search: not started");
        }
    }
};

// Returns mu and the number of evaluations; *slope is read (hint, <= 0 = none)
// and replaced by the secant slope dN/dmu of the final bracket when known.
static int find_mu(gf2_ctx *c, const gf2_dims *d, const gf2_params *p, const double *F,
                   const double2 *Sig, double mu0, double *mu_out, int *evals_out,
                   double *slope) {
    if (d->nelec < 0 || d->nelec > 2 * c->n)
        return fail(GF2_EBRACKET, "mu search: nelec outside [0, 2n]");
    MuSearch ms;
    ms.start(p, mu0, slope ? *slope : 0.0, p->tol_N);
    while (!ms.done) {
        double f;
        GF2_TRY(particle_excess(c, d, ms.pending, F, Sig, &f));
        GF2_TRY(ms.feed(f));
    }
    if (ms.have_slope && slope) *slope = ms.slope;
    *mu_out = ms.mu;
    *evals_out = ms.evals;
    return GF2_OK;
}

// One pass of 2.a-2.b without the Fock rebuild: mu, P_out, G(i w), moments, E_2b.
static int density_pass(gf2_ctx *c, const gf2_dims *d, const gf2_params *p, const double *F,
                        const double2 *Sig, const double *Sig1, double *mu, double *P_out,
                        double2 *G_iw, double *mom, double *trPS, double *e2b, int *evals,
                        double *slope) {
    GF2_TRY(find_mu(c, d, p, F, Sig, *mu, mu, evals, slope));
    double r[2];
    const int mode = Sig ? GF2_DYSON_ENERGY : GF2_DYSON_FULL;
    GF2_TRY(dyson_run(c, d, mode, *mu, F, Sig, Sig1, G_iw, P_out, mom, r));
    *trPS = r[0];
    *e2b = r[1];
    return GF2_OK;
}

// Solve the bordered Pulay system (oldest first) exactly as the oracle does.
// Returns false if a pivot is negligible.
static bool solve_pivoted(int n, std::vector<double> A, std::vector<double> b,
                          std::vector<double> &x) {
    double scale = 0.0;
    for (double v : A) scale = std::fmax(scale, std::fabs(v));
    for (int k = 0; k < n; ++k) {
        int r = k;
        for (int i = k + 1; i < n; ++i)
            if (std::fabs(A[i * n + k]) > std::fabs(A[r * n + k])) r = i;
        if (!(std::fabs(A[r * n + k]) > 1e-14 * scale)) return false;
        if (r != k) {
            for (int j = 0; j < n; ++j) std::swap(A[k * n + j], A[r * n + j]);
            std::swap(b[k], b[r]);
        }
        for (int i = k + 1; i < n; ++i) {
            const double f = A[i * n + k] / A[k * n + k];
            for (int j = k; j < n; ++j) A[i * n + j] -= f * A[k * n + j];
            b[i] -= f * b[k];
        }
    }
    x.assign(n, 0.0);
    for (int k = n - 1; k >= 0; --k) {
        double s = b[k];
        for (int j = k + 1; j < n; ++j) s -= A[k * n + j] * x[j];
        x[k] = s / A[k * n + k];
    }
    return true;
}

// ---------------------------------------------------------------------------
// Inner-loop reductions and Pulay updates on the device.  Reduction results go
// to a small device array (`red`, IL_RED doubles per system) that the caller
// copies to the host; the batched driver copies the arrays of all systems in
// one transfer, overlapped with the next Dyson round of the other systems.

constexpr int IL_THREADS = 256;
constexpr int IL_MAXDEPTH = 32;
constexpr int IL_RED = 40;    // >= 1 + IL_MAXDEPTH

struct SlotList {
    int id[IL_MAXDEPTH];      // Pulay slots, oldest first
    double c[IL_MAXDEPTH];    // mixing coefficients (k_pulay_mix)
    int k;
};

// fixed-order block reduction (op 0: max, else sum) of one value per thread
template <int OP>
__device__ double block_reduce(double v, double *sh) {
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int s = IL_THREADS / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
            sh[threadIdx.x] = OP == 0 ? fmax(sh[threadIdx.x], sh[threadIdx.x + s])
                                      : sh[threadIdx.x] + sh[threadIdx.x + s];
        __syncthreads();
    }
    return sh[0];
}

// red[0] = max_e |a[e] - b[e]|
__global__ __launch_bounds__(IL_THREADS) void k_maxdiff(int ne, const double *__restrict__ a,
                                                        const double *__restrict__ b,
                                                        double *__restrict__ red) {
    __shared__ double sh[IL_THREADS];
    double m = 0.0;
    for (int e = threadIdx.x; e < ne; e += IL_THREADS) m = fmax(m, fabs(a[e] - b[e]));
    m = block_reduce<0>(m, sh);
    if (threadIdx.x == 0) red[0] = m;
}

// red[1 + j] = <r_s, r_{id[j]}> (one workgroup per j), r_o = slots + (2 o + 1) ne
__global__ __launch_bounds__(IL_THREADS) void k_pulay_dots(int ne, int s, const double *__restrict__ slots,
                                                           SlotList L, double *__restrict__ red) {
    __shared__ double sh[IL_THREADS];
    const double *rs = slots + (size_t)(2 * s + 1) * ne;
    const double *ro = slots + (size_t)(2 * L.id[blockIdx.x] + 1) * ne;
    double acc = 0.0;
    for (int e = threadIdx.x; e < ne; e += IL_THREADS) acc += rs[e] * ro[e];
    acc = block_reduce<1>(acc, sh);
    if (threadIdx.x == 0) red[1 + blockIdx.x] = acc;
}

// slot s: x_s = P_in, r_s = P_out - P_in
__global__ void k_pulay_push(int ne, const double *__restrict__ Pin, const double *__restrict__ Pout,
                             double *__restrict__ xs) {
    double *rs = xs + ne;
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < ne; e += gridDim.x * blockDim.x) {
        const double x = Pin[e];
        xs[e] = x;
        rs[e] = Pout[e] - x;
    }
}

// P_next = sum_a c_a (x_a + (1 - damp) r_a)   (may overwrite P_in: reads only slots)
__global__ void k_pulay_mix(int ne, const double *__restrict__ slots, SlotList L, double damp,
                            double *__restrict__ Pnext) {
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < ne; e += gridDim.x * blockDim.x) {
        double acc = 0.0;
        for (int a = 0; a < L.k; ++a) {
            const double *x = slots + (size_t)(2 * L.id[a]) * ne;
            acc = fma(L.c[a], fma(1.0 - damp, x[ne + e], x[e]), acc);
        }
        Pnext[e] = acc;
    }
}

static unsigned grid_for(size_t ne) { return (unsigned)std::min<size_t>((ne + 255) / 256, 1024); }

// Pulay restart factor (see InnerLoop::on_red) and the largest mixing
// coefficient accepted before the history is cut to the newest pair
constexpr double PULAY_RESTART = 10.0;
constexpr double PULAY_CMAX = 20.0;

struct Pulay {
    int depth = 1;
    // device slots: x_a, r_a (ring of depth entries), host B_ab = <r_a, r_b>
    std::vector<int> order;          // slot ids, oldest first
    std::vector<double> B;           // depth x depth, indexed by slot
    int last = -1;                   // slot pushed last
    int free_slot() const {
        for (int s = 0; s < depth; ++s) {
            bool used = false;
            for (int o : order) used |= (o == s);
            if (!used) return s;
        }
        return -1;
    }
    // coefficients c (sum c_a = 1) minimising |sum c_a r_a|; a singular
    // system, or one whose coefficients exceed PULAY_CMAX, drops all but the
    // newest pair
    std::vector<double> coef() {
        for (;;) {
            const int k = (int)order.size();
            std::vector<double> A((k + 1) * (k + 1), 0.0), rhs(k + 1, 0.0), sol;
            double dmax = 0.0;
            for (int a = 0; a < k; ++a) dmax = std::fmax(dmax, B[order[a] * (depth + 1)]);
            dmax = std::fmax(dmax, 1e-300);
            for (int a = 0; a < k; ++a)
                for (int b = 0; b < k; ++b) A[a * (k + 1) + b] = B[order[a] * depth + order[b]] / dmax;
            for (int a = 0; a < k; ++a) {
                A[k * (k + 1) + a] = 1.0;
                A[a * (k + 1) + k] = 1.0;
            }
            rhs[k] = 1.0;
            if (solve_pivoted(k + 1, A, rhs, sol)) {
                double cmax = 0.0;
                for (int a = 0; a < k; ++a) cmax = std::fmax(cmax, std::fabs(sol[a]));
                // extrapolation too far: treated like a singular system
                if (k == 1 || cmax <= PULAY_CMAX) return std::vector<double>(sol.begin(), sol.begin() + k);
            }
            if (k == 1) return std::vector<double>(1, 1.0);
            order.erase(order.begin(), order.end() - 1);
        }
    }
};

// The inner loop (steps 2.a-2.b) of one system as a state machine.  Phase 0:
// the mu search wants N(ms.pending) (a density-mode solve, see on_eval); phase 1: the density
// pass wants a FULL (ENERGY when Sigma is set) solve at mu writing P_out,
// G(i w) and the tail moments; phase 3: device reductions were enqueued into
// `red` and on_red wants their values (want 1: max|P_out - P_in|; want 2: the
// Pulay dots); phase 2: converged.  The single-system loop and the batched
// driver feed it the same solves and reductions in the same order.
struct InnerLoop {
    gf2_ctx *c = nullptr;
    const gf2_dims *d = nullptr;
    const gf2_params *p = nullptr;
    const double2 *Sig = nullptr;
    const double *Sig1 = nullptr;
    double *Pin = nullptr, *Pout = nullptr, *F = nullptr, *slots = nullptr;
    double *mom = nullptr;
    double *red = nullptr;
    double2 *G_iw = nullptr;
    Pulay pl;
    MuSearch ms;
    bool have_Pin = false;
    double mu = 0.0, slope = 0.0, trPS = 0.0, e2b = 0.0;
    double rprev = INFINITY;   // max|P_out - P_in| of the previous pass
    double rbest = INFINITY;   // smallest max|P_out - P_in| of this inner loop
    double tol_pass = 0.0;     // mu acceptance of the current pass
    int it = 0, n_inner = 0, n_eval = 0, phase = 0, want = 0;

    // tol_N, or with tol_N_rel > 0 the inexact rule max(tol_N, tol_N_rel * rprev)
    // (at most 1e-6): early passes, whose P is still far from the fixed point,
    // locate mu less tightly; once rprev <= tol_N / tol_N_rel the rule is tol_N.
    double pass_tolerance() const {
        if (!(p->tol_N_rel > 0.0)) return p->tol_N;
        return std::fmax(p->tol_N, std::fmin(1e-6, p->tol_N_rel * rprev));
    }

    int density_mode() const { return Sig ? GF2_DYSON_ENERGY : GF2_DYSON_FULL; }
    // doubles of `red` that on_red reads
    int red_count() const { return want == 1 ? 1 : 1 + (int)pl.order.size(); }

    // workspaces and starting point (P from the state if present, F, mu);
    // red_dev: IL_RED doubles of device memory for the reductions
    int start(gf2_ctx *ctx, const gf2_dims *dd, const gf2_params *pp, const gf2_state *st,
              const double2 *sig, const double *sig1, double *red_dev) {
        c = ctx; d = dd; p = pp; Sig = sig; Sig1 = sig1; red = red_dev;
        const size_t ne = (size_t)c->n * c->n;
        GF2_TRY(c->it_Pout.ensure(ne * 8));
        GF2_TRY(c->it_Pin.ensure(ne * 8));
        GF2_TRY(c->it_F.ensure(ne * 8));
        GF2_TRY(c->it_mom.ensure(3 * ne * 8));
        GF2_TRY(c->it_G_iw.ensure((size_t)d->niw * ne * 16));
        GF2_TRY(c->it_hist.ensure((size_t)2 * p->mix_depth * ne * 8));
        Pin = c->it_Pin.as<double>();
        Pout = c->it_Pout.as<double>();
        F = c->it_F.as<double>();
        mom = c->it_mom.as<double>();
        G_iw = c->it_G_iw.as<double2>();
        slots = c->it_hist.as<double>();
        have_Pin = st->has_P != 0;
        if (have_Pin) GF2_TRY(copy_d2d(c, Pin, st->P, ne * 8));
        GF2_TRY(copy_d2d(c, F, st->F, ne * 8));
        mu = st->mu;
        slope = 0.0;
        pl = Pulay();
        pl.depth = p->mix_depth;
        pl.B.assign((size_t)pl.depth * pl.depth, 0.0);
        it = 1;
        n_inner = n_eval = 0;
        phase = 0;
        want = 0;
        rprev = INFINITY;
        rbest = INFINITY;
        tol_pass = pass_tolerance();
        ms.start(p, mu, slope, tol_pass);
        return GF2_OK;
    }
    // result of the phase-0 solve at ms.pending.  That solve runs in the
    // density mode: trace_n is what a TRACE solve would give (the search
    // sees the same values), and when the search accepts the point just
    // evaluated its P, G(i w) and moments are already in place, so the
    // density solve at mu is skipped.
    int on_eval(double trace_n, double trps, double e2) {
        const double x = ms.pending;
        GF2_TRY(ms.feed(trace_n - (double)d->nelec));
        if (ms.done) {
            mu = ms.mu;
            if (ms.have_slope) slope = ms.slope;
            phase = 1;
            if (ms.mu == x) return on_density(trps, e2);
        }
        return GF2_OK;
    }
    // the density solve at mu has written Pout, G_iw and mom
    int on_density(double trps, double e2) {
        const int ne = c->n * c->n;
        trPS = trps;
        e2b = e2;
        n_eval += ms.evals;
        n_inner = it;
        if (!have_Pin) {
            GF2_TRY(copy_d2d(c, Pin, Pout, (size_t)ne * 8));
            have_Pin = true;
            return next_iteration();
        }
        hipLaunchKernelGGL(k_maxdiff, dim3(1), dim3(IL_THREADS), 0, c->stream, ne, Pout, Pin, red);
        GF2_HIP(hipGetLastError());
        phase = 3;
        want = 1;
        return GF2_OK;
    }
    // h: the first red_count() values of `red`
    int on_red(const double *h) {
        const int ne = c->n * c->n;
        if (want == 1) {
            // converged only when this pass located mu to tol_N
            if (h[0] < p->tol_P && tol_pass <= p->tol_N) {
                phase = 2;
                want = 0;
                return GF2_OK;
            }
            rprev = h[0];
            // restart: a residual more than PULAY_RESTART times the best one of
            // this inner loop drops the history (the mix is a damped step)
            if (h[0] > PULAY_RESTART * rbest) pl.order.clear();
            rbest = std::fmin(rbest, h[0]);
            // push (P_in, r = P_out - P_in), dropping the oldest beyond depth
            if ((int)pl.order.size() == pl.depth) pl.order.erase(pl.order.begin());
            const int s = pl.free_slot();
            hipLaunchKernelGGL(k_pulay_push, dim3(grid_for(ne)), dim3(256), 0, c->stream, ne, Pin, Pout,
                               slots + (size_t)(2 * s) * ne);
            pl.order.push_back(s);
            pl.last = s;
            SlotList L{};
            L.k = (int)pl.order.size();
            for (int a = 0; a < L.k; ++a) L.id[a] = pl.order[a];
            hipLaunchKernelGGL(k_pulay_dots, dim3(L.k), dim3(IL_THREADS), 0, c->stream, ne, s, slots,
                               L, red);
            GF2_HIP(hipGetLastError());
            want = 2;
            return GF2_OK;
        }
        // want == 2: B row/column of the new slot, then the mixed P_in
        const int s = pl.last;
        for (size_t a = 0; a < pl.order.size(); ++a) {
            const int o = pl.order[a];
            pl.B[s * pl.depth + o] = h[1 + a];
            pl.B[o * pl.depth + s] = h[1 + a];
        }
        const std::vector<double> cf = pl.coef();
        SlotList L{};
        L.k = (int)cf.size();
        for (int a = 0; a < L.k; ++a) {
            L.id[a] = pl.order[a];
            L.c[a] = cf[a];
        }
        hipLaunchKernelGGL(k_pulay_mix, dim3(grid_for(ne)), dim3(256), 0, c->stream, ne, slots, L,
                           p->damp_P, Pin);
        GF2_HIP(hipGetLastError());
        want = 0;
        return next_iteration();
    }
    int next_iteration() {
        GF2_TRY(fock_run(c, Pin, F));
        if (++it > p->max_inner) return fail(GF2_ENOCONV, "gf2_iterate: inner loop did not converge");
        tol_pass = pass_tolerance();
        ms.start(p, mu, slope, tol_pass);
        phase = 0;
        return GF2_OK;
    }
};

static int check_dims(gf2_ctx *c, const gf2_dims *d, const char *who) {
    if (!c || !d) return fail(GF2_EINVAL, std::string(who) + ": NULL argument");
    if (!c->has_system) return fail(GF2_ESTATE, std::string(who) + ": no system set");
    if (d->n != c->n) return fail(GF2_EINVAL, std::string(who) + ": dims->n differs from the system");
    if (d->ntau < 4 || d->niw < 1 || !(d->beta > 0.0))
        return fail(GF2_EINVAL, std::string(who) + ": bad dims (ntau >= 4, niw >= 1, beta > 0)");
    if (d->nelec < 0 || d->nelec > 2 * d->n)
        return fail(GF2_EBRACKET, std::string(who) + ": nelec outside [0, 2n]");
    return GF2_OK;
}

static int check_params(const gf2_params *p, const char *who) {
    if (!p) return fail(GF2_EINVAL, std::string(who) + ": params is NULL");
    if (!(p->tol_mu > 0) || !(p->tol_N > 0) || !(p->tol_P > 0) || p->max_inner < 1 ||
        !(p->tol_N_rel >= 0) ||
        p->max_bisect < 1 || !(p->mu_halfwidth > 0) || p->mix_depth < 1 || p->mix_depth > 32 ||
        !(p->damp_P >= 0 && p->damp_P < 1) || !(p->damp_Sigma >= 0 && p->damp_Sigma < 1) ||
        (p->mu_method != GF2_MU_BISECT && p->mu_method != GF2_MU_ILLINOIS &&
         p->mu_method != GF2_MU_SECANT) ||
        p->prec < GF2_PREC_FP64 || p->prec > GF2_PREC_BF16MIX ||
        (p->sigma_df != 0 && p->sigma_df != 1) ||
        (p->sigma_df == 1 && p->prec != GF2_PREC_FP64 && p->prec != GF2_PREC_FP32))
        return fail(GF2_EINVAL, std::string(who) + ": bad parameters");
    return GF2_OK;
}

}  // namespace gf2

using namespace gf2;

extern "C" int gf2_density_fock(gf2_ctx *c, const gf2_dims *d, const gf2_params *p,
                                const double *F_in, const void *Sigma_iw, const double *Sigma1,
                                double *mu_inout, double *P_out, double *F_out, void *G_iw_out,
                                double *host_out) {
    GF2_TRY(check_dims(c, d, "gf2_density_fock"));
    GF2_TRY(check_params(p, "gf2_density_fock"));
    if (!F_in || !mu_inout || !P_out || !host_out)
        return fail(GF2_EINVAL, "gf2_density_fock: NULL argument");
    GF2_HIP(hipSetDevice(c->device));
    const size_t ne = (size_t)c->n * c->n;
    GF2_TRY(c->it_mom.ensure(3 * ne * 8));
    double trPS = 0, e2b = 0;
    int evals = 0;
    double mu = *mu_inout;
    double slope = 0.0;
    GF2_TRY(density_pass(c, d, p, F_in, static_cast<const double2 *>(Sigma_iw), Sigma1, &mu, P_out,
                         static_cast<double2 *>(G_iw_out), c->it_mom.as<double>(), &trPS, &e2b,
                         &evals, &slope));
    *mu_inout = mu;
    double e1b = 0.0;
    if (F_out) {
        GF2_TRY(fock_run(c, P_out, F_out));
        double ph, pf;
        GF2_TRY(dot(c, ne, P_out, c->h.as<double>(), &ph));
        GF2_TRY(dot(c, ne, P_out, F_out, &pf));
        e1b = 0.5 * (ph + pf);
    }
    host_out[0] = trPS;
    host_out[1] = e1b;
    host_out[2] = e2b;
    host_out[3] = (double)evals;
    return GF2_OK;
}

namespace gf2 {

// Steps 3 and the Sigma part of an outer iteration: Sigma(tau) from G(tau),
// damping, Sigma(i w) and Sigma_1.  Iteration 0 (Hartree-Fock) has no Sigma.
static int iter_sigma_prep(gf2_ctx *c, const gf2_dims *d, const gf2_state *st, const double2 **Sig,
                           const double **Sig1, bool *need) {
    const size_t ne = (size_t)c->n * c->n;
    const size_t nt = (size_t)d->ntau * ne;
    GF2_TRY(c->it_Sig1.ensure(ne * 8));
    *Sig = nullptr;
    *Sig1 = nullptr;
    *need = st->iteration != 0;
    if (!*need) return GF2_OK;
    GF2_TRY(c->it_Sig_new.ensure(nt * 8));
    GF2_TRY(c->it_Sig_iw.ensure((size_t)d->niw * ne * 16));
    return GF2_OK;
}

// new Sigma(tau) in it_Sig_new: check, damp, keep, transform to iw
static int iter_sigma_post(gf2_ctx *c, const gf2_dims *d, const gf2_params *p, gf2_state *st,
                           const double2 **Sig, const double **Sig1, double *t_four) {
    const size_t nt = (size_t)d->ntau * c->n * c->n;
    double *Snew = c->it_Sig_new.as<double>();
    // (Sigma(tau) is exactly symmetric: the contraction computes the entries
    // j >= i and copies them to (j, i), so the reduced-precision forms seed no
    // antisymmetric part that the loop would amplify)
    int bad = 0;
    GF2_TRY(any_nonfinite(c, nt, Snew, &bad));
    if (bad) return fail(GF2_ENONFINITE, "gf2_iterate: non-finite self-energy");
    if (st->iteration >= 2 && p->damp_Sigma > 0.0)
        GF2_TRY(axpby(c, nt, p->damp_Sigma, st->Sigma_tau, 1.0 - p->damp_Sigma, Snew));
    GF2_TRY(copy_d2d(c, st->Sigma_tau, Snew, nt * 8));
    const double tf = now_ms();
    GF2_TRY(fourier_tau2iw(c, d, st->Sigma_tau, c->it_Sig_iw.as<double2>(), c->it_Sig1.as<double>()));
    GF2_HIP(hipStreamSynchronize(c->stream));
    *t_four += now_ms() - tf;
    *Sig = c->it_Sig_iw.as<double2>();
    *Sig1 = c->it_Sig1.as<double>();
    return GF2_OK;
}

static int iter_sigma(gf2_ctx *c, const gf2_dims *d, const gf2_params *p, gf2_state *st,
                      const double2 **Sig, const double **Sig1, double *t_sig, double *t_four) {
    bool need;
    GF2_TRY(iter_sigma_prep(c, d, st, Sig, Sig1, &need));
    if (!need) return GF2_OK;
    GF2_HIP(hipStreamSynchronize(c->stream));
    const double ts = now_ms();
    if (p->sigma_df)
        GF2_TRY(sigma_df_run(c, d, p->prec, st->G_tau, c->it_Sig_new.as<double>()));
    else
        GF2_TRY(sigma_run(c, d, p->prec, st->G_tau, c->it_Sig_new.as<double>()));
    GF2_HIP(hipStreamSynchronize(c->stream));
    *t_sig += now_ms() - ts;
    return iter_sigma_post(c, d, p, st, Sig, Sig1, t_four);
}

// End of an outer iteration after the inner loop: F(P_out), E_1b, G(tau),
// state update and report (ms_* filled by the caller).
static int iter_finish(gf2_ctx *c, const gf2_dims *d, gf2_state *st, InnerLoop &il,
                       gf2_report *rep, double *t_four) {
    const size_t ne = (size_t)c->n * c->n;
    double *Pout = il.Pout, *F = il.F;
    GF2_TRY(fock_run(c, Pout, F));
    double ph, pf;
    GF2_TRY(dot(c, ne, Pout, c->h.as<double>(), &ph));
    GF2_TRY(dot(c, ne, Pout, F, &pf));
    const double e1b = 0.5 * (ph + pf);
    const double tf2 = now_ms();
    GF2_TRY(fourier_iw2tau(c, d, il.G_iw, il.mom, st->G_tau));
    GF2_HIP(hipStreamSynchronize(c->stream));
    *t_four += now_ms() - tf2;
    double dP = INFINITY;
    if (st->has_P) GF2_TRY(max_abs_diff(c, ne, Pout, st->P, &dP));
    GF2_TRY(copy_d2d(c, st->P, Pout, ne * 8));
    GF2_TRY(copy_d2d(c, st->F, F, ne * 8));
    GF2_HIP(hipStreamSynchronize(c->stream));
    const double E = e1b + il.e2b;
    rep->energy = E;
    rep->e1b = e1b;
    rep->e2b = il.e2b;
    rep->dE = std::isfinite(st->energy) ? E - st->energy : INFINITY;
    rep->dP = dP;
    rep->mu = il.mu;
    rep->n_inner = il.n_inner;
    rep->n_eval = il.n_eval;
    st->mu = il.mu;
    st->energy = E;
    st->has_P = 1;
    st->iteration += 1;
    return GF2_OK;
}

static int check_state(const gf2_state *st, const gf2_report *rep, const char *who) {
    if (!st || !rep || !st->F || !st->P || !st->G_tau || !st->Sigma_tau)
        return fail(GF2_EINVAL, std::string(who) + ": NULL state array or report");
    return GF2_OK;
}

}  // namespace gf2

extern "C" int gf2_iterate(gf2_ctx *c, const gf2_dims *d, const gf2_params *p, gf2_state *st,
                           gf2_report *rep) {
    GF2_TRY(check_dims(c, d, "gf2_iterate"));
    GF2_TRY(check_params(p, "gf2_iterate"));
    GF2_TRY(check_state(st, rep, "gf2_iterate"));
    if (p->sigma_df && c->df_m < 1)
        return fail(GF2_ESTATE, "gf2_iterate: sigma_df = 1 without density-fitting factors");
    GF2_HIP(hipSetDevice(c->device));
    const double t0 = now_ms();
    double t_sig = 0.0, t_four = 0.0;
    const double2 *Sig = nullptr;
    const double *Sig1 = nullptr;
    GF2_TRY(iter_sigma(c, d, p, st, &Sig, &Sig1, &t_sig, &t_four));

    const double ti = now_ms();
    GF2_TRY(c->it_red.ensure(IL_RED * 8));
    InnerLoop il;
    GF2_TRY(il.start(c, d, p, st, Sig, Sig1, c->it_red.as<double>()));
    while (il.phase != 2) {
        double r2[2];
        if (il.phase == 0) {
            double tn;
            GF2_TRY(dyson_run(c, d, il.density_mode(), il.ms.pending, il.F, Sig, Sig1, il.G_iw,
                              il.Pout, il.mom, r2, &tn));
            GF2_TRY(il.on_eval(tn, r2[0], r2[1]));
        } else if (il.phase == 1) {
            GF2_TRY(dyson_run(c, d, il.density_mode(), il.mu, il.F, Sig, Sig1, il.G_iw, il.Pout,
                              il.mom, r2));
            GF2_TRY(il.on_density(r2[0], r2[1]));
        } else {
            double h[IL_RED];
            GF2_HIP(hipMemcpyAsync(h, il.red, il.red_count() * 8, hipMemcpyDeviceToHost, c->stream));
            GF2_HIP(hipStreamSynchronize(c->stream));
            GF2_TRY(il.on_red(h));
        }
    }
    const double t_inner_end = now_ms();
    GF2_TRY(iter_finish(c, d, st, il, rep, &t_four));
    rep->ms_sigma = t_sig;
    rep->ms_fourier = t_four;
    rep->ms_inner = t_inner_end - ti;
    rep->ms_total = now_ms() - t0;
    return GF2_OK;
}

// Batched sweep: the inner loops of all systems advance in lockstep; every
// round is one dyson_round over all systems that still need a solve.
extern "C" int gf2_iterate_batched(gf2_ctx *const *ctxs, int nsys, const gf2_dims *dims,
                                   const gf2_params *p, gf2_state *states, gf2_report *reps) {
    if (!ctxs || nsys < 1 || !dims || !states || !reps)
        return fail(GF2_EINVAL, "gf2_iterate_batched: NULL argument or nsys < 1");
    GF2_TRY(check_params(p, "gf2_iterate_batched"));
    if (p->sigma_df) return fail(GF2_EINVAL, "gf2_iterate_batched: sigma_df is for gf2_iterate only");
    gf2_ctx *lead = ctxs[0];
    for (int s = 0; s < nsys; ++s) {
        GF2_TRY(check_dims(ctxs[s], &dims[s], "gf2_iterate_batched"));
        GF2_TRY(check_state(&states[s], &reps[s], "gf2_iterate_batched"));
        if (ctxs[s]->device != lead->device)
            return fail(GF2_EINVAL, "gf2_iterate_batched: contexts on different devices");
        for (int t = 0; t < s; ++t)
            if (ctxs[t] == ctxs[s]) return fail(GF2_EINVAL, "gf2_iterate_batched: context repeated");
    }
    GF2_HIP(hipSetDevice(lead->device));
    // everything runs on the lead context's stream
    struct StreamSwap {
        std::vector<hipStream_t> saved;
        gf2_ctx *const *cs;
        int ns;
        ~StreamSwap() {
            for (int s = 0; s < ns; ++s) cs[s]->stream = saved[s];
        }
    } swap{std::vector<hipStream_t>(nsys), ctxs, nsys};
    for (int s = 0; s < nsys; ++s) {
        swap.saved[s] = ctxs[s]->stream;
        GF2_HIP(hipStreamSynchronize(ctxs[s]->stream));
    }
    for (int s = 0; s < nsys; ++s) ctxs[s]->stream = lead->stream;

    const double t0 = now_ms();
    double t_sig = 0.0, t_four = 0.0;
    std::vector<const double2 *> Sig(nsys);
    std::vector<const double *> Sig1(nsys);
    {
        // Sigma(tau) of every system that needs one: one captured graph
        std::vector<gf2_ctx *> cs;
        std::vector<int> nt;
        std::vector<const double *> G;
        std::vector<double *> So;
        for (int s = 0; s < nsys; ++s) {
            bool need;
            GF2_TRY(iter_sigma_prep(ctxs[s], &dims[s], &states[s], &Sig[s], &Sig1[s], &need));
            if (!need) continue;
            cs.push_back(ctxs[s]);
            nt.push_back(dims[s].ntau);
            G.push_back(states[s].G_tau);
            So.push_back(ctxs[s]->it_Sig_new.as<double>());
        }
        if (!cs.empty()) {
            GF2_HIP(hipStreamSynchronize(lead->stream));
            const double ts = now_ms();
            GF2_TRY(sigma_run_batched(lead, cs, nt, p->prec, G, So));
            GF2_HIP(hipStreamSynchronize(lead->stream));
            t_sig += now_ms() - ts;
            for (int s = 0; s < nsys; ++s)
                if (states[s].iteration != 0)
                    GF2_TRY(iter_sigma_post(ctxs[s], &dims[s], p, &states[s], &Sig[s], &Sig1[s], &t_four));
        }
    }

    const double ti = now_ms();
    // reduction arrays of all systems side by side, copied to pinned memory at once
    GF2_TRY(lead->bat_red.ensure((size_t)nsys * IL_RED * 8));
    const size_t red_bytes = (size_t)nsys * IL_RED * 8;
    if (lead->bat_red_h_bytes < red_bytes) {
        if (lead->bat_red_h) (void)hipHostFree(lead->bat_red_h);
        lead->bat_red_h = nullptr;
        lead->bat_red_h_bytes = 0;
        GF2_HIP(hipHostMalloc(&lead->bat_red_h, red_bytes, hipHostMallocDefault));
        lead->bat_red_h_bytes = red_bytes;
    }
    double *red_h = static_cast<double *>(lead->bat_red_h);
    std::vector<InnerLoop> il(nsys);
    for (int s = 0; s < nsys; ++s)
        GF2_TRY(il[s].start(ctxs[s], &dims[s], p, &states[s], Sig[s], Sig1[s],
                            lead->bat_red.as<double>() + (size_t)s * IL_RED));
    std::vector<DysonReq> req(nsys);
    std::vector<double> res;
    std::vector<char> red_wait(nsys);
    for (;;) {
        bool any = false, any_red = false;
        for (int s = 0; s < nsys; ++s) {
            red_wait[s] = il[s].phase == 3;
            any_red |= red_wait[s] != 0;
            DysonReq &q = req[s];
            q = DysonReq{};
            q.c = ctxs[s];
            q.d = &dims[s];
            q.F = il[s].F;
            q.Sig = Sig[s];
            if (il[s].phase == 0 || il[s].phase == 1) {
                q.mode = il[s].density_mode();
                q.mu = il[s].phase == 0 ? il[s].ms.pending : il[s].mu;
                q.Sig1 = Sig1[s];
                q.G_iw = il[s].G_iw;
                q.P = il[s].Pout;
                q.mom = il[s].mom;
                any = true;
            } else {
                q.mode = -1;
            }
        }
        if (!any && !any_red) break;
        // the pending reductions come back with the round of the other systems
        if (any_red)
            GF2_HIP(hipMemcpyAsync(red_h, lead->bat_red.ptr, red_bytes, hipMemcpyDeviceToHost,
                                   lead->stream));
        if (any) GF2_TRY(dyson_round(lead, req, res));
        else GF2_HIP(hipStreamSynchronize(lead->stream));
        for (int s = 0; s < nsys; ++s) {
            const double *r = &res[(size_t)3 * s];
            if (red_wait[s]) GF2_TRY(il[s].on_red(red_h + (size_t)s * IL_RED));
            else if (req[s].mode < 0) continue;
            else if (il[s].phase == 0) GF2_TRY(il[s].on_eval(r[2], r[0], r[1]));
            else GF2_TRY(il[s].on_density(r[0], r[1]));
        }
    }
    const double t_inner = now_ms() - ti;
    for (int s = 0; s < nsys; ++s) GF2_TRY(iter_finish(ctxs[s], &dims[s], &states[s], il[s], &reps[s], &t_four));
    const double t_total = now_ms() - t0;
    for (int s = 0; s < nsys; ++s) {
        reps[s].ms_sigma = t_sig;
        reps[s].ms_fourier = t_four;
        reps[s].ms_inner = t_inner;
        reps[s].ms_total = t_total;
    }
    return GF2_OK;
}
