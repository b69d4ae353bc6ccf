// Imaginary time <-> Matsubara transforms (FP64).
//
// Conventions: G(i w_n) = int_0^beta e^{i w_n tau} G(tau) dtau,
// G(tau) = (1/beta) sum_{n in Z} e^{-i w_n tau} G(i w_n), w_n = (2n+1) pi/beta,
// uniform grid tau_k = k h, h = beta/M, k = 0..M.
//
// TAU -> IW (Sigma):  every element is interpolated by the not-a-knot cubic
// spline through its M+1 samples and the spline's Fourier integral is taken
// exactly interval by interval:
//   Sigma(i w_n) = sum_j e^{i w_n tau_j} sum_k c_kj h^{k+1} mu_k(w_n h),
//   mu_k(t) = int_0^1 s^k e^{i t s} ds.
// Steps: (1) one thread per element solves the spline system along tau
// (uniform spacing: m_1 = r_1/6 and m_{M-1} = r_{M-1}/6 follow from the
// not-a-knot conditions, the rest is a diagonally dominant tridiagonal solve);
// (2) the four sums over j are length-M DFTs in n (e^{i w_n tau_j} is
// M-periodic), done as one FP64 MFMA GEMM against a cos/sin table;
// (3) one block per residue r expands to all n = r (mod M): the write of
// Sigma(i w) is the HBM-bound part.
//
// IW -> TAU (G):  R_n = G_n - G1/(iw) - G2/(iw)^2 - G3/(iw)^3 is folded
// modulo M (the read of G(i w) is the HBM-bound part), then
//   G(tau_k) = (2/beta) sum_r [cos(t_kr) Re F_r + sin(t_kr) Im F_r] + tail(tau_k),
//   t_kr = pi k (2r+1)/M,
// as one FP64 GEMM with K = 2M, and the tail
//   -G1/2 + G2 (2 tau - beta)/4 + G3 (beta tau - tau^2)/4 is added.
//
// Non-equidistant grid (gf2_set_tau_grid; the paper's choice, Implementation
// section): the same spline, integral and tail, but without the M-periodic
// structure the sums over grid points are FP64 MFMA GEMMs against tables
// built once per (grid, niw, beta):
//   TAU -> IW: W[4j + k][n'] = Re / Im of e^{i w_n tau_j} h_j^{k+1} mu_k(w_n h_j)
//              (n' < niw: real part of frequency n', else imaginary part of
//              n' - niw); Sigma(i w) = W^T C, C[4j + k][e] the spline
//              coefficients with h_j = tau_{j+1} - tau_j, K = 4M;
//   IW -> TAU: T[n'][k] = cos(w_n tau_k) / sin(w_n tau_k); G(tau_k) =
//              (2/beta) T^T R + tail(tau_k), R the tail-subtracted G(i w) in
//              planar form [2 niw][n^2], K = 2 niw.
#include "gf2_internal.h"

#include <algorithm>
#include <cmath>

namespace gf2 {

// ---- (1) spline coefficients -------------------------------------------------
// Thomas coefficients of the constant tridiagonal (1, 4, 1) system:
// cp[0] = 1/4, cp[i] = 1/(4 - cp[i-1]); cp[i] is also 1/(pivot i).
__global__ void k_thomas_cp(int nn, double *__restrict__ cp) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    double c = 0.25;
    for (int i = 0; i < nn; ++i) {
        cp[i] = c;
        c = 1.0 / (4.0 - c);
    }
}

// One thread per matrix element e.  Second derivatives m_j (j = 0..M) of the
// not-a-knot spline through Y[0..M][e] go to mwork; the polynomial
// coefficients on interval j go to coef[j][k*ne + e] (k = 0..3).
__global__ void k_spline(int ne, int M, double h, const double *__restrict__ Y,
                         const double *__restrict__ cp, double *__restrict__ coef,
                         double *__restrict__ mwork) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= ne) return;
    const long long s = ne;
    auto y = [&](int j) { return Y[(long long)j * s + e]; };
    auto m = [&](int j) -> double & { return mwork[(long long)j * s + e]; };
    const double c6 = 6.0 / (h * h);
    auto r = [&](int j) { return c6 * (y(j - 1) - 2.0 * y(j) + y(j + 1)); };
    // not-a-knot on a uniform grid: m_0 = 2 m_1 - m_2 turns row 1 into 6 m_1 = r_1
    const double m1 = r(1) / 6.0;
    const double mM1 = r(M - 1) / 6.0;
    m(1) = m1;
    m(M - 1) = mM1;
    if (M >= 4) {
        // rows j = 2..M-2: m_{j-1} + 4 m_j + m_{j+1} = r_j, m_1 and m_{M-1} known
        const int nn = M - 3;
        double dprev = 0.0;
        for (int i = 0; i < nn; ++i) {
            const int j = i + 2;
            double rhs = r(j);
            if (i == 0) rhs -= m1;
            if (i == nn - 1) rhs -= mM1;
            const double dp = (rhs - dprev) * cp[i];
            m(j) = dp;
            dprev = dp;
        }
        double xn = m(M - 2);
        for (int i = nn - 2; i >= 0; --i) {
            const double xi = m(i + 2) - cp[i] * xn;
            m(i + 2) = xi;
            xn = xi;
        }
    }
    m(0) = 2.0 * m(1) - m(2);
    m(M) = 2.0 * m(M - 1) - m(M - 2);
    const long long ld = 4LL * ne;
    for (int j = 0; j < M; ++j) {
        const double y0 = y(j), y1 = y(j + 1), m0 = m(j), m1j = m(j + 1);
        double *row = coef + (long long)j * ld;
        row[e] = y0;
        row[s + e] = (y1 - y0) / h - h * (2.0 * m0 + m1j) / 6.0;
        row[2 * s + e] = 0.5 * m0;
        row[3 * s + e] = (m1j - m0) / (6.0 * h);
    }
}

// ---- twiddle tables --------------------------------------------------------------
// tau->iw: T[j][r'] r' < M: cos(pi (2r+1) j / M), r' >= M: sin(...)   (rows j < M)
__global__ void k_twiddle_t2i(int M, double *__restrict__ T) {
    const long long total = (long long)M * 2 * M;
    for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < total;
         idx += (long long)gridDim.x * blockDim.x) {
        const long long j = idx / (2 * M), rp = idx % (2 * M);
        const long long r = rp < M ? rp : rp - M;
        const long long num = ((2 * r + 1) * j) % (2 * M);
        double sn, cs;
        sincospi((double)num / (double)M, &sn, &cs);
        T[idx] = rp < M ? cs : sn;
    }
}

// iw->tau: T[r'][k] (rows r' < 2M, cols k = 0..M): r' < M: cos(pi k (2r+1)/M), else sin
__global__ void k_twiddle_i2t(int M, double *__restrict__ T) {
    const long long total = 2LL * M * (M + 1);
    for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < total;
         idx += (long long)gridDim.x * blockDim.x) {
        const long long rp = idx / (M + 1), k = idx % (M + 1);
        const long long r = rp < M ? rp : rp - M;
        const long long num = (k * (2 * r + 1)) % (2 * M);
        double sn, cs;
        sincospi((double)num / (double)M, &sn, &cs);
        T[idx] = rp < M ? cs : sn;
    }
}

// mu_k(t) = int_0^1 s^k e^{i t s} ds, k = 0..3
__device__ void unit_moments(double t, double2 mu[4]) {
    if (t < 1.0) {
        // Taylor series sum_p (i t)^p / (p! (p + k + 1))
        double tr = 1.0, ti = 0.0;   // (i t)^p / p!
        double a[4][2] = {{0, 0}, {0, 0}, {0, 0}, {0, 0}};
        for (int p = 0; p < 30; ++p) {
            if (p > 0) {
                // multiply by (i t)/p
                const double nr = -ti * t / p, ni = tr * t / p;
                tr = nr;
                ti = ni;
            }
            for (int k = 0; k < 4; ++k) {
                const double w = 1.0 / (double)(p + k + 1);
                a[k][0] += tr * w;
                a[k][1] += ti * w;
            }
        }
        for (int k = 0; k < 4; ++k) mu[k] = make_double2(a[k][0], a[k][1]);
    } else {
        double sn, cs;
        sincos(t, &sn, &cs);
        // 1/(i t) = -i/t
        const double it = 1.0 / t;
        // m0 = (e - 1)/(i t) = -i (e - 1)/t
        double mr = (sn) * it, mi = -(cs - 1.0) * it;
        mu[0] = make_double2(mr, mi);
        for (int k = 1; k < 4; ++k) {
            const double xr = cs - k * mr, xi = sn - k * mi;   // e - k m
            mr = xi * it;
            mi = -xr * it;
            mu[k] = make_double2(mr, mi);
        }
    }
}

// Table of h^{k+1} mu_k(w_n h) for n < niw: tab[n*4 + k]
__global__ void k_moments_table(int niw, int M, double h, double2 *__restrict__ tab) {
    const int nidx = blockIdx.x * blockDim.x + threadIdx.x;
    if (nidx >= niw) return;
    // w_n h = pi (2n+1)/M, computed from the exact rational
    const double t = M_PI * (double)(2LL * nidx + 1) / (double)M;
    double2 mu[4];
    unit_moments(t, mu);
    double hp = h;
    for (int k = 0; k < 4; ++k) {
        tab[(long long)nidx * 4 + k] = make_double2(hp * mu[k].x, hp * mu[k].y);
        hp *= h;
    }
}

// (3) expansion: out[n][e] = sum_k tab[n][k] * Ck[r][e], n = r + q M
__global__ void k_expand(int ne, int M, int niw, const double *__restrict__ Cmat,
                         const double2 *__restrict__ tab, double2 *__restrict__ out) {
    const int r = blockIdx.y;
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= ne || r >= M || r >= niw) return;
    const long long ld = 4LL * ne;
    double cr[4], ci[4];
    for (int k = 0; k < 4; ++k) {
        cr[k] = Cmat[(long long)r * ld + (long long)k * ne + e];
        ci[k] = Cmat[(long long)(M + r) * ld + (long long)k * ne + e];
    }
    for (long long nn = r; nn < niw; nn += M) {
        double sr = 0.0, si = 0.0;
        for (int k = 0; k < 4; ++k) {
            const double2 t = tab[nn * 4 + k];
            sr += t.x * cr[k] - t.y * ci[k];
            si += t.x * ci[k] + t.y * cr[k];
        }
        out[nn * ne + e] = make_double2(sr, si);
    }
}

__global__ void k_moment1(int ne, int M, const double *__restrict__ Y, double *__restrict__ S1) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= ne) return;
    S1[e] = -(Y[e] + Y[(long long)M * ne + e]);
}

// ---- non-equidistant grid ----------------------------------------------------------
// Thomas factors of the not-a-knot system for the second derivatives m_1 ..
// m_{M-1} (m_0, m_M eliminated by the not-a-knot conditions): row i (unknown
// m_{i+1}) has sub a_i, diagonal b_i, super c_i; thom[3i..3i+2] = a_i, the
// modified super c'_i and 1 / (b_i - a_i c'_{i-1}).
__global__ void k_grid_thomas(int M, const double *__restrict__ tau, double *__restrict__ thom) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    const int nu = M - 1;
    double cprev = 0.0;
    for (int i = 0; i < nu; ++i) {
        const int j = i + 1;
        const double hl = tau[j] - tau[j - 1], hr = tau[j + 1] - tau[j];
        double a = hl, b = 2.0 * (hl + hr), cc = hr;
        if (j == 1) {            // m_0 = (1 + h0/h1) m_1 - (h0/h1) m_2
            b += hl * (1.0 + hl / hr);
            cc -= hl * hl / hr;
            a = 0.0;
        }
        if (j == M - 1) {        // m_M = (1 + hM/hM1) m_{M-1} - (hM/hM1) m_{M-2}
            b += hr * (1.0 + hr / hl);
            a -= hr * hr / hl;
            cc = 0.0;
        }
        const double inv = 1.0 / (b - a * cprev);
        const double cp = cc * inv;
        thom[3 * i] = a;
        thom[3 * i + 1] = cp;
        thom[3 * i + 2] = inv;
        cprev = cp;
    }
}

// One thread per element e: not-a-knot spline through Y[0..M][e] on the grid;
// coefficients of interval j to coef[j][k*ne + e]; mwork holds m_0..m_M.
__global__ void k_grid_spline(int ne, int M, const double *__restrict__ tau,
                              const double *__restrict__ thom, const double *__restrict__ Y,
                              double *__restrict__ coef, double *__restrict__ mwork) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= ne) return;
    const long long s = ne;
    auto y = [&](int j) { return Y[(long long)j * s + e]; };
    auto m = [&](int j) -> double & { return mwork[(long long)j * s + e]; };
    auto slope = [&](int j) { return (y(j + 1) - y(j)) / (tau[j + 1] - tau[j]); };
    // forward sweep over rows i = 0..M-2 (unknown m_{i+1})
    double dprev = 0.0, sl = slope(0);
    for (int i = 0; i < M - 1; ++i) {
        const double sr = slope(i + 1);
        const double r = 6.0 * (sr - sl);
        const double dp = (r - thom[3 * i] * dprev) * thom[3 * i + 2];
        m(i + 1) = dp;
        dprev = dp;
        sl = sr;
    }
    double xn = m(M - 1);
    for (int i = M - 3; i >= 0; --i) {
        const double xi = m(i + 1) - thom[3 * i + 1] * xn;
        m(i + 1) = xi;
        xn = xi;
    }
    const double h0 = tau[1] - tau[0], h1 = tau[2] - tau[1];
    const double hM = tau[M] - tau[M - 1], hM1 = tau[M - 1] - tau[M - 2];
    m(0) = (1.0 + h0 / h1) * m(1) - (h0 / h1) * m(2);
    m(M) = (1.0 + hM / hM1) * m(M - 1) - (hM / hM1) * m(M - 2);
    const long long ld = 4LL * ne;
    for (int j = 0; j < M; ++j) {
        const double h = tau[j + 1] - tau[j];
        const double y0 = y(j), y1 = y(j + 1), m0 = m(j), m1j = m(j + 1);
        double *row = coef + (long long)j * ld;
        row[e] = y0;
        row[s + e] = (y1 - y0) / h - h * (2.0 * m0 + m1j) / 6.0;
        row[2 * s + e] = 0.5 * m0;
        row[3 * s + e] = (m1j - m0) / (6.0 * h);
    }
}

// e^{i pi q x}, x = tau / beta, q odd: the argument reduced mod 2 first
__device__ __forceinline__ void phase_pi(long long q, double x, double &sn, double &cs) {
    double a = fmod((double)q * x, 2.0);
    sincospi(a, &sn, &cs);
}

// W[4j + k][n'] (rows j < M, k < 4; columns n' < 2 niw), one thread per (j, n)
__global__ void k_grid_w(int M, int niw, double beta, const double *__restrict__ tau,
                         double *__restrict__ W) {
    const long long total = (long long)M * niw;
    const long long ldw = 2LL * niw;
    for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < total;
         idx += (long long)gridDim.x * blockDim.x) {
        const int j = (int)(idx / niw), nn = (int)(idx % niw);
        const double h = tau[j + 1] - tau[j];
        const long long q = 2LL * nn + 1;
        const double t = M_PI * (double)q * h / beta;     // w_n h_j
        double2 mu[4];
        unit_moments(t, mu);
        double sn, cs;
        phase_pi(q, tau[j] / beta, sn, cs);                // e^{i w_n tau_j}
        double hp = h;
        for (int k = 0; k < 4; ++k) {
            const double re = hp * (cs * mu[k].x - sn * mu[k].y);
            const double im = hp * (cs * mu[k].y + sn * mu[k].x);
            W[(long long)(4 * j + k) * ldw + nn] = re;
            W[(long long)(4 * j + k) * ldw + niw + nn] = im;
            hp *= h;
        }
    }
}

// T[n'][k] (rows n' < 2 niw, columns k <= M): cos / sin (w_n tau_k)
__global__ void k_grid_t(int ntau, int niw, double beta, const double *__restrict__ tau,
                         double *__restrict__ T) {
    const long long total = (long long)niw * ntau;
    for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < total;
         idx += (long long)gridDim.x * blockDim.x) {
        const int nn = (int)(idx / ntau), k = (int)(idx % ntau);
        double sn, cs;
        phase_pi(2LL * nn + 1, tau[k] / beta, sn, cs);
        T[(long long)nn * ntau + k] = cs;
        T[(long long)(niw + nn) * ntau + k] = sn;
    }
}

// Sig_iw[n][e] = P[n][e] + i P[niw + n][e]
__global__ void k_grid_interleave(long long ne, int niw, const double *__restrict__ P,
                                  double2 *__restrict__ out) {
    const long long total = (long long)niw * ne;
    for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < total;
         idx += (long long)gridDim.x * blockDim.x)
        out[idx] = make_double2(P[idx], P[total + idx]);
}

// planar R: R[n][e] = Re, R[niw + n][e] = Im of G_n - G1/(iw) - G2/(iw)^2 - G3/(iw)^3
__global__ void k_grid_residual(int ne, int niw, double beta, const double2 *__restrict__ G,
                                const double *__restrict__ mom, double *__restrict__ R) {
    const long long total = (long long)niw * ne;
    for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < total;
         idx += (long long)gridDim.x * blockDim.x) {
        const long long nn = idx / ne, e = idx % ne;
        const double iw1 = beta / (M_PI * (double)(2 * nn + 1));   // 1/w_n
        const double2 x = G[idx];
        R[idx] = x.x + mom[ne + e] * iw1 * iw1;
        R[total + idx] = x.y + mom[e] * iw1 - mom[2 * ne + e] * iw1 * iw1 * iw1;
    }
}

__global__ void k_grid_add_tail(int ne, int ntau, double beta, const double *__restrict__ tau,
                                const double *__restrict__ mom, double *__restrict__ Gt) {
    const long long total = (long long)ntau * ne;
    for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < total;
         idx += (long long)gridDim.x * blockDim.x) {
        const long long k = idx / ne, e = idx % ne;
        const double t = tau[k];
        Gt[idx] += -0.5 * mom[e] + mom[ne + e] * (2.0 * t - beta) / 4.0 +
                   mom[2 * ne + e] * (beta * t - t * t) / 4.0;
    }
}

static unsigned grid_blocks(long long total) {
    return (unsigned)std::min<long long>((total + 255) / 256, 16384);
}

static int grid_check(gf2_ctx *c, const gf2_dims *d) {
    if (d->ntau != c->grid_ntau)
        return fail(GF2_EINVAL, "gf2_fourier: dims->ntau differs from the tau grid set on the context");
    const double tM = c->grid_host.back();
    if (!(std::fabs(tM - d->beta) <= 1e-12 * d->beta))
        return fail(GF2_EINVAL, "gf2_fourier: the tau grid ends at " + std::to_string(tM) +
                                    ", not at beta");
    return GF2_OK;
}

static int fourier_tau2iw_grid(gf2_ctx *c, const gf2_dims *d, const double *Sig_tau,
                               double2 *Sig_iw, double *Sig1) {
    GF2_TRY(grid_check(c, d));
    const int n = d->n, M = d->ntau - 1, niw = d->niw;
    const int ne = n * n;
    const double *tau = c->grid_tau.as<double>();
    GF2_TRY(c->grid_coef.ensure(((size_t)M * 4 + M + 1) * ne * 8));
    GF2_TRY(c->grid_plan.ensure((size_t)2 * niw * ne * 8));
    double *coef = c->grid_coef.as<double>();
    double *mwork = coef + (size_t)M * 4 * ne;
    double *Pl = c->grid_plan.as<double>();
    if (c->grid_w_niw != niw || c->grid_w_beta != d->beta) {
        GF2_TRY(c->grid_W.ensure((size_t)4 * M * 2 * niw * 8));
        hipLaunchKernelGGL(k_grid_w, dim3(grid_blocks((long long)M * niw)), dim3(256), 0,
                           c->stream, M, niw, d->beta, tau, c->grid_W.as<double>());
        GF2_HIP(hipGetLastError());
        c->grid_w_niw = niw;
        c->grid_w_beta = d->beta;
    }
    hipLaunchKernelGGL(k_grid_spline, dim3((ne + 127) / 128), dim3(128), 0, c->stream, ne, M, tau,
                       c->grid_thom.as<double>(), Sig_tau, coef, mwork);
    GF2_HIP(hipGetLastError());
    const int ph = prof_begin(c, GF2_KC_T2I_EXPAND);
    // Pl[n'][e] = sum_{4j+k} W[4j+k][n'] coef[j][k*ne + e]
    GemmArgsF64 g{c->grid_W.as<double>(), 2LL * niw, coef, (long long)ne, Pl, (long long)ne,
                  2 * niw, ne, 4 * M, 1.0};
    GF2_TRY(gemm_f64_kmajor(c, g));
    hipLaunchKernelGGL(k_grid_interleave, dim3(grid_blocks((long long)niw * ne)), dim3(256), 0,
                       c->stream, (long long)ne, niw, Pl, Sig_iw);
    prof_end(c, ph, 16.0 * (double)ne * niw);
    if (Sig1)
        hipLaunchKernelGGL(k_moment1, dim3((ne + 255) / 256), dim3(256), 0, c->stream, ne, M,
                           Sig_tau, Sig1);
    GF2_HIP(hipGetLastError());
    return GF2_OK;
}

int fourier_tau2iw(gf2_ctx *c, const gf2_dims *d, const double *Sig_tau, double2 *Sig_iw,
                   double *Sig1) {
    if (c->grid_ntau > 0) return fourier_tau2iw_grid(c, d, Sig_tau, Sig_iw, Sig1);
    const int n = d->n, M = d->ntau - 1, niw = d->niw;
    const int ne = n * n;
    const double h = d->beta / M;
    // buffers: coef [M][4ne], mwork [M+1][ne], C [2M][4ne], twiddle [M][2M], table [niw][4]
    const size_t coef_b = (size_t)M * 4 * ne * 8;
    const size_t mw_b = (size_t)(M + 1) * ne * 8;
    const size_t C_b = (size_t)2 * M * 4 * ne * 8;
    const size_t tw_b = (size_t)M * 2 * M * 8;
    const size_t tab_b = (size_t)niw * 4 * 16;
    const size_t cp_b = (size_t)std::max(M, 1) * 8;
    GF2_TRY(c->four_c.ensure(coef_b + mw_b + cp_b));
    GF2_TRY(c->four_C.ensure(C_b));
    GF2_TRY(c->four_twid.ensure(tw_b + tab_b));
    double *coef = c->four_c.as<double>();
    double *mwork = coef + (size_t)M * 4 * ne;
    double *cp = mwork + (size_t)(M + 1) * ne;
    double *Cm = c->four_C.as<double>();
    double *tw = c->four_twid.as<double>();
    double2 *tab = reinterpret_cast<double2 *>(tw + (size_t)M * 2 * M);

    hipLaunchKernelGGL(k_thomas_cp, dim3(1), dim3(64), 0, c->stream, std::max(M - 3, 0), cp);
    hipLaunchKernelGGL(k_spline, dim3((ne + 127) / 128), dim3(128), 0, c->stream, ne, M, h, Sig_tau,
                       cp, coef, mwork);
    {
        const long long tot = (long long)M * 2 * M;
        const unsigned blocks = (unsigned)std::min<long long>((tot + 255) / 256, 8192);
        hipLaunchKernelGGL(k_twiddle_t2i, dim3(blocks), dim3(256), 0, c->stream, M, tw);
    }
    hipLaunchKernelGGL(k_moments_table, dim3((niw + 255) / 256), dim3(256), 0, c->stream, niw, M, h,
                       tab);
    GF2_HIP(hipGetLastError());
    // C[r'][kk*ne + e] = sum_j T[j][r'] coef[j][kk*ne + e]
    GemmArgsF64 g{tw, 2LL * M, coef, 4LL * ne, Cm, 4LL * ne, 2 * M, 4 * ne, M, 1.0};
    GF2_TRY(gemm_f64_kmajor(c, g));
    const int nr = std::min(M, niw);
    const int ph = prof_begin(c, GF2_KC_T2I_EXPAND);
    hipLaunchKernelGGL(k_expand, dim3((ne + 255) / 256, nr), dim3(256), 0, c->stream, ne, M, niw,
                       Cm, tab, Sig_iw);
    prof_end(c, ph, 16.0 * (double)ne * niw);
    if (Sig1)
        hipLaunchKernelGGL(k_moment1, dim3((ne + 255) / 256), dim3(256), 0, c->stream, ne, M,
                           Sig_tau, Sig1);
    GF2_HIP(hipGetLastError());
    return GF2_OK;
}

// ---- iw -> tau -------------------------------------------------------------------
// fold: Fre[r][e] = sum_{n = r mod M} Re R_n, Fim likewise
__global__ void k_fold(int ne, int M, int niw, double beta, const double2 *__restrict__ G,
                       const double *__restrict__ mom, double *__restrict__ Fre,
                       double *__restrict__ Fim) {
    const int r = blockIdx.y;
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= ne) return;
    const double g1 = mom[e], g2 = mom[ne + e], g3 = mom[2 * ne + e];
    double sr = 0.0, si = 0.0;
    for (long long nn = r; nn < niw; nn += M) {
        const double w = M_PI * (double)(2 * nn + 1) / beta;
        const double iw1 = 1.0 / w;
        const double2 x = G[nn * ne + e];
        // R = G + i G1/w + G2/w^2 - i G3/w^3
        sr += x.x + g2 * iw1 * iw1;
        si += x.y + g1 * iw1 - g3 * iw1 * iw1 * iw1;
    }
    Fre[(long long)r * ne + e] = sr;
    Fim[(long long)r * ne + e] = si;
}

__global__ void k_add_tail(int ne, int ntau, double beta, const double *__restrict__ mom,
                           double *__restrict__ Gt) {
    const long long total = (long long)ntau * ne;
    const int M = ntau - 1;
    for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < total;
         idx += (long long)gridDim.x * blockDim.x) {
        const long long k = idx / ne, e = idx % ne;
        const double tau = beta * (double)k / (double)M;
        Gt[idx] += -0.5 * mom[e] + mom[ne + e] * (2.0 * tau - beta) / 4.0 +
                   mom[2 * ne + e] * (beta * tau - tau * tau) / 4.0;
    }
}

static int fourier_iw2tau_grid(gf2_ctx *c, const gf2_dims *d, const double2 *G_iw,
                               const double *mom, double *G_tau) {
    GF2_TRY(grid_check(c, d));
    const int n = d->n, niw = d->niw, ntau = d->ntau;
    const int ne = n * n;
    const double *tau = c->grid_tau.as<double>();
    GF2_TRY(c->grid_plan.ensure((size_t)2 * niw * ne * 8));
    double *R = c->grid_plan.as<double>();
    if (c->grid_t_niw != niw || c->grid_t_beta != d->beta) {
        GF2_TRY(c->grid_T.ensure((size_t)2 * niw * ntau * 8));
        hipLaunchKernelGGL(k_grid_t, dim3(grid_blocks((long long)niw * ntau)), dim3(256), 0,
                           c->stream, ntau, niw, d->beta, tau, c->grid_T.as<double>());
        GF2_HIP(hipGetLastError());
        c->grid_t_niw = niw;
        c->grid_t_beta = d->beta;
    }
    const int ph = prof_begin(c, GF2_KC_I2T_FOLD);
    hipLaunchKernelGGL(k_grid_residual, dim3(grid_blocks((long long)niw * ne)), dim3(256), 0,
                       c->stream, ne, niw, d->beta, G_iw, mom, R);
    prof_end(c, ph, 16.0 * (double)ne * niw);
    GF2_HIP(hipGetLastError());
    // G_tau[k][e] = (2/beta) sum_{n'} T[n'][k] R[n'][e]
    GemmArgsF64 g{c->grid_T.as<double>(), (long long)ntau, R, (long long)ne, G_tau, (long long)ne,
                  ntau, ne, 2 * niw, 2.0 / d->beta};
    GF2_TRY(gemm_f64_kmajor(c, g));
    hipLaunchKernelGGL(k_grid_add_tail, dim3(grid_blocks((long long)ntau * ne)), dim3(256), 0,
                       c->stream, ne, ntau, d->beta, tau, mom, G_tau);
    GF2_HIP(hipGetLastError());
    return GF2_OK;
}

int fourier_iw2tau(gf2_ctx *c, const gf2_dims *d, const double2 *G_iw, const double *mom,
                   double *G_tau) {
    if (c->grid_ntau > 0) return fourier_iw2tau_grid(c, d, G_iw, mom, G_tau);
    const int n = d->n, M = d->ntau - 1, niw = d->niw, ntau = d->ntau;
    const int ne = n * n;
    const size_t F_b = (size_t)2 * M * ne * 8;
    const size_t tw_b = (size_t)2 * M * (M + 1) * 8;
    GF2_TRY(c->four_fold.ensure(F_b + tw_b));
    double *Fre = c->four_fold.as<double>();
    double *Fim = Fre + (size_t)M * ne;
    double *tw = Fre + (size_t)2 * M * ne;
    const int ph = prof_begin(c, GF2_KC_I2T_FOLD);
    hipLaunchKernelGGL(k_fold, dim3((ne + 255) / 256, M), dim3(256), 0, c->stream, ne, M, niw,
                       d->beta, G_iw, mom, Fre, Fim);
    prof_end(c, ph, 16.0 * (double)ne * niw);
    {
        const long long tot = 2LL * M * (M + 1);
        const unsigned blocks = (unsigned)std::min<long long>((tot + 255) / 256, 8192);
        hipLaunchKernelGGL(k_twiddle_i2t, dim3(blocks), dim3(256), 0, c->stream, M, tw);
    }
    GF2_HIP(hipGetLastError());
    // G_tau[k][e] = (2/beta) sum_{r'} T[r'][k] F[r'][e]
    GemmArgsF64 g{tw, (long long)(M + 1), Fre, (long long)ne, G_tau, (long long)ne, ntau, ne,
                  2 * M, 2.0 / d->beta};
    GF2_TRY(gemm_f64_kmajor(c, g));
    {
        const long long tot = (long long)ntau * ne;
        const unsigned blocks = (unsigned)std::min<long long>((tot + 255) / 256, 8192);
        hipLaunchKernelGGL(k_add_tail, dim3(blocks), dim3(256), 0, c->stream, ne, ntau, d->beta,
                           mom, G_tau);
    }
    GF2_HIP(hipGetLastError());
    return GF2_OK;
}

}  // namespace gf2

using namespace gf2;

extern "C" int gf2_set_tau_grid(gf2_ctx *c, int ntau, const double *tau) {
    if (!c) return fail(GF2_EINVAL, "gf2_set_tau_grid: ctx is NULL");
    if (ntau == 0) {
        c->grid_ntau = 0;
        c->grid_host.clear();
        return GF2_OK;
    }
    if (ntau < 4 || !tau) return fail(GF2_EINVAL, "gf2_set_tau_grid: needs ntau >= 4 and tau");
    GF2_HIP(hipSetDevice(c->device));
    std::vector<double> h((size_t)ntau);
    GF2_HIP(hipMemcpyAsync(h.data(), tau, (size_t)ntau * 8, hipMemcpyDeviceToHost, c->stream));
    GF2_HIP(hipStreamSynchronize(c->stream));
    const int M = ntau - 1;
    const double tM = h[M];
    if (h[0] != 0.0 || !(tM > 0.0) || !std::isfinite(tM))
        return fail(GF2_EINVAL, "gf2_set_tau_grid: the grid must start at 0 and end at beta > 0");
    for (int k = 0; k < M; ++k)
        if (!(h[k + 1] > h[k])) return fail(GF2_EINVAL, "gf2_set_tau_grid: tau must increase");
    for (int k = 0; k <= M; ++k)
        if (!(std::fabs(h[k] + h[M - k] - tM) <= 1e-12 * tM))
            return fail(GF2_EINVAL, "gf2_set_tau_grid: the grid must be symmetric about beta/2");
    GF2_TRY(c->grid_tau.ensure((size_t)ntau * 8));
    GF2_TRY(c->grid_thom.ensure((size_t)3 * M * 8));
    GF2_HIP(hipMemcpyAsync(c->grid_tau.ptr, h.data(), (size_t)ntau * 8, hipMemcpyHostToDevice,
                           c->stream));
    hipLaunchKernelGGL(k_grid_thomas, dim3(1), dim3(64), 0, c->stream, M, c->grid_tau.as<double>(),
                       c->grid_thom.as<double>());
    GF2_HIP(hipGetLastError());
    GF2_HIP(hipStreamSynchronize(c->stream));   // h goes out of scope
    c->grid_host = std::move(h);
    c->grid_ntau = ntau;
    c->grid_w_niw = c->grid_t_niw = 0;
    c->grid_w_beta = c->grid_t_beta = 0.0;
    return GF2_OK;
}

extern "C" int gf2_fourier(gf2_ctx *c, const gf2_dims *d, int dir, const void *in,
                           const double *moments, void *out, double *moment1_out) {
    if (!c || !d || !in || !out) return fail(GF2_EINVAL, "gf2_fourier: NULL argument");
    if (d->n < 1 || d->ntau < 4 || d->niw < 1 || !(d->beta > 0.0))
        return fail(GF2_EINVAL, "gf2_fourier: bad dims (n >= 1, ntau >= 4, niw >= 1, beta > 0)");
    GF2_HIP(hipSetDevice(c->device));
    if (dir == GF2_TAU2IW)
        return fourier_tau2iw(c, d, static_cast<const double *>(in), static_cast<double2 *>(out),
                              moment1_out);
    if (dir == GF2_IW2TAU) {
        if (!moments) return fail(GF2_EINVAL, "gf2_fourier: IW2TAU needs the tail moments");
        return fourier_iw2tau(c, d, static_cast<const double2 *>(in), moments,
                              static_cast<double *>(out));
    }
    return fail(GF2_EINVAL, "gf2_fourier: bad direction");
}
