// Scalar controller of AMP-PCG: the attainable-accuracy indicator eta_k, the
// latched precision selector and the dynamic-scaling exponent.  Compiled both
// for the device (it runs in the last work-group of the update kernel) and
// for the host (amp_selector_replay), so the two evaluate identical
// floating-point expressions.  Contraction into fused multiply-adds is
// disabled here so that host and device round the same way.
#pragma once

#include <math.h>
#include <stdint.h>

#if defined(__HIPCC__)
#define AMP_HD __host__ __device__
#else
#define AMP_HD
#endif

namespace amp {

constexpr double kEps32 = 5.9604644775390625e-08;  // 2^-24, unit roundoff of IEEE single
constexpr int kRing = 128;                          // residual-norm window (d, ell <= 100)

enum Status : int { RUNNING = 0, CONVERGED = 1, NEED_VERIFY = 2, MAXIT = 3, BREAKDOWN = 4 };
enum EtaMode : int { ETA_DELAY = 0, ETA_LINEAR = 1, UR_FIXED64 = 2, UR_FIXED32 = 3 };
enum Scaling : int { SCALE_POW2 = 0, SCALE_PAPER = 1, SCALE_NONE = 2 };

// Everything the device iteration needs besides the vectors.  Lives in device
// memory; written only by single threads in kernel epilogues.
struct Ctrl {
    // configuration (set by the host before the solve)
    int u0, eta_mode, d, ell, scaling, T_z, T_p, maxit, rr_period, verify, max_repl, chebyshev;
    double C, tau_zs, tau_zh, tol, gain;
    int extra16;            // log2 of the FP16 preconditioner data's static scale
    int pad0;
    // iteration state
    int k;                  // current iteration index
    int status;             // Status
    int iters;              // completed iterations
    int uz, ur;             // precisions of iteration k (latched)
    int r_store, p_store;   // precision in which r_k and p_{k-1} are held
    int k_z32, k_z16, k_r32, n_repl;
    int e, e_prev, have_e;  // pow2 scaling exponents
    int rr_pending;         // a periodic replacement completes the current iteration
    double bnorm, tol_b;
    double rho, rho_prev, beta, gamma, alpha;
    double delta;           // ||r_k||
    double maxr, maxr_prev; // max|r_k|, max|r_{k-1}|
    double maxz, maxp;      // max|z^_{k-1}|, max|p^_{k-1}|
    double omega_eff;       // multiplier applied to r_k (includes the static storage scale)
    double true_res;        // last FP64 true residual norm
    double ring[kRing];     // ||r_t|| for the last kRing iterations
    // reduction plumbing
    unsigned int counter;
    unsigned int pad2;
    unsigned long long maxbits[4];  // atomicMax targets (bit patterns of non-negative doubles)
    double *delta_history;  // nullable
    int32_t *prec_history;  // nullable
};

// ceil(log2(v)) for finite v > 0, exact (no libm rounding).
AMP_HD inline int ceil_log2(double v) {
    int e;
    double m = frexp(v, &e);  // v = m 2^e, m in [0.5, 1)
    return (m == 0.5) ? e - 1 : e;
}

#pragma clang fp contract(off)

// eq. (eta_k): eps32 * sum_{t=k-d}^{k} ((3+C) delta_{t-1} + (2+C) delta_t);
// +inf while the window reaches before t = 0.
AMP_HD inline double eta_delay(const double *ring, int k, int d, double C) {
    if (k - d - 1 < 0) return INFINITY;
    double s = 0.0;
    for (int t = k - d; t <= k; ++t)
        s = s + ((3.0 + C) * ring[(t - 1) % kRing] + (2.0 + C) * ring[t % kRing]);
    return kEps32 * s;
}

// eq. (linear criterion): eps32 (5+2C) delta_{k-1} / (1 - rate),
// rate = (delta_k / delta_{k-ell})^(1/ell); +inf when undefined or rate >= 1.
AMP_HD inline double eta_linear(const double *ring, int k, int ell, double C) {
    if (k < ell || k < 1) return INFINITY;
    double den = ring[(k - ell) % kRing];
    if (!(den > 0.0)) return INFINITY;
    double rate = pow(ring[k % kRing] / den, 1.0 / (double)ell);
    if (!(rate < 1.0)) return INFINITY;
    return kEps32 * (5.0 + 2.0 * C) * ring[(k - 1) % kRing] / (1.0 - rate);
}

AMP_HD inline double eta_value(const Ctrl &c, int k) {
    switch (c.eta_mode) {
        case ETA_DELAY: return eta_delay(c.ring, k, c.d, c.C);
        case ETA_LINEAR: return eta_linear(c.ring, k, c.ell, c.C);
        case UR_FIXED32: return -INFINITY;
        default: return INFINITY;
    }
}

AMP_HD inline int lower_prec(int a, int b) { return a < b ? a : b; }

// eq. (precision_selector); the u_r switch uses eq. (precision switch
// criterion): FP32 once eta <= tol ||b||.
AMP_HD inline void select_precision(double nu, int u0, double tau_zs, double tau_zh, double eta,
                                    double tol_b, int *uz, int *ur) {
    if (nu >= tau_zs) *uz = u0;
    else if (nu >= tau_zh) *uz = lower_prec(u0, 32);
    else *uz = lower_prec(u0, 16);
    *ur = (eta <= tol_b) ? 32 : 64;
}

// Decide (u_z, u_r, omega) of iteration k from delta_k = c.delta, max|r_k| =
// c.maxr and the previous iteration's maxima.  Latched: precisions never rise.
AMP_HD inline void prepare_iteration(Ctrl &c, int k) {
    c.k = k;
    double eta = eta_value(c, k);
    int suz, sur;
    select_precision(c.delta / c.bnorm, c.u0, c.tau_zs, c.tau_zh, eta, c.tol_b, &suz, &sur);
    c.uz = lower_prec(c.uz, suz);
    c.ur = lower_prec(c.ur, sur);
    if (c.uz <= 32 && c.k_z32 < 0) c.k_z32 = k;
    if (c.uz <= 16 && c.k_z16 < 0) c.k_z16 = k;
    if (c.ur <= 32 && c.k_r32 < 0) c.k_r32 = k;
    if (c.prec_history) c.prec_history[k] = c.uz | (c.ur << 8);

    double omega;
    if (c.scaling == SCALE_PAPER) {
        omega = 1.0 / c.delta;
    } else if (c.scaling == SCALE_NONE) {
        omega = 1.0;
    } else {
        int e;
        if (!(c.maxr > 0.0)) {
            e = c.have_e ? c.e : 0;
        } else if (!c.chebyshev || k == 0 || !(c.maxz > 0.0) || !c.have_e) {
            e = c.T_z - ceil_log2(c.maxr * c.gain);
        } else {
            e = c.e + c.T_z - ceil_log2(c.maxz * c.maxr / c.maxr_prev);
        }
        if (k > 0 && c.have_e && c.maxp > 0.0) {
            int ep = c.e + c.T_p - ceil_log2(c.maxp);
            e = e < ep ? e : ep;
        }
        c.e_prev = c.e;
        c.e = e;
        c.have_e = 1;
        omega = ldexp(1.0, e);
    }
    int extra = (c.uz == 16) ? c.extra16 : 0;
    c.omega_eff = ldexp(omega, -extra);
}

#pragma clang fp contract(on)

}  // namespace amp
