// Scalar controller of AMP-PCG: the attainable-accuracy indicator eta_k, the
// latched precision selector and the dynamic-scaling exponent.  Compiled both
// for the device (every work-group of the preconditioning kernel evaluates it
// redundantly from the same inputs) and for the host (amp_selector_replay),
// so all of them evaluate identical floating-point expressions.  Contraction
// into fused multiply-adds is disabled here so host and device round alike.
#pragma once

#include <math.h>
#include <stdint.h>

#if defined(__HIPCC__)
#define AMP_HD __host__ __device__
#else
#define AMP_HD
#endif
// branch hints: the common path of an iteration is laid out contiguously
#define AMP_LIKELY(x) __builtin_expect(!!(x), 1)
#define AMP_UNLIKELY(x) __builtin_expect(!!(x), 0)

namespace amp {

constexpr double kEps32 = 5.9604644775390625e-08;  // 2^-24, unit roundoff of IEEE single
constexpr int kRing = 128;                          // residual-norm window (d, ell <= 100)

enum Status : int { RUNNING = 0, CONVERGED = 1, NEED_VERIFY = 2, MAXIT = 3, BREAKDOWN = 4 };
enum EtaMode : int { ETA_DELAY = 0, ETA_LINEAR = 1, UR_FIXED64 = 2, UR_FIXED32 = 3 };
enum Scaling : int { SCALE_POW2 = 0, SCALE_PAPER = 1, SCALE_NONE = 2 };
// What the residual partial sums entering the preconditioning kernel hold.
enum ResKind : int { RES_INIT = 0, RES_UPDATE = 1, RES_VERIFY = 2, RES_PERIODIC = 3 };

// Solve configuration: constant during a solve, passed to kernels by value.
struct Cfg {
    int u0, eta_mode, d, ell, scaling, T_z, T_p, maxit, verify, max_repl, chebyshev, diff;
    int rr_period, extra16;   // extra16: log2 of the FP16 preconditioner data's static scale
    int defer_x;              // 1: x is updated every other iteration (two steps at once)
    int rr_switch;            // 1: r is replaced by fl32(b - A x) at the u_r switch
    int zero_q;               // 1: the update clears q after reading it (matrix-free product; x every iteration)
    int g_stream, g_slice;    // work-groups of the streaming / sliced-ELL kernels (= partial counts)
    int g_pre;                // partials written by the preconditioning stage
    double C, tau_zs, tau_zh, tol, gain;
    double *ring;             // ||r_t|| for the last kRing iterations (device)
    double *delta_history;    // nullable
    int32_t *prec_history;    // nullable
    double *scalar_history;   // nullable: omega, rho, gamma, alpha per iteration
    int32_t *spmv_iter;       // nullable: iteration index each product launch performed (-1: passed through)
    int spmv_launch;          // index of this launch in spmv_iter
};

// Iteration state.  Each kernel reads the state its predecessor wrote and
// work-group 0 writes the successor state to a different buffer, so no
// kernel reads what it writes.
struct St {
    int k;                    // current iteration index
    int status;               // Status
    int iters;                // completed iterations
    int uz, ur;               // precisions of iteration k (latched)
    int r_store, p_store;     // precision in which r_k and p_{k-1} are held
    int pbuf;                 // which of the two p buffers holds p_{k-1}
    int k_z32, k_z16, k_r32, n_repl;
    int e, have_e;            // pow2 scaling exponent of iteration k
    int kind;                 // ResKind of the pending residual partials
    int xp;                   // 1: x lacks alpha_{k-1} p_{k-1} (deferred to the next update)
    int x_pu, x_pb;           // precision and buffer of that p
    double omega;             // omega_k (without the static storage scale)
    double bnorm, tol_b;
    double rho, rho_prev, beta, gamma, alpha;
    double delta;             // ||r_k||
    double maxr, maxr_prev;   // max|r_k|, max|r_{k-1}|
    double maxz, maxp;        // max|z^_{k-1}|, max|p^_{k-1}|
    double omega_eff;         // multiplier applied to r_k (includes the static storage scale)
    double true_res;          // last FP64 true residual norm
    double x_alpha;           // the alpha of the deferred x update
};

// ceil(log2(v)) for finite v > 0, exact (no libm rounding).
AMP_HD inline int ceil_log2(double v) {
    int e;
    double m = frexp(v, &e);  // v = m 2^e, m in [0.5, 1)
    return (m == 0.5) ? e - 1 : e;
}

// (the library is compiled with -ffp-contract=off; the pragma keeps this
// header exact when it is included elsewhere)
#pragma clang fp contract(off)

// eq. (eta_k): eps32 * sum_{t=k-d}^{k} ((3+C) delta_{t-1} + (2+C) delta_t);
// +inf while the window reaches before t = 0.  ring[t % kRing] = delta_t for
// t < k; delta_k is passed separately.
AMP_HD inline double eta_delay(const double *ring, int k, int d, double C, double delta_k) {
    if (k - d - 1 < 0) return INFINITY;
    double s = 0.0;
    for (int t = k - d; t <= k; ++t) {
        const double dt = (t == k) ? delta_k : ring[t % kRing];
        s = s + ((3.0 + C) * ring[(t - 1) % kRing] + (2.0 + C) * dt);
    }
    return kEps32 * s;
}

// eq. (linear criterion): eps32 (5+2C) delta_{k-1} / (1 - rate),
// rate = (delta_k / delta_{k-ell})^(1/ell); +inf when undefined or rate >= 1.
AMP_HD inline double eta_linear(const double *ring, int k, int ell, double C, double delta_k) {
    if (k < ell || k < 1) return INFINITY;
    double den = ring[(k - ell) % kRing];
    if (!(den > 0.0)) return INFINITY;
    double rate = pow(delta_k / den, 1.0 / (double)ell);
    if (!(rate < 1.0)) return INFINITY;
    return kEps32 * (5.0 + 2.0 * C) * ring[(k - 1) % kRing] / (1.0 - rate);
}

AMP_HD inline double eta_value(const Cfg &c, const double *ring, int k, double delta_k) {
    switch (c.eta_mode) {
        case ETA_DELAY: return eta_delay(ring, k, c.d, c.C, delta_k);
        case ETA_LINEAR: return eta_linear(ring, k, c.ell, c.C, delta_k);
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

// Decide (u_z, u_r, omega) of iteration k from delta_k = s.delta, max|r_k| =
// s.maxr and the previous iteration's maxima.  Latched: precisions never rise.
// eta_pre: the delay indicator of (k, delta_k) when the caller has already
// formed it (the device does, in parallel), else null.
AMP_HD inline void prepare_iteration(St &s, const Cfg &c, const double *ring, int k,
                                     const double *eta_pre = nullptr) {
    s.k = k;
    double eta = AMP_LIKELY(eta_pre && c.eta_mode == ETA_DELAY) ? *eta_pre : eta_value(c, ring, k, s.delta);
    int suz, sur;
    select_precision(s.delta / s.bnorm, c.u0, c.tau_zs, c.tau_zh, eta, s.tol_b, &suz, &sur);
    s.uz = lower_prec(s.uz, suz);
    s.ur = lower_prec(s.ur, sur);
    if (s.uz <= 32 && s.k_z32 < 0) s.k_z32 = k;
    if (s.uz <= 16 && s.k_z16 < 0) s.k_z16 = k;
    if (s.ur <= 32 && s.k_r32 < 0) s.k_r32 = k;

    double omega;
    if (AMP_UNLIKELY(c.scaling == SCALE_PAPER)) {
        omega = 1.0 / s.delta;
    } else if (AMP_UNLIKELY(c.scaling == SCALE_NONE)) {
        omega = 1.0;
    } else {
        int e;
        if (!(s.maxr > 0.0)) {
            e = s.have_e ? s.e : 0;
        } else if (!c.chebyshev || k == 0 || !(s.maxz > 0.0) || !s.have_e) {
            e = c.T_z - ceil_log2(s.maxr * c.gain);
        } else {
            e = s.e + c.T_z - ceil_log2(s.maxz * s.maxr / s.maxr_prev);
        }
        if (k > 0 && s.have_e && s.maxp > 0.0) {
            int ep = s.e + c.T_p - ceil_log2(s.maxp);
            e = e < ep ? e : ep;
        }
        s.e = e;
        s.have_e = 1;
        omega = ldexp(1.0, e);
    }
    s.omega = omega;
    int extra = (s.uz == 16) ? c.extra16 : 0;
    s.omega_eff = ldexp(omega, -extra);
}

// Consume the residual of the iteration just finished (iteration iters-1):
// test for convergence and prepare the next iteration.
AMP_HD inline void finish_iteration(St &s, const Cfg &c, const double *ring, double delta_new,
                                    double maxr_new, const double *eta_pre = nullptr) {
    s.maxr_prev = s.maxr;
    s.maxr = maxr_new;
    s.delta = delta_new;
    if (AMP_UNLIKELY(delta_new <= s.tol_b)) {
        s.status = c.verify ? NEED_VERIFY : CONVERGED;
        return;
    }
    if (AMP_UNLIKELY(!isfinite(delta_new))) {
        s.status = BREAKDOWN;
        return;
    }
    if (AMP_UNLIKELY(s.iters >= c.maxit)) {
        s.status = MAXIT;
        return;
    }
    prepare_iteration(s, c, ring, s.iters, eta_pre);
}

}  // namespace amp
