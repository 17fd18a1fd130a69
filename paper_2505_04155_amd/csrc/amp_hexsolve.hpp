// AMP-PCG on the matrix-free hexahedral operator (Section 5.5, Ex. jac
// libp): the solve's product, initial-residual and true-residual kernels for
// a matrix handle that wraps an operator instead of a sliced-ELL matrix.
// The controller, preconditioning and update kernels are the sliced-ELL
// solve's own; the product writes its partials (gamma, max|p|) in the same
// places, so they follow unchanged.
//
// q is summed by atomic adds, so it must be zero before each product: the
// update kernel clears the q it has consumed (Cfg::zero_q), and the start of
// a solve clears both precisions' q.  t = A x for the FP64 residuals is
// formed in the FP64 q buffer, which is zero whenever those kernels run,
// and cleared again after use.
#pragma once

#include "amp_hex.hpp"
#include "amp_kernels.hpp"

namespace amp {

constexpr int kHexWaves = 4;                 // elements in flight per work-group
constexpr int NTH = kHexWaves * WAVE;        // threads per work-group of these kernels

// The elements of work-group wg: pass t gives wave w element
// (wg.lb kHexWaves + w) + t wg.G kHexWaves.  The trip count is the same for
// every wave of the work-group.  f(active, ex, ey, ez).
template <typename F>
__device__ __forceinline__ void hex_elements(const HexView &h, Wg wg, F f) {
    const int64_t E = (int64_t)h.ex * h.ey * h.ez;
    const int wave = threadIdx.x / WAVE;
    const int64_t stride = (int64_t)wg.G * kHexWaves;
    for (int64_t base = (int64_t)wg.lb * kHexWaves; base < E; base += stride) {
        const int64_t e = base + wave;
        const bool active = e < E;
        const int64_t ee = active ? e : 0;
        f(active, (int)(ee % h.ex), (int)((ee / h.ex) % h.ey), (int)(ee / ((int64_t)h.ex * h.ey)));
    }
}

// the same for one wave (sized for FP64, used for either precision)
template <int N>
struct HexLdsBlock1 {
    HexLds<N, double> w[1];
};

// The product of an iteration in three launches, so that the element
// kernel runs one wave per element (the shape of the standalone operator;
// a grid of at most GMAX multi-wave work-groups holds 256 VGPRs per lane):
//   k_hex_beta    one work-group: beta from the rho partials, the checks of
//                 spmv_stage, the state for the product;
//   k_hex_elem    one wave per element: p = z + beta p_old at every gathered
//                 node (the owner copy stores it), q += A_e p_e (atomic adds),
//                 per-element gamma_e = p_e^T A_e p_e and max|p| of the owned
//                 nodes;
//   k_hex_reduce  G work-groups: each sums a contiguous range of the element
//                 partials in element order (the update reads G partials).
__global__ void __launch_bounds__(NT) k_hex_beta(const St *in, const double *part, int gpart, Cfg c, int uzf,
                                                 St *out) {
    __shared__ St s;
    const Wg wg{0, 1};
    PartRegs<2, NT> pr;
    load_parts<2, NT>(part, gpart, pr);
    load_state(s, in);
    if (s.status != RUNNING) {
        store_state(s, out, wg);
        return;
    }
    const double rho_prev = s.rho;
    const int k = s.k;
    double tot[2];
    reduce_loaded<1, 1, NT>(pr, gpart, tot);
    const double rho = tot[0], mz = tot[1];
    const double beta = (k > 0) ? rho / rho_prev : 0.0;
    const bool brk = !(rho > 0.0) || !isfinite(beta);
    if (threadIdx.x == 0) {
        s.rho_prev = rho_prev;
        s.rho = rho;
        s.beta = beta;
        s.maxz = mz;
        if (brk) s.status = BREAKDOWN;
        if (c.scalar_history) c.scalar_history[4 * k + 1] = rho;
        if (!brk && c.spmv_iter) c.spmv_iter[c.spmv_launch] = k;
        if (!brk && uzf != 0 && s.uz != uzf) s.status = BREAKDOWN;   // only from a non-finite residual
    }
    store_state(s, out, wg);
}

template <int N, int UZ, int UR, bool FIRST>
__device__ __forceinline__ void hex_elem_body(const HexView &h, int ex, int ey, int ez, const Bufs &B, int pb,
                                              double beta_d, HexLdsBlock1<N> &lds, double &gam, double &mp) {
    typedef typename Prec<UZ>::T TZ;
    typedef typename Prec<UZ>::C CZ;
    typedef typename Prec<UR>::T T;
    constexpr int ps = pslot(UZ);
    HexLds<N, T> &L = *reinterpret_cast<HexLds<N, T> *>(&lds.w[0]);
    const TZ *z = (const TZ *)B.z[ps];
    const TZ *po = (const TZ *)B.p[ps][pb];
    TZ *pn = (TZ *)B.p[ps][pb ^ 1];
    T *q = (T *)B.q[pslot(UR)];
    const CZ beta = (CZ)beta_d;
    const int lane = threadIdx.x % WAVE;
    const int i = lane % (N + 1), j = (lane / (N + 1)) % (N + 1);
    hex_wave_apply<N, T, false>(
        h, true, ex, ey, ez, L,
        [&](int k, int64_t dof) -> T {
            const TZ pv = FIRST ? z[dof] : (TZ)((CZ)z[dof] + beta * (CZ)po[dof]);
            if (hex_owner<N>(h, ex, ey, ez, i, j, k)) {
                pn[dof] = pv;
                mp = fmax(mp, fabs((double)pv));
            }
            return (T)pv;
        },
        [&](int, int64_t dof, T a, T u) {
            unsafeAtomicAdd(q + dof, a);
            gam += (double)u * (double)a;
        });
}

template <int N, int UZF>
__global__ void __launch_bounds__((N + 1) * (N + 1)) k_hex_elem(HexView h, Bufs B, const St *st, double *epart) {
    constexpr int NP = (N + 1) * (N + 1);
    __shared__ St s;
    __shared__ HexLdsBlock1<N> lds;
    __shared__ double s_g[NP], s_m[NP];
    load_state(s, st);
    if (s.status != RUNNING) return;
    int ex, ey, ez;
    hex_element(h, ex, ey, ez);
    const int uz = (UZF != 0) ? UZF : s.uz, ur = s.ur, pb = s.pbuf;
    const bool first = s.k == 0;
    const double beta = s.beta;
    double gam = 0.0, mp = 0.0;
#define AMP_HE(UZ, UR)                                                                          \
    do {                                                                                        \
        if (first) hex_elem_body<N, UZ, UR, true>(h, ex, ey, ez, B, pb, beta, lds, gam, mp);    \
        else hex_elem_body<N, UZ, UR, false>(h, ex, ey, ez, B, pb, beta, lds, gam, mp);         \
    } while (0)
#define AMP_HE_R(UZ)                 \
    do {                             \
        if (ur == 64) AMP_HE(UZ, 64); \
        else AMP_HE(UZ, 32);          \
    } while (0)
    if constexpr (UZF == 64) AMP_HE_R(64);
    else if constexpr (UZF == 32) AMP_HE_R(32);
    else if constexpr (UZF == 16) AMP_HE_R(16);
    else {
        if (uz == 64) AMP_HE_R(64);
        else if (uz == 32) AMP_HE_R(32);
        else AMP_HE_R(16);
    }
#undef AMP_HE_R
#undef AMP_HE
    // the element's partials, summed over its lines in lane order
    s_g[threadIdx.x] = gam;
    s_m[threadIdx.x] = mp;
    __syncthreads();
    if (threadIdx.x == 0) {
        double g = 0.0, m = 0.0;
        for (int l = 0; l < NP; ++l) {
            g += s_g[l];
            m = fmax(m, s_m[l]);
        }
        const int64_t E = (int64_t)h.ex * h.ey * h.ez, e = ((int64_t)ez * h.ey + ey) * h.ex + ex;
        epart[e] = g;
        epart[E + e] = m;
    }
}

typedef void (*HexElemFn)(HexView, Bufs, const St *, double *);
template <int N>
inline HexElemFn hex_elem_fn_n(int uzf) {
    switch (uzf) {
        case 16: return k_hex_elem<N, 16>;
        case 32: return k_hex_elem<N, 32>;
        case 64: return k_hex_elem<N, 64>;
        default: return k_hex_elem<N, 0>;
    }
}
inline HexElemFn hex_elem_fn(int order, int uzf) { return order == 7 ? hex_elem_fn_n<7>(uzf) : hex_elem_fn_n<3>(uzf); }

// Work-group lb of G sums the element partials of its contiguous range in
// element order (thread t takes every NT-th element of the range, then the
// fixed reduction tree): part[lb] = sum gamma_e, part[GMAX + lb] = max.
__global__ void __launch_bounds__(NT) k_hex_reduce(const double *epart, int64_t E, const St *st, double *part) {
    __shared__ St s;
    load_state(s, st);
    if (s.status != RUNNING) return;
    const Wg wg = grid_wg();
    int64_t lo, hi;
    block_range(E, 1, wg.lb, wg.G, lo, hi);
    double g = 0.0, m = 0.0;
    for (int64_t e = lo + threadIdx.x; e < hi; e += NT) {
        g += epart[e];
        m = fmax(m, epart[E + e]);
    }
    double v2[2] = {g, m};
    block_reduce<1, 1>(v2);
    if (threadIdx.x == 0) {
        part[wg.lb] = v2[0];
        part[GMAX + wg.lb] = v2[1];
    }
}

// Whether an FP64 residual kernel runs for this state (mode as k_true_res;
// -1: r0 at the start of the solve, always).
__device__ __forceinline__ bool hex_res_runs(const St &s, int mode) {
    return mode < 0 || (mode == 0 && s.status == NEED_VERIFY) || (mode == 1 && s.status == RUNNING) || mode == 2;
}

// t = A x (FP64) into the FP64 q buffer (zero on entry), when the residual
// kernel that follows runs.
template <int N>
__global__ void __launch_bounds__(NTH) k_hex_xapply(HexView h, Bufs B, int mode, const St *in) {
    __shared__ HexLds<N, double> L[kHexWaves];
    __shared__ St s;
    if (mode >= 0) {
        load_state(s, in);
        if (!hex_res_runs(s, mode)) return;   // uniform: every thread read the same state
    }
    const Wg wg = grid_wg();
    const double *x = B.x;
    double *t = (double *)B.q[0];
    const int wave = threadIdx.x / WAVE;
    hex_elements(h, wg, [&](bool active, int ex, int ey, int ez) {
        hex_wave_apply<N, double, true>(h, active, ex, ey, ez, L[wave], [&](int, int64_t dof) { return x[dof]; },
                                  [&](int, int64_t dof, double a, double) { unsafeAtomicAdd(t + dof, a); });
    });
}

// r0 = b - t (FP64) and the partials of k_init (||r0||^2, ||b||^2, max|r0|);
// t cleared.  One contiguous range of rows per work-group.
__global__ void __launch_bounds__(NT) k_hex_init_finish(Bufs B, int64_t np) {
    const Wg wg = grid_wg();
    int64_t lo, hi;
    block_range(np, (int64_t)NT * VEC, wg.lb, wg.G, lo, hi);
    double *t = (double *)B.q[0];
    double *r = (double *)B.r[0];
    double sr = 0.0, sb = 0.0, mr = 0.0;
    for (int64_t row = lo + threadIdx.x; row < hi; row += NT) {
        const double v = B.b[row] - t[row];
        r[row] = v;
        t[row] = 0.0;
        sr += v * v;
        sb += B.b[row] * B.b[row];
        mr = fmax(mr, fabs(v));
    }
    double v3[3] = {sr, sb, mr};
    block_reduce<2, 1>(v3);
    if (threadIdx.x == 0) {
        B.part_res[wg.lb] = v3[0];
        B.part_res[GMAX + wg.lb] = v3[1];
        B.part_res[2 * GMAX + wg.lb] = v3[2];
    }
}

// The FP64 true residual b - t (modes of k_true_res), t cleared.
template <int RS>
__device__ __forceinline__ void hex_true_res_rows(const Bufs &B, int64_t lo, int64_t hi, bool write, double &st,
                                                  double &ss, double &mr) {
    typedef typename Prec<RS>::T TR;
    TR *r = (TR *)B.r[pslot(RS)];
    double *t = (double *)B.q[0];
    for (int64_t row = lo + threadIdx.x; row < hi; row += NT) {
        const double v = B.b[row] - t[row];
        t[row] = 0.0;
        const TR tr = (TR)v;
        if (write) r[row] = tr;
        st += v * v;
        ss += (double)tr * (double)tr;
        mr = fmax(mr, fabs((double)tr));
    }
}

__global__ void __launch_bounds__(NT) k_hex_true_res_finish(Cfg c, Bufs B, int64_t np, int mode, const St *in,
                                                            St *out) {
    __shared__ St s;
    const Wg wg = grid_wg();
    load_state(s, in);
    if (!hex_res_runs(s, mode)) {
        store_state(s, out, wg);
        return;
    }
    int64_t lo, hi;
    block_range(np, (int64_t)NT * VEC, wg.lb, wg.G, lo, hi);
    double st = 0.0, ss = 0.0, mr = 0.0;
    if (s.r_store == 64) hex_true_res_rows<64>(B, lo, hi, mode != 2, st, ss, mr);
    else hex_true_res_rows<32>(B, lo, hi, mode != 2, st, ss, mr);
    double v3[3] = {st, ss, mr};
    block_reduce<2, 1>(v3);
    if (threadIdx.x == 0) {
        B.part_res[wg.lb] = v3[0];
        B.part_res[GMAX + wg.lb] = v3[1];
        B.part_res[2 * GMAX + wg.lb] = v3[2];
        if (mode == 0) {
            s.status = RUNNING;
            s.kind = RES_VERIFY;
        } else if (mode == 1) {
            s.kind = RES_PERIODIC;
        }
    }
    store_state(s, out, wg);
}

}  // namespace amp
