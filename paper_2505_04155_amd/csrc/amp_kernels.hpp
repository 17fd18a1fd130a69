// HIP kernels of one AMP-PCG iteration (Alg. 3).  Three launches per
// iteration, in the paper's order:
//
//   k_precond  [prologue: consume ||r_k||, max|r_k| -> convergence test,
//               eta_k, precisionSelector, omega_k]
//              y = omega r (u_r), z = M^{-1} y (u_z), partials of rho = r^T z
//   k_spmv     [prologue: rho_k, beta_{k-1}]
//              p = z + beta p (u_z, written for the own rows and recomputed
//              on the fly at the gathered columns), q = A p (u_r), partials
//              of gamma = q^T p
//   k_update   [prologue: gamma, alpha]
//              r -= alpha q (u_r), partials of ||r||^2; x += alpha p (FP64)
//              applied two iterations at a time (see update_run)
//
// plus k_init (r0 = b - A x0) and k_true_res (FP64 b - A x for the
// termination check, periodic replacement, or a report).
//
// Cross-work-group reductions use no atomics and no fences: every
// work-group writes its partial sums; every work-group of the next kernel
// adds all of them in the same fixed order and evaluates the controller
// from identical inputs, so all reach identical decisions.  Work-group 0
// writes the resulting state to a buffer that no work-group of the same
// kernel reads.  Each kernel issues its partial loads together with the
// state load, and the streaming kernels their first body loads before the
// reduction (a barrier waits only for LDS, so these stay in flight).
#pragma once

#include <type_traits>

#include "amp_device.hpp"

namespace amp {

// State slots of a solve (the chain each kernel reads from and writes to).
enum Slot : int {
    ST_INIT = 0, ST_PRE = 1, ST_SPMV = 2, ST_RES = 3, ST_TR = 4, ST_REPORT = 5,
    ST_PREI = 6, ST_CH0 = 7, ST_CH1 = 8, ST_FIN = 9, ST_COUNT = 10
};

// Working vectors, indexed by precision slot (0: FP64, 1: FP32, 2: FP16).
// All are padded to np elements; p is double-buffered.
struct Bufs {
    double *x;
    const double *b;
    void *r[3], *z[3], *q[3];
    void *p[3][2];
    const void *dinv[3];
    double *part_res;   // 3 x GMAX: sum a, sum b, max
    double *part_pre;   // 2 x GMAX: rho, max|z|
    double *part_spmv;  // 2 x GMAX: gamma, max|p|
};

__host__ __device__ constexpr int pslot(int u) { return u == 64 ? 0 : (u == 32 ? 1 : 2); }

template <typename T>
struct alignas(sizeof(T) * VEC) V4 {
    T v[VEC];
};
template <typename T>
__device__ __forceinline__ V4<T> ld4(const T *p, int64_t i) {
    return *reinterpret_cast<const V4<T> *>(p + i);
}
template <typename T>
__device__ __forceinline__ void st4(T *p, int64_t i, const V4<T> &x) {
    *reinterpret_cast<V4<T> *>(p + i) = x;
}

// Streaming loop over this work-group's contiguous element range.
#define AMP_STREAM_LOOP(i, np, wg)                                                      \
    int64_t lo_, hi_;                                                                    \
    block_range((np), (int64_t)NT * VEC, (wg).lb, (wg).G, lo_, hi_);                     \
    for (int64_t i = lo_ + (int64_t)threadIdx.x * VEC; i < hi_; i += (int64_t)NT * VEC)

// ----------------------------------------------------------------------------
// state plumbing
// ----------------------------------------------------------------------------

// What a kernel's first memory round trip needs besides the state pointer:
// the producer's partial arrays, how many work-groups wrote them, and the
// residual-norm window.  The single-system kernels take these as their
// leading scalar arguments, which the hardware preloads into registers, so
// the first loads are issued without waiting for the argument segment.
struct Early {
    const double *part;
    int g;
    const double *ring;
    uint32_t touched;   // touch_args() of the kernel (0 where there is none)
};

// Load the incoming state into LDS (all threads see it after the barrier).
__device__ __forceinline__ void load_state(St &s, const St *in) {
    if (threadIdx.x == 0) s = *in;
    __syncthreads();
}

__device__ __forceinline__ void store_state(const St &s, St *out, Wg wg) {
    if (wg.lb == 0 && threadIdx.x == 0) *out = s;
}

// Record ||r_i|| (work-group 0 only; nobody reads index i in this kernel).
__device__ __forceinline__ void record_delta(const Cfg &c, int i, double d, Wg wg) {
    if (wg.lb == 0) {
        c.ring[i % kRing] = d;
        if (c.delta_history) c.delta_history[i] = d;
    }
}

// ----------------------------------------------------------------------------
// deferred x update
// ----------------------------------------------------------------------------

// x += alpha p over this work-group's element range (the range every
// streaming kernel of the system uses, so each x element is always updated
// by the same work-group and thread).
template <int UPP>
__device__ __forceinline__ void flush_x_body(double alpha, const void *pv, double *x, int64_t np, Wg wg) {
    typedef typename Prec<UPP>::T TP;
    const TP *p = (const TP *)pv;
    AMP_STREAM_LOOP(i, np, wg) {
        const V4<TP> pv4 = ld4(p, i);
        V4<double> xv = ld4(x, i);
#pragma unroll
        for (int e = 0; e < VEC; ++e) xv.v[e] = xv.v[e] + alpha * (double)pv4.v[e];
        st4(x, i, xv);
    }
}

// Apply the state's pending step alpha_{k-1} p_{k-1} to x, if any, and clear
// it.  Every thread of the work-group calls this (it has a barrier).
__device__ __forceinline__ void stop_flush(St &s, const Bufs &B, int64_t np, Wg wg) {
    const int xp = s.xp, pu = s.x_pu, pb = s.x_pb;
    const double a = s.x_alpha;
    if (xp) {
        const void *p = B.p[pslot(pu)][pb];
        if (pu == 64) flush_x_body<64>(a, p, B.x, np, wg);
        else if (pu == 32) flush_x_body<32>(a, p, B.x, np, wg);
        else flush_x_body<16>(a, p, B.x, np, wg);
    }
    __syncthreads();
    if (threadIdx.x == 0) s.xp = 0;
}

// ----------------------------------------------------------------------------
// sliced-ELL row products
// ----------------------------------------------------------------------------

// Slots are read in chunks of kChunk: the chunk's values and gathers are
// all issued before the first product is added, so a wave keeps up to
// 2 kChunk loads in flight.  Slots past the row width repeat a valid slot's
// loads (cache hits) and add nothing; the sum runs in slot order.

// q_i = sum_j a_ij p_j with FP64 values and accumulation, slot order.
template <typename CS, typename PF>
__device__ __forceinline__ double row_dot64(const Sell &A, const CS &sc, int64_t base, int w, PF pval) {
    double acc = 0.0;
    for (int j0 = 0; j0 < w; j0 += kChunk) {
        int32_t c[kChunk];
        bool dg[kChunk];
        double v[kChunk], pj[kChunk];
        sc.chunk(j0, w, c, dg);
#pragma unroll
        for (int u = 0; u < kChunk; ++u) {
            const int j = j0 + u < w ? j0 + u : w - 1;
            v[u] = A.v64[base + (int64_t)j * SLICE];
            pj[u] = (double)pval(c[u]);
        }
#pragma unroll
        for (int u = 0; u < kChunk; ++u) {
            const double t = acc + v[u] * pj[u];
            acc = (j0 + u < w) ? t : acc;
        }
    }
    return acc;
}

// FP32 values and accumulation.  DIFF: off-diagonal slots add a_ij (p_j - p_i)
// in slot order, then the diagonal slot's row sum s_i adds s_i p_i; padding
// slots (value 0) add 0 exactly.  Otherwise the textbook form.
template <bool DIFF, typename CS, typename PF>
__device__ __forceinline__ float row_dot32(const Sell &A, const CS &sc, int64_t base, int w, float pi, PF pval) {
    const float *vals = DIFF ? A.v32 : A.v32p;
    float acc = 0.0f, dterm = 0.0f;
    for (int j0 = 0; j0 < w; j0 += kChunk) {
        int32_t c[kChunk];
        bool dg[kChunk];
        float v[kChunk], pj[kChunk];
        sc.chunk(j0, w, c, dg);
#pragma unroll
        for (int u = 0; u < kChunk; ++u) {
            const int j = j0 + u < w ? j0 + u : w - 1;
            v[u] = vals[base + (int64_t)j * SLICE];
            pj[u] = (float)pval(c[u]);
        }
#pragma unroll
        for (int u = 0; u < kChunk; ++u) {
            const bool in = j0 + u < w;
            if (!DIFF) {
                const float t = acc + v[u] * pj[u];
                acc = in ? t : acc;
            } else {
                const float td = dterm + v[u] * pj[u];
                const float to = acc + v[u] * (pj[u] - pi);
                dterm = (in && dg[u]) ? td : dterm;
                acc = (in && !dg[u]) ? to : acc;
            }
        }
    }
    return DIFF ? dterm + acc : acc;
}

// Slices of this work-group: contiguous range, one slice per wave at a time,
// the next slice's descriptor in flight while the current one is processed.
#define AMP_SLICE_LOOP(A, sl, wg, BS)                                                    \
    int64_t slo_, shi_;                                                                  \
    block_range((A).nslices, 1, (wg).lb, (wg).G, slo_, shi_);                            \
    const int64_t sfirst_ = slo_ + __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);   \
    uint32_t nrec_ = rec_word((A).srec, sfirst_, shi_);                                  \
    for (int64_t sl = sfirst_; sl < shi_; sl += (BS) / WAVE)

#define AMP_SLICE_ROW(A, sl, lane, row, base, w, BS)                                     \
    const SliceRec rec_ = rec_from(nrec_);                                               \
    nrec_ = rec_word((A).srec, (sl) + (BS) / WAVE, shi_);                                \
    const int lane = threadIdx.x % WAVE;                                                 \
    const int64_t row = (sl) * SLICE + lane, base = rec_.ptr + lane;                     \
    const int w = rec_.width

#define AMP_WITH_COLS(A, sl, lane, sc) \
    with_rec_cols(rec_, (A).col, (A).offs, (A).np, sl, lane, [&](const auto &sc)

// ----------------------------------------------------------------------------
// several lanes per row
// ----------------------------------------------------------------------------
//
// A matrix built with L = 2^lgL lanes per row (for long rows; index mode
// only) has slices of 64 / L rows: entry e of the slice's g-th row sits in
// lane g L + (e mod L), slot e / L.  A lane sums its own slots in slot order;
// the row's total is then formed by xor-butterfly shuffles across its L
// lanes, which gives every lane of the row the same bits (each pairwise add
// is commutative).

// Sum of v over the lanes of each row (all lanes of a row receive it).
__device__ __forceinline__ double row_lanes_sum(double v, int lgL) {
    for (int m = 1; m < (1 << lgL); m <<= 1) v = v + __shfl_xor(v, m);
    return v;
}
__device__ __forceinline__ float row_lanes_sum(float v, int lgL) {
    for (int m = 1; m < (1 << lgL); m <<= 1) v = v + __shfl_xor(v, m);
    return v;
}

// FP64 products q_i = sum_j a_ij pval(j) of this work-group's slices, one
// slice per wave at a time; f(row, sub, q_i) is called on every lane (sub:
// the lane's index within its row, 0 for one row per lane).
template <int BS, bool LANES, typename PF, typename F>
__device__ __forceinline__ void rows_dot64(const Sell &A, Wg wg, PF pval, F f) {
    if constexpr (!LANES) {
        AMP_SLICE_LOOP(A, sl, wg, BS) {
            AMP_SLICE_ROW(A, sl, lane, row, base, w, BS);
            double ax = 0.0;
            AMP_WITH_COLS(A, sl, lane, sc) { ax = row_dot64(A, sc, base, w, pval); });
            f(row, 0, ax);
        }
    } else {
        const int lgL = A.lgL;
        int64_t slo, shi;
        block_range(A.nslices, 1, wg.lb, wg.G, slo, shi);
        const int lane = threadIdx.x % WAVE;
        for (int64_t sl = slo + __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE); sl < shi; sl += BS / WAVE) {
            const SliceRec rec = A.srec[sl];
            const int64_t row = sl * (SLICE >> lgL) + (lane >> lgL);
            const IdxCols sc{A.col + rec.ptr + lane, row};
            const double ax = row_lanes_sum(row_dot64(A, sc, rec.ptr + lane, rec.width, pval), lgL);
            f(row, lane & ((1 << lgL) - 1), ax);
        }
    }
}

// ----------------------------------------------------------------------------
// k_init: r0 = b - A x0 in FP64; partials ||r0||^2, ||b||^2, max|r0|
// ----------------------------------------------------------------------------

template <int BS, bool LANES = false>
__device__ __forceinline__ void init_stage(const Sell &A, const Bufs &B, Wg wg) {
    double sr = 0.0, sb = 0.0, mr = 0.0;
    double *r = (double *)B.r[0];
    const double *x = B.x;
    rows_dot64<BS, LANES>(A, wg, [&](int64_t c) { return x[c]; }, [&](int64_t row, int sub, double ax) {
        if (sub != 0) return;
        const double t = B.b[row] - ax;
        r[row] = t;
        sr += t * t;
        sb += B.b[row] * B.b[row];
        mr = fmax(mr, fabs(t));
    });
    double v3[3] = {sr, sb, mr};
    block_reduce<2, 1, BS>(v3);
    sr = v3[0];
    sb = v3[1];
    mr = v3[2];
    if (threadIdx.x == 0) {
        B.part_res[wg.lb] = sr;
        B.part_res[GMAX + wg.lb] = sb;
        B.part_res[2 * GMAX + wg.lb] = mr;
    }
}

template <bool LANES>
__global__ void __launch_bounds__(NTS) k_init(Sell A, Bufs B) { init_stage<NTS, LANES>(A, B, grid_wg()); }

// ----------------------------------------------------------------------------
// k_precond
// ----------------------------------------------------------------------------

// Prologue inputs of the preconditioning kernel, loaded before the state so
// that both round trips overlap: the residual partials (entries below the
// larger producer grid; the reduction keeps those below the count of the
// producer the state names) and the window of residual norms.
struct ResIn {
    PartRegs<3> pr;
    double ring_v;
};
static_assert(kRing <= NT, "one ring entry per thread");

// The Early arguments of each stage, from the solve's configuration.
__device__ __forceinline__ Early res_early(const Cfg &c, const Bufs &B) {
    return Early{B.part_res, c.g_stream > c.g_slice ? c.g_stream : c.g_slice, c.ring, 0u};
}
__device__ __forceinline__ Early pre_early(const Cfg &c, const Bufs &B) {
    return Early{B.part_pre, c.g_pre, nullptr, 0u};
}
__device__ __forceinline__ Early spmv_early(const Cfg &c, const Bufs &B) {
    return Early{B.part_spmv, c.g_slice, nullptr, 0u};
}

__device__ __forceinline__ void res_loads(const Early &e, ResIn &ri) {
    load_parts<3>(e.part, e.g, ri.pr);
    ri.ring_v = (threadIdx.x < kRing) ? e.ring[threadIdx.x] : 0.0;
}

// Prologue: totals of the residual partials -> controller.  Sets s.status.
__device__ __forceinline__ void consume_residual(St &s, const Cfg &c, const Bufs &B, Wg wg, const ResIn &ri) {
    __shared__ int rec;
    __shared__ double recv;
    __shared__ double ring[kRing];   // the residual-norm window, read in parallel for the controller
    if (threadIdx.x < kRing) ring[threadIdx.x] = ri.ring_v;
    const int G = (s.kind == RES_UPDATE) ? c.g_stream : c.g_slice;
    double tot[3];
    reduce_loaded<2, 1>(ri.pr, G, tot);   // its barrier also publishes ring[]
    const double a = tot[0], b = tot[1], m = tot[2];
    // eq. (eta_k), delay form, for the iteration the controller prepares next
    // (k = iters, delta_k from these totals): lane j of wave 0 forms term j
    // of the window as the serial evaluation would, lane 0 adds the terms in
    // window order (the same sum, without a serial chain of LDS reads)
    const int kk = (s.kind == RES_INIT) ? 0 : s.iters;
    const bool par = c.eta_mode == ETA_DELAY && c.d < WAVE && kk - c.d - 1 >= 0;
    double term = 0.0;
    if (par && threadIdx.x <= c.d) {
        const double dk = sqrt(s.kind == RES_UPDATE ? a : b);
        const int t = kk - c.d + threadIdx.x;
        const double dt = (t == kk) ? dk : ring[t % kRing];
        term = (3.0 + c.C) * ring[(t - 1) % kRing] + (2.0 + c.C) * dt;
    }
    if (threadIdx.x == 0) {
        // the parallel form covers windows of at most WAVE terms; a longer
        // one (d >= WAVE) is summed serially here, from the same window and
        // delta_k (the other indicators are evaluated by the controller)
        double eta_pre = INFINITY;
        if (par) {
            double sum = 0.0;
            for (int j = 0; j <= c.d; ++j) sum = sum + readlane_f64(term, j);
            eta_pre = kEps32 * sum;
        } else if (c.eta_mode == ETA_DELAY) {
            eta_pre = eta_delay(ring, kk, c.d, c.C, sqrt(s.kind == RES_UPDATE ? a : b));
        }
        // the controller runs on a register copy of the state (the LDS copy
        // would put a round trip on every field it reads and updates)
        St cs = s;
        int rk = -1;
        double rv = 0.0;
        if (AMP_LIKELY(cs.kind == RES_UPDATE || cs.kind == RES_PERIODIC)) {
            const double d = sqrt(cs.kind == RES_UPDATE ? a : b);
            if (cs.kind == RES_PERIODIC) cs.n_repl += 1;
            rk = cs.iters;
            rv = d;
            finish_iteration(cs, c, ring, d, m, &eta_pre);
        } else if (cs.kind == RES_INIT) {
            cs.bnorm = sqrt(b);
            cs.tol_b = c.tol * cs.bnorm;
            cs.delta = sqrt(a);
            cs.true_res = cs.delta;   // r0 = b - A x0 is formed in FP64: it is the true residual
            cs.maxr = m;
            cs.maxr_prev = m;
            rk = 0;
            rv = cs.delta;
            if (cs.delta <= cs.tol_b) cs.status = CONVERGED;
            else if (c.maxit <= 0) cs.status = MAXIT;
            else prepare_iteration(cs, c, ring, 0, &eta_pre);
        } else {  // RES_VERIFY: a = ||t||^2 (exact t), b = ||fl(t)||^2
            cs.true_res = sqrt(a);
            if (cs.true_res <= cs.tol_b) {
                cs.status = CONVERGED;
            } else if (cs.n_repl >= c.max_repl) {
                cs.status = MAXIT;
            } else {
                cs.n_repl += 1;
                cs.delta = sqrt(b);
                cs.maxr = m;
                rk = cs.iters;
                rv = cs.delta;
                if (cs.iters >= c.maxit) {
                    cs.status = MAXIT;
                } else {
                    cs.status = RUNNING;
                    prepare_iteration(cs, c, ring, cs.iters, &eta_pre);
                }
            }
        }
        s = cs;
        rec = rk;
        recv = rv;
    }
    __syncthreads();
    if (threadIdx.x == 0 && rec >= 0) {
        record_delta(c, rec, recv, wg);
        if (wg.lb == 0 && s.status == RUNNING) {
            if (c.prec_history) c.prec_history[s.k] = s.uz | (s.ur << 8);
            if (c.scalar_history) c.scalar_history[4 * s.k] = s.omega;
        }
    }
}

// One VEC-element chunk of a vector whose element size (8, 4 or 2 bytes) is
// known only from the state, as raw bits: four 8-byte loads at offsets
// clamped to the chunk, with no branch on the size, so that the loads stay
// in flight until the bits are used.
struct Raw {
    uint2 w[4];
};
static_assert(VEC == 4, "a chunk is at most 32 bytes");
__device__ __forceinline__ void raw_load(const void *base, int bytes, int64_t i, Raw &r) {
    const char *p = (const char *)base + i * bytes;   // i is a multiple of VEC: 8-byte aligned
    const int last = VEC * bytes - 8;
#pragma unroll
    for (int h = 0; h < 4; ++h) r.w[h] = *(const uint2 *)(p + (8 * h < last ? 8 * h : last));
}
template <typename T>
__device__ __forceinline__ V4<T> raw_as(const Raw &r) {
    static_assert(sizeof(V4<T>) <= sizeof(Raw), "chunk fits");
    V4<T> v;
    __builtin_memcpy(&v, &r, sizeof(V4<T>));
    return v;
}

// r_k and the Jacobi data for this thread's first two chunks, loaded before
// the controller has chosen iteration k's precisions (r is held in r_store,
// which the controller does not change; the Jacobi data in the incoming u_z,
// used only if u_z stays).
struct PcPre {
    Raw r[2], d[2];
    int uz;
};

template <int RS, int UR, int UZ>
__device__ __forceinline__ void precond_body(const St &s, const Bufs &B, int64_t np, Wg wg, const PcPre &pre,
                                             double &rho, double &mz) {
    typedef typename Prec<RS>::T TRS;
    typedef typename Prec<UR>::T TR;
    typedef typename Prec<UZ>::T TZ;
    typedef typename Prec<UZ>::C CZ;
    const TRS *r = (const TRS *)B.r[pslot(RS)];
    TR *rn = (TR *)B.r[pslot(UR)];
    TZ *z = (TZ *)B.z[pslot(UZ)];
    const TZ *dv = (const TZ *)B.dinv[pslot(UZ)];
    const TR w = (TR)s.omega_eff;
    auto chunk = [&](int64_t i, const V4<TRS> &rv, const V4<TZ> &dd) {
        V4<TZ> zz;
        V4<TR> rr;
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
            const TR re = (TR)rv.v[e];
            rr.v[e] = re;
            const TZ y = narrow<TZ>(re * w);           // computed in u_r, stored in u_z
            const TZ ze = (TZ)((CZ)y * (CZ)dd.v[e]);   // computed and stored in u_z
            zz.v[e] = ze;
            rho += (double)re * (double)ze;
            mz = fmax(mz, fabs((double)ze));
        }
        st4(z, i, zz);
        if (RS != UR) st4(rn, i, rr);
    };
    int64_t lo, hi;
    block_range(np, (int64_t)NT * VEC, wg.lb, wg.G, lo, hi);
    int64_t i = lo + (int64_t)threadIdx.x * VEC;
    if (pre.uz == UZ) {   // chunks 0 and 1 are in registers
#pragma unroll
        for (int j = 0; j < 2; ++j, i += (int64_t)NT * VEC)
            if (i < hi) chunk(i, raw_as<TRS>(pre.r[j]), raw_as<TZ>(pre.d[j]));
    }
    // the rest of the range (large systems), two chunks per pass with all
    // their loads issued first
    constexpr int64_t step = (int64_t)NT * VEC;
    for (; i + step < hi; i += 2 * step) {
        const V4<TRS> ra = ld4(r, i), rb = ld4(r, i + step);
        const V4<TZ> da = ld4(dv, i), db = ld4(dv, i + step);
        chunk(i, ra, da);
        chunk(i + step, rb, db);
    }
    if (i < hi) chunk(i, ld4(r, i), ld4(dv, i));
}

// At a u_z switch p_{k-1} is first rounded to the new u_z.
template <int PS, int UZ>
__device__ __forceinline__ void convert_p(const Bufs &B, int pb, int64_t np, Wg wg) {
    typedef typename Prec<PS>::T TPS;
    typedef typename Prec<UZ>::T TZ;
    const TPS *po = (const TPS *)B.p[pslot(PS)][pb];
    TZ *pn = (TZ *)B.p[pslot(UZ)][pb];
    AMP_STREAM_LOOP(i, np, wg) {
        const V4<TPS> a = ld4(po, i);
        V4<TZ> b;
#pragma unroll
        for (int e = 0; e < VEC; ++e) b.v[e] = narrow<TZ>(a.v[e]);
        st4(pn, i, b);
    }
}

// Residual replacement at the u_r switch (the alternative to carrying the
// recurrence residual that Sections 1.1 and 3.1 mention): on the iteration
// whose u_r first drops to FP32, r_k is fl32(b - A x_k), formed with the
// FP64 values and FP64 accumulation, instead of the recurrence residual
// rounded to FP32.  delta_k keeps the recurrence value that drove the
// decision.  Rows of this work-group's element range [lo, hi) (whole
// slices: lo and hi are multiples of NT VEC), one slice per wave; x_k at a
// gathered column includes a pending deferred step alpha_{k-1} p_{k-1},
// rounded exactly as stop_flush applies it.
template <int PU>
__device__ __forceinline__ void switch_replace_body(const Sell &A, const Bufs &B, const St &s, int64_t lo,
                                                    int64_t hi) {
    typedef typename Prec<PU == 0 ? 64 : PU>::T TP;
    // (a select, not an index: an argument array indexed at run time is
    // copied to private memory)
    constexpr int ps = pslot(PU == 0 ? 64 : PU);
    const TP *pp = (const TP *)(s.x_pb ? B.p[ps][1] : B.p[ps][0]);
    const double a = s.x_alpha;
    const double *x = B.x;
    float *r = (float *)B.r[1];
    auto xval = [&](int64_t c) -> double {
        if (PU == 0) return x[c];
        return x[c] + a * (double)pp[c];
    };
    const int lgL = A.lgL, R = SLICE >> lgL;   // rows per slice (several lanes per row: see rows_dot64)
    const int64_t s0 = lo / R, s1 = (hi / R < A.nslices) ? hi / R : A.nslices;
    const int lane = threadIdx.x % WAVE;
    // one slot at a time (this runs once per solve; a lean loop keeps the
    // preconditioning kernel's register budget); the sum runs in slot order
    // with one rounding per operation, as row_dot64
    for (int64_t sl = s0 + __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE); sl < s1; sl += NT / WAVE) {
        const SliceRec rec_ = A.srec[sl];
        const int64_t row = sl * R + (lane >> lgL), base = rec_.ptr + lane;
        double ax = 0.0;
        for (int j = 0; j < rec_.width; ++j) {
            int64_t c;
            if (rec_.soff >= 0) {
                const int64_t cc = row + A.offs[rec_.soff + j];
                c = (cc >= 0 && cc < A.np) ? cc : row;
            } else {
                c = A.col[base + (int64_t)j * SLICE];
            }
            ax = ax + A.v64[base + (int64_t)j * SLICE] * xval(c);
        }
        ax = row_lanes_sum(ax, lgL);
        if ((lane & ((1 << lgL) - 1)) == 0) r[row] = (float)(B.b[row] - ax);
    }
}

__device__ __forceinline__ void switch_replace(const Sell &A, const Bufs &B, const St &s, int64_t np, Wg wg) {
    int64_t lo, hi;
    block_range(np, (int64_t)NT * VEC, wg.lb, wg.G, lo, hi);
    if (!s.xp) switch_replace_body<0>(A, B, s, lo, hi);
    else if (s.x_pu == 64) switch_replace_body<64>(A, B, s, lo, hi);
    else if (s.x_pu == 32) switch_replace_body<32>(A, B, s, lo, hi);
    else switch_replace_body<16>(A, B, s, lo, hi);
    __syncthreads();   // the rows' residuals are read by other threads of the work-group
}

// Whether this iteration replaces r (its u_r has just dropped to FP32).
__device__ __forceinline__ bool switch_replaces(const Cfg &c, const St &s) {
    return c.rr_switch && s.r_store == 64 && s.ur == 32;
}

__device__ __forceinline__ void precond_stage(const Cfg &c, const Sell &A, const Bufs &B, int64_t np, const St *in,
                                              St *out, Wg wg, const Early &e) {
    __shared__ St s;
    ResIn ri;
    res_loads(e, ri);
    load_state(s, in);
    pin(e.touched);
    if (s.status != RUNNING) {
        stop_flush(s, B, np, wg);
        store_state(s, out, wg);
        return;
    }
    PcPre pre;
    {
        int64_t lo, hi;
        block_range(np, (int64_t)NT * VEC, wg.lb, wg.G, lo, hi);
        const int64_t i0 = lo + (int64_t)threadIdx.x * VEC;
        pre.uz = s.uz;
        const void *rv = B.r[pslot(s.r_store)];
        const void *dv = B.dinv[pslot(s.uz)];
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            // chunks past this work-group's range load chunk 0 (unused): no branch
            const int64_t i = i0 + (int64_t)j * NT * VEC < hi ? i0 + (int64_t)j * NT * VEC : 0;
            raw_load(rv, s.r_store / 8, i, pre.r[j]);
            raw_load(dv, s.uz / 8, i, pre.d[j]);
        }
    }
    consume_residual(s, c, B, wg, ri);
    __syncthreads();
    if (s.status != RUNNING) {   // the solve stops here: x gets its pending step
        stop_flush(s, B, np, wg);
        store_state(s, out, wg);
        return;
    }
    int rs = s.r_store;
    const int ur = s.ur, uz = s.uz;
    if (switch_replaces(c, s)) {   // r_k := fl32(b - A x_k); the preloaded chunks are not used
        switch_replace(A, B, s, np, wg);
        rs = 32;
        pre.uz = 0;
        if (threadIdx.x == 0) s.n_repl += 1;
    }
    double rho = 0.0, mz = 0.0;
#define AMP_PC(RS, UR, UZ) precond_body<RS, UR, UZ>(s, B, np, wg, pre, rho, mz)
#define AMP_PC_Z(RS, UR)                  \
    if (uz == 64) AMP_PC(RS, UR, 64);       \
    else if (uz == 32) AMP_PC(RS, UR, 32);  \
    else AMP_PC(RS, UR, 16);
    if (rs == 64 && ur == 64) { AMP_PC_Z(64, 64) }
    else if (rs == 64) { AMP_PC_Z(64, 32) }
    else { AMP_PC_Z(32, 32) }
#undef AMP_PC_Z
#undef AMP_PC
    const bool conv = (s.k > 0 && s.p_store != uz);
    if (conv) {
        if (s.p_store == 64 && uz == 32) convert_p<64, 32>(B, s.pbuf, np, wg);
        else if (s.p_store == 64) convert_p<64, 16>(B, s.pbuf, np, wg);
        else convert_p<32, 16>(B, s.pbuf, np, wg);
    }
    double v2[2] = {rho, mz};
    block_reduce<1, 1>(v2);
    rho = v2[0];
    mz = v2[1];
    if (threadIdx.x == 0) {
        B.part_pre[wg.lb] = rho;
        B.part_pre[GMAX + wg.lb] = mz;
        s.r_store = s.ur;
        if (conv) s.p_store = uz;
    }
    store_state(s, out, wg);
}

__global__ void __launch_bounds__(NT) k_precond(const St *in, const double *part, int gpart, int grid,
                                                const double *ring, Cfg c, Bufs B, int64_t np, St *out, Sell A) {
    precond_stage(c, A, B, np, in, out, launch_wg(grid), Early{part, gpart, ring,
                  touch_args<32 + sizeof(Cfg) + sizeof(Bufs)>()});
}

// ----------------------------------------------------------------------------
// k_spmv: p = z + beta p_{k-1} (u_z), q = A p (u_r), gamma = q^T p
// ----------------------------------------------------------------------------

// Slots per pass of the product's offset-mode loop (8: one chunk, 16: two).
#ifndef AMP_SPMV_SPC
#define AMP_SPMV_SPC 16
#endif

// p = z + beta p_old (u_z) for the work-group's rows, q = A p (u_r) with the
// p entries recomputed at every gathered column, gamma and max|p| partials.
// Offset-mode slices read their neighbours from the guarded views of z and
// p_old (index = column + guard, no range test: a slot whose column lies
// outside [0, np) has value 0 and reads a zero of the margin); the values
// load from the slice's scalar base plus the lane's offset, the offsets are
// scalar loads.  Sums run in slot order as in row_dot64 / row_dot32: FP64
// values and accumulation for u_r = FP64; FP32 for u_r = FP32, in the
// row-sum/difference form when DIFF (off-diagonal slots add
// a_ij (p_j - p_i), then the diagonal slot's row sum adds s_i p_i).
// Slices are dealt per XCD (xcd_wave_slices).
// PRIO: issue priority by progress (progress_prio); off where the
// work-groups sharing a CU belong to different systems with unequal work.
// SPC: slots per pass (whole chunks); it changes only how many loads are in
// flight, never the order of the sums.
// LANES: the matrix may have several lanes per row (index-mode slices only;
// see rows_dot64).
// NTL: the offset-mode values are loaded with a non-temporal hint (a value
// plane larger than the memory-side cache, kMallBytes).
template <int UZ, int UR, bool DIFF, bool FIRST, int BS, bool PRIO = true, int SPC = AMP_SPMV_SPC,
          bool LANES = false, bool NTL = false>
__device__ __forceinline__ void spmv_p_body(const Sell &A, Wg wg, const void *zv, const void *pov, void *pnv,
                                            void *qv, double beta_d, double &gam, double &mp) {
    typedef typename Prec<UZ>::T TZ;
    typedef typename Prec<UZ>::C CZ;
    typedef typename Prec<UR>::T TQ;
    typedef typename Prec<UR>::C CA;   // value plane and accumulation type
    const TZ *zg = (const TZ *)zv - A.guard;
    const TZ *pg = (const TZ *)pov - A.guard;
    TZ *pn = (TZ *)pnv;
    TQ *q = (TQ *)qv;
    const CA *vals = (UR == 64) ? (const CA *)A.v64 : (DIFF ? (const CA *)A.v32 : (const CA *)A.v32p);
    const CZ beta = (CZ)beta_d;
    constexpr int NW = BS / WAVE, NCH = SPC / kChunk;
    static_assert(SPC % kChunk == 0 && SPC >= kChunk, "whole chunks per pass");
    // p at guarded index i
    auto pval = [&](uint32_t i) -> TZ {
        if (FIRST) return at32(zg, i);
        return (TZ)((CZ)at32(zg, i) + beta * (CZ)at32(pg, i));
    };
    const int lane = threadIdx.x % WAVE;
    int64_t sfirst, sstep, shi;
    xcd_wave_slices(A.nslices, wg, NW, __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE), sfirst, sstep, shi);
    uint32_t nrec = rec_word(A.srec, sfirst, shi);
    for (int64_t sl = sfirst; sl < shi; sl += sstep) {
        if (PRIO) progress_prio(sl - sfirst, shi - sfirst);
        const SliceRec rec = rec_from(nrec);
        nrec = rec_word(A.srec, sl + sstep, shi);
        const int lgL = LANES ? A.lgL : 0;
        const int64_t row = LANES ? sl * (SLICE >> lgL) + (lane >> lgL) : sl * SLICE + lane;
        const bool lead = !LANES || (lane & ((1 << lgL) - 1)) == 0;   // the lane that writes the row's results
        const uint32_t ru = (uint32_t)row, rowg = (uint32_t)(row + A.guard);   // < 2^31
        const int w = rec.width;
        const TZ pi = pval(rowg);
        if (pn && lead) st32(pn, ru, pi);
        if (lead) mp = fmax(mp, fabs((double)pi));
        const CA pic = (CA)pi;
        CA acc = (CA)0, dterm = (CA)0;
        auto add = [&](CA v, CA pj, bool dg, bool in) {
            if (UR == 64 || !DIFF) {
                const CA t = acc + v * pj;
                acc = in ? t : acc;
            } else {
                const CA td = dterm + v * pj;
                const CA to = acc + v * (pj - pic);
                dterm = (in && dg) ? td : dterm;
                acc = (in && !dg) ? to : acc;
            }
        };
        if (!LANES && rec.soff >= 0) {
            const KOffs ol = A.koffs + rec.soff;
            const CA *vs = vals + rec.ptr;   // the slice's values, slot j at vs[64 j + lane]
            // one pass over slots [j0, j0 + NC kChunk): offsets (scalar loads;
            // a chunk past the width reuses the first chunk's), then every
            // value load and gather, then the sums in slot order
            auto pass = [&](auto ncc, int j0) {
                constexpr int NC = decltype(ncc)::value, PS = NC * kChunk;
                int32_t o[PS];
#pragma unroll
                for (int ch = 0; ch < NC; ++ch) {
                    const int jc = (j0 + ch * kChunk < w) ? j0 + ch * kChunk : j0;
#pragma unroll
                    for (int u = 0; u < kChunk; ++u) o[ch * kChunk + u] = ol[jc + u];
                }
                CA v[PS];
                TZ pj[PS];
                const bool full = j0 + PS <= w;
#pragma unroll
                for (int u = 0; u < PS; ++u) {
                    const int j = full ? j0 + u : (j0 + u < w ? j0 + u : w - 1);
                    v[u] = at32t<NTL>(vs, (uint32_t)(lane + j * SLICE));
                    pj[u] = pval(rowg + (uint32_t)o[u]);
                }
#pragma unroll
                for (int u = 0; u < PS; ++u) add(v[u], (CA)pj[u], o[u] == 0, full || j0 + u < w);
            };
            // passes of NCH chunks while more than one chunk's slots remain,
            // then single chunks (short rows issue no repeated loads for a
            // second chunk)
            int j0 = 0;
            if constexpr (NCH > 1) {
                for (; w - j0 > kChunk; j0 += SPC) pass(std::integral_constant<int, NCH>{}, j0);
            }
            for (; j0 < w; j0 += kChunk) pass(std::integral_constant<int, 1>{}, j0);
        } else {
            const IdxCols sc{A.col + rec.ptr + lane, row};
            const int64_t base = rec.ptr + lane;
            for (int j0 = 0; j0 < w; j0 += kChunk) {
                int32_t c[kChunk];
                bool dg[kChunk];
                CA v[kChunk];
                TZ pj[kChunk];
                sc.chunk(j0, w, c, dg);
#pragma unroll
                for (int u = 0; u < kChunk; ++u) {
                    const int j = j0 + u < w ? j0 + u : w - 1;
                    v[u] = vals[base + (int64_t)j * SLICE];
                    pj[u] = pval((uint32_t)(c[u] + A.guard));
                }
#pragma unroll
                for (int u = 0; u < kChunk; ++u) add(v[u], (CA)pj[u], dg[u], j0 + u < w);
            }
        }
        if constexpr (LANES) {   // the row's total over its lanes
            acc = row_lanes_sum(acc, lgL);
            if (UR == 32 && DIFF) dterm = row_lanes_sum(dterm, lgL);
        }
        const TQ qq = (TQ)((UR == 32 && DIFF) ? dterm + acc : acc);
        if (lead) {
            st32(q, ru, qq);
            gam += (double)qq * (double)pi;
        }
    }
}

// UZF: the u_z of every iteration when the solve's options fix it (only
// that precision's bodies are compiled), else 0 (read from the state).  A
// state whose u_z differs from UZF can only come from a non-finite residual:
// it ends the solve as a breakdown.
template <int BS, bool PRIO = true, int UZF = 0, int SPC = AMP_SPMV_SPC, bool LANES = false, bool NTL = false>
__device__ __forceinline__ void spmv_stage(const Cfg &c, const Sell &A, const Bufs &B, const St *in, St *out,
                                           Wg wg, const Early &e) {
    __shared__ St s;
    PartRegs<2, BS> pr;
    load_parts<2, BS>(e.part, e.g, pr);   // in flight during the state load
    load_state(s, in);
    pin(e.touched);
    if (s.status != RUNNING) {
        store_state(s, out, wg);
        return;
    }
    // Every thread forms beta from the totals (no broadcast step); the state
    // fields it needs are read before the reduction's barriers, after which
    // only thread 0 writes the state.
    const double rho_prev = s.rho;
    const int k = s.k, uz = s.uz, ur = s.ur, ps = pslot(uz), pb = s.pbuf;
    double tot[2];
    reduce_loaded<1, 1, BS>(pr, e.g, tot);
    const double rho = tot[0], mz = tot[1];
    const double beta = (k > 0) ? rho / rho_prev : 0.0;
    const bool brk = !(rho > 0.0) || !isfinite(beta);
    if (threadIdx.x == 0) {
        s.rho_prev = rho_prev;
        s.rho = rho;
        s.beta = beta;
        s.maxz = mz;
        if (brk) s.status = BREAKDOWN;
        if (wg.lb == 0 && c.scalar_history) c.scalar_history[4 * k + 1] = rho;
    }
    if (brk) {
        store_state(s, out, wg);
        return;
    }
    if (c.spmv_iter && wg.lb == 0 && threadIdx.x == 0) c.spmv_iter[c.spmv_launch] = k;
    if (UZF != 0 && uz != UZF) {
        if (threadIdx.x == 0) s.status = BREAKDOWN;
        store_state(s, out, wg);
        return;
    }
    const bool first = (k == 0);
    double gam = 0.0, mp = 0.0;
#define AMP_SP(UZ, UR, DF)                                                                                \
    do {                                                                                                 \
        if (first)                                                                                       \
            spmv_p_body<UZ, UR, DF, true, BS, PRIO, SPC, LANES, NTL>(A, wg, B.z[ps], B.p[ps][pb],         \
                                                         B.p[ps][pb ^ 1], B.q[pslot(UR)], beta, gam, mp); \
        else                                                                                             \
            spmv_p_body<UZ, UR, DF, false, BS, PRIO, SPC, LANES, NTL>(A, wg, B.z[ps], B.p[ps][pb],        \
                                                          B.p[ps][pb ^ 1], B.q[pslot(UR)], beta, gam, mp); \
    } while (0)
#define AMP_SP_R(UZ)                          \
    do {                                      \
        if (ur == 64) AMP_SP(UZ, 64, false);  \
        else if (c.diff) AMP_SP(UZ, 32, true); \
        else AMP_SP(UZ, 32, false);           \
    } while (0)
    if constexpr (UZF == 64) AMP_SP_R(64);
    else if constexpr (UZF == 32) AMP_SP_R(32);
    else if constexpr (UZF == 16) AMP_SP_R(16);
    else {
        if (uz == 64) AMP_SP_R(64);
        else if (uz == 32) AMP_SP_R(32);
        else AMP_SP_R(16);
    }
#undef AMP_SP_R
#undef AMP_SP
    double v2[2] = {gam, mp};
    block_reduce<1, 1, BS>(v2);
    gam = v2[0];
    mp = v2[1];
    if (threadIdx.x == 0) {
        B.part_spmv[wg.lb] = gam;
        B.part_spmv[GMAX + wg.lb] = mp;
    }
    store_state(s, out, wg);
}

template <int UZF, bool LANES = false, bool NTL = false>
__global__ void __launch_bounds__(NTP, (UZF == 16 || UZF == 32) ? AMP_SPMV_WAVES : 4)
    k_spmv(const St *in, const double *part, int gpart, int grid, Cfg c, Sell A, Bufs B, St *out) {
    spmv_stage<NTP, true, UZF, AMP_SPMV_SPC, LANES, NTL>(
        c, A, B, in, out, launch_wg(grid),
        Early{part, gpart, nullptr, touch_args<24 + sizeof(Cfg) + sizeof(Sell) + sizeof(Bufs)>()});
}

typedef void (*SpmvFn)(const St *, const double *, int, int, Cfg, Sell, Bufs, St *);

// The product kernel for the options' fixed u_z (0: read from the state),
// the matrix's lanes per row (any layout with lanes > 1 takes the general
// u_z path: its long rows make the product bound by the values) and
// whether its values are streamed with a non-temporal hint.
inline SpmvFn spmv_fn(int uzf, bool lanes = false, bool nt = false) {
    if (lanes) return k_spmv<0, true>;
    switch (uzf) {
        case 16: return nt ? k_spmv<16, false, true> : k_spmv<16>;
        case 32: return nt ? k_spmv<32, false, true> : k_spmv<32>;
        case 64: return nt ? k_spmv<64, false, true> : k_spmv<64>;
        default: return nt ? k_spmv<0, false, true> : k_spmv<0>;
    }
}

// Stand-alone product (tests, measurement): with first = true, q = A z;
// otherwise p = z + beta p_old as in the iteration.
template <int UZ, int UR, bool DIFF, bool LANES = false>
__global__ void __launch_bounds__(NTS) k_spmv_fixed(Sell A, const void *z, const void *po, void *pn, void *q,
                                                   int first, double beta, double *part) {
    double gam = 0.0, mp = 0.0;
    const Wg wg = grid_wg();
    if (first) spmv_p_body<UZ, UR, DIFF, true, NTS, true, AMP_SPMV_SPC, LANES>(A, wg, z, po, pn, q, beta, gam, mp);
    else spmv_p_body<UZ, UR, DIFF, false, NTS, true, AMP_SPMV_SPC, LANES>(A, wg, z, po, pn, q, beta, gam, mp);
    gam = block_sum<NTS>(gam);
    if (threadIdx.x == 0 && part) part[wg.lb] = gam;
}

// ----------------------------------------------------------------------------
// k_update: x += alpha p (FP64), r -= alpha q (u_r); partials ||r||^2, max|r|
// ----------------------------------------------------------------------------

// The body loads for this thread's first two chunks are issued before the
// partials of gamma are reduced; the precisions come from the incoming state
// (the update does not change them).  XM: what happens to x (FP64).
//   0: nothing; alpha_k p_k becomes the pending step (x is not read)
//   1: x += alpha_k p_k
//   2: x += alpha_{k-1} p_{k-1}, then x += alpha_k p_k (p_{k-1} in u_z as p_k)
// Each step is rounded as on its own, so x is bitwise the same in all modes.
// ZQ: clear q after reading it (the matrix-free product sums into q).
template <int UP, int UR, int XM, bool ZQ = false>
__device__ __forceinline__ void update_run(const Cfg &c, const Bufs &B, int64_t np, St &s, const PartRegs<2> &pr,
                                           int gpart, St *out, Wg wg) {
    typedef typename Prec<UP>::T TP;
    typedef typename Prec<UR>::T TR;
    const int pbuf = s.pbuf, k = s.k;
    const double rho = s.rho;
    const TP *p = (const TP *)B.p[pslot(UP)][pbuf ^ 1];
    const TP *pq = (const TP *)B.p[pslot(UP)][s.x_pb];   // p_{k-1} (XM 2)
    const double aq = s.x_alpha;
    TR *r = (TR *)B.r[pslot(UR)];
    const TR *q = (const TR *)B.q[pslot(UR)];
    int64_t lo, hi;
    block_range(np, (int64_t)NT * VEC, wg.lb, wg.G, lo, hi);
    constexpr int64_t step = (int64_t)NT * VEC;
    const int64_t i0 = lo + (int64_t)threadIdx.x * VEC;
    // Chunks loaded ahead: two, or one when a chunk's operands are wide (the
    // registers for two would lower the number of resident waves).
    constexpr int chunk_bytes = VEC * ((XM >= 1 ? 8 + (int)sizeof(TP) : 0) + (XM == 2 ? (int)sizeof(TP) : 0) +
                                       2 * (int)sizeof(TR));
    constexpr int PF = chunk_bytes <= 112 ? 2 : 1;
    // chunks past this work-group's range load chunk 0 (unused): no branch
    const int64_t j0 = i0 < hi ? i0 : 0, j1 = i0 + step < hi ? i0 + step : 0;
    V4<TP> p0, p1, pq0, pq1;
    V4<double> x0, x1;
    V4<TR> r0, r1, q0, q1;
    if (XM >= 1) {
        p0 = ld4(p, j0);
        x0 = ld4(B.x, j0);
    }
    if (XM == 2) pq0 = ld4(pq, j0);
    r0 = ld4(r, j0);
    q0 = ld4(q, j0);
    if (PF == 2) {
        if (XM >= 1) {
            p1 = ld4(p, j1);
            x1 = ld4(B.x, j1);
        }
        if (XM == 2) pq1 = ld4(pq, j1);
        r1 = ld4(r, j1);
        q1 = ld4(q, j1);
    }
    // every thread forms alpha from the totals (the state fields it needs
    // were read above, before the reduction's barriers)
    double tot[2];
    reduce_loaded<1, 1>(pr, gpart, tot);
    const double gam = tot[0], mp = tot[1];
    const double alpha = rho / gam;
    const bool brk = !(gam > 0.0) || !isfinite(alpha);
    if (threadIdx.x == 0) {
        s.gamma = gam;
        s.alpha = alpha;
        s.maxp = mp;
        if (brk) s.status = BREAKDOWN;
        if (wg.lb == 0 && c.scalar_history) {
            c.scalar_history[4 * k + 2] = gam;
            c.scalar_history[4 * k + 3] = alpha;
        }
    }
    if (brk) {   // breakdown: x_k is the result; it gets its pending step
        __syncthreads();
        stop_flush(s, B, np, wg);
        store_state(s, out, wg);
        return;
    }
    const TR a = (TR)alpha;
    double dd = 0.0, mr = 0.0;
    auto chunk = [&](int64_t i, const V4<TP> &pv4, const V4<TP> &pqv, V4<double> xv, V4<TR> rv, const V4<TR> &qv) {
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
            if (XM == 2) xv.v[e] = xv.v[e] + aq * (double)pqv.v[e];
            if (XM >= 1) xv.v[e] = xv.v[e] + alpha * (double)pv4.v[e];
            const TR rn = (TR)(rv.v[e] - a * qv.v[e]);
            rv.v[e] = rn;
            dd += (double)rn * (double)rn;
            mr = fmax(mr, fabs((double)rn));
        }
        if (XM >= 1) st4(B.x, i, xv);
        st4(r, i, rv);
        if (ZQ) {
            V4<TR> zero;
#pragma unroll
            for (int e = 0; e < VEC; ++e) zero.v[e] = (TR)0;
            st4((TR *)q, i, zero);
        }
    };
    if (i0 < hi) chunk(i0, p0, pq0, x0, r0, q0);
    if (PF == 2 && i0 + step < hi) chunk(i0 + step, p1, pq1, x1, r1, q1);
    // the rest of the range (large systems): two chunks per pass with all
    // their loads issued first where two chunks were loaded ahead above
    // (the register budget is the same), else one
    int64_t i = i0 + PF * step;
    for (; PF == 2 && i + step < hi; i += 2 * step) {
        V4<TP> pa, pb, pqa, pqb;
        V4<double> xa, xb;
        if (XM >= 1) {
            pa = ld4(p, i);
            pb = ld4(p, i + step);
            xa = ld4(B.x, i);
            xb = ld4(B.x, i + step);
        }
        if (XM == 2) {
            pqa = ld4(pq, i);
            pqb = ld4(pq, i + step);
        }
        const V4<TR> ra = ld4(r, i), rb = ld4(r, i + step), qa = ld4(q, i), qb = ld4(q, i + step);
        chunk(i, pa, pqa, xa, ra, qa);
        chunk(i + step, pb, pqb, xb, rb, qb);
    }
    for (; i < hi; i += step) {
        V4<TP> pv4, pqv;
        V4<double> xv;
        if (XM >= 1) {
            pv4 = ld4(p, i);
            xv = ld4(B.x, i);
        }
        if (XM == 2) pqv = ld4(pq, i);
        chunk(i, pv4, pqv, xv, ld4(r, i), ld4(q, i));
    }
    double v2[2] = {dd, mr};
    block_reduce<1, 1>(v2);
    dd = v2[0];
    mr = v2[1];
    if (threadIdx.x == 0) {
        B.part_res[wg.lb] = dd;
        B.part_res[GMAX + wg.lb] = 0.0;
        B.part_res[2 * GMAX + wg.lb] = mr;
        if (XM == 0) {
            s.xp = 1;
            s.x_pu = UP;
            s.x_pb = pbuf ^ 1;
            s.x_alpha = alpha;
        } else {
            s.xp = 0;
        }
        s.pbuf = pbuf ^ 1;
        s.p_store = UP;
        s.iters = k + 1;
        s.kind = RES_UPDATE;
    }
    store_state(s, out, wg);
}

__device__ __forceinline__ void update_stage(const Cfg &c, const Bufs &B, int64_t np, const St *in, St *out,
                                             Wg wg, const Early &e) {
    __shared__ St s;
    PartRegs<2> pr;
    load_parts<2>(e.part, e.g, pr);   // in flight during the state load
    load_state(s, in);
    pin(e.touched);
    if (s.status != RUNNING) {   // stopped in the product kernel (breakdown)
        stop_flush(s, B, np, wg);
        store_state(s, out, wg);
        return;
    }
    const int uz = s.uz, ur = s.ur;
    int xm;
    if (s.xp && s.x_pu != uz) {   // pending step in another precision (a u_z switch): apply it first
        stop_flush(s, B, np, wg);
        xm = 1;
    } else {
        xm = s.xp ? 2 : (c.defer_x ? 0 : 1);
    }
#define AMP_UPD(UP, UR)                                                                    \
    do {                                                                                   \
        if (c.zero_q) update_run<UP, UR, 1, true>(c, B, np, s, pr, e.g, out, wg);          \
        else if (xm == 0) update_run<UP, UR, 0>(c, B, np, s, pr, e.g, out, wg);            \
        else if (xm == 1) update_run<UP, UR, 1>(c, B, np, s, pr, e.g, out, wg);            \
        else update_run<UP, UR, 2>(c, B, np, s, pr, e.g, out, wg);                         \
    } while (0)
    if (ur == 64) {
        if (uz == 64) AMP_UPD(64, 64);
        else if (uz == 32) AMP_UPD(32, 64);
        else AMP_UPD(16, 64);
    } else {
        if (uz == 64) AMP_UPD(64, 32);
        else if (uz == 32) AMP_UPD(32, 32);
        else AMP_UPD(16, 32);
    }
#undef AMP_UPD
}

__global__ void __launch_bounds__(NT) k_update(const St *in, const double *part, int gpart, int grid, Cfg c,
                                               Bufs B, int64_t np, St *out) {
    update_stage(c, B, np, in, out, launch_wg(grid),
                 Early{part, gpart, nullptr, touch_args<24 + sizeof(Cfg) + sizeof(Bufs)>()});
}

// ----------------------------------------------------------------------------
// k_true_res: t = b - A x (FP64).  mode 0: termination check (runs only when
// the state asks for it; r := fl(t) for a possible replacement); mode 1:
// periodic replacement of r (completes the iteration); mode 2: report only
// (writes nothing but partials).  Partials: ||t||^2, ||fl(t)||^2, max|fl(t)|.
// ----------------------------------------------------------------------------

template <int RS, int BS, bool LANES = false>
__device__ __forceinline__ void true_res_body(const Sell &A, const Bufs &B, Wg wg, bool write, double &st,
                                              double &ss, double &mr) {
    typedef typename Prec<RS>::T TR;
    TR *r = (TR *)B.r[pslot(RS)];
    const double *x = B.x;
    rows_dot64<BS, LANES>(A, wg, [&](int64_t c) { return x[c]; }, [&](int64_t row, int sub, double ax) {
        if (sub != 0) return;
        const double t = B.b[row] - ax;
        const TR tr = (TR)t;
        if (write) r[row] = tr;
        st += t * t;
        ss += (double)tr * (double)tr;
        mr = fmax(mr, fabs((double)tr));
    });
}

template <int BS, bool LANES = false>
__device__ __forceinline__ void true_res_stage(const Cfg &c, const Sell &A, const Bufs &B, int mode, const St *in,
                                               St *out, Wg wg) {
    __shared__ St s;
    load_state(s, in);
    const bool run = (mode == 0 && s.status == NEED_VERIFY) || (mode == 1 && s.status == RUNNING) || mode == 2;
    if (!run) {
        store_state(s, out, wg);
        return;
    }
    double st = 0.0, ss = 0.0, mr = 0.0;
    if (s.r_store == 64) true_res_body<64, BS, LANES>(A, B, wg, mode != 2, st, ss, mr);
    else true_res_body<32, BS, LANES>(A, B, wg, mode != 2, st, ss, mr);
    double v3[3] = {st, ss, mr};
    block_reduce<2, 1, BS>(v3);
    st = v3[0];
    ss = v3[1];
    mr = v3[2];
    if (threadIdx.x == 0) {
        B.part_res[wg.lb] = st;
        B.part_res[GMAX + wg.lb] = ss;
        B.part_res[2 * GMAX + wg.lb] = mr;
        if (mode == 0) {
            s.status = RUNNING;
            s.kind = RES_VERIFY;
        } else if (mode == 1) {
            s.kind = RES_PERIODIC;
        }
    }
    store_state(s, out, wg);
}

template <bool LANES>
__global__ void __launch_bounds__(NTS) k_true_res(Cfg c, Sell A, Bufs B, int mode, const St *in, St *out) {
    true_res_stage<NTS, LANES>(c, A, B, mode, in, out, grid_wg());
}

// ----------------------------------------------------------------------------
// single-work-group solve: the stages above in a loop inside one launch
// ----------------------------------------------------------------------------

// One work-group (NT threads) runs a whole solve from the state in
// st[ST_INIT] (r0 and its partials already formed with G = 1): the same
// stages, on the same state slots, in the same order as the host would
// enqueue them with one work-group per kernel (the product stage here with
// NT threads instead of NTS).  The loop ends when the state stops
// (converged, maxit, breakdown) or after `cap` passes; the last state is
// copied to st[ST_FIN] (with status MAXIT if the cap was reached while
// running).
// PRIO: issue priority by progress in the product stage (off where the
// work-groups sharing a CU belong to different systems).
template <bool PRIO = true>
__device__ __forceinline__ void solo_solve(const Cfg &c, const Sell &A, const Bufs &B, St *st, int cap) {
    const Wg wg{0, 1};
    __shared__ int status;
    int in = ST_INIT, last = ST_INIT;
    for (int pass = 0; pass < cap; ++pass) {
        precond_stage(c, A, B, A.np, st + in, st + ST_PRE, wg, res_early(c, B));
        __syncthreads();
        if (threadIdx.x == 0) status = st[ST_PRE].status;
        __syncthreads();
        last = ST_PRE;
        if (status == NEED_VERIFY) {
            true_res_stage<NT>(c, A, B, 0, st + ST_PRE, st + ST_TR, wg);
            __syncthreads();
            in = last = ST_TR;
            continue;
        }
        if (status != RUNNING) break;
        spmv_stage<NT, PRIO>(c, A, B, st + ST_PRE, st + ST_SPMV, wg, pre_early(c, B));
        __syncthreads();
        update_stage(c, B, A.np, st + ST_SPMV, st + ST_RES, wg, spmv_early(c, B));
        __syncthreads();
        in = last = ST_RES;
    }
    __shared__ St f;
    load_state(f, st + last);
    stop_flush(f, B, A.np, wg);   // the cap ends a running solve: x gets its pending step
    if (threadIdx.x == 0) {
        if (f.status == RUNNING || f.status == NEED_VERIFY) f.status = MAXIT;
        st[ST_FIN] = f;
    }
}

__global__ void __launch_bounds__(NT) k_solo(Cfg c, Sell A, Bufs B, St *st, int cap) { solo_solve(c, A, B, st, cap); }

// Fixed-order total of G partials into *out (one work-group).
__global__ void __launch_bounds__(NT) k_reduce_to(const double *part, int G, int is_max, double *out) {
    const double t = is_max ? reduce_max(part, G) : reduce_sum(part, G);
    if (threadIdx.x == 0) *out = t;
}

// ----------------------------------------------------------------------------
// stand-alone preconditioner application (tests / measurement)
// ----------------------------------------------------------------------------

template <int UR, int UZ>
__global__ void __launch_bounds__(NT) k_precond_fixed(Bufs B, int64_t np, double omega_eff, double *part) {
    typedef typename Prec<UR>::T TR;
    typedef typename Prec<UZ>::T TZ;
    typedef typename Prec<UZ>::C CZ;
    const TR *r = (const TR *)B.r[pslot(UR)];
    TZ *z = (TZ *)B.z[pslot(UZ)];
    const TZ *dv = (const TZ *)B.dinv[pslot(UZ)];
    const TR w = (TR)omega_eff;
    double rho = 0.0;
    const Wg wg = grid_wg();
    AMP_STREAM_LOOP(i, np, wg) {
        const V4<TR> rv = ld4(r, i);
        const V4<TZ> dd = ld4(dv, i);
        V4<TZ> zz;
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
            const TZ y = narrow<TZ>(rv.v[e] * w);
            zz.v[e] = (TZ)((CZ)y * (CZ)dd.v[e]);
            rho += (double)rv.v[e] * (double)zz.v[e];
        }
        st4(z, i, zz);
    }
    rho = block_sum(rho);
    if (threadIdx.x == 0) part[wg.lb] = rho;
}

}  // namespace amp
