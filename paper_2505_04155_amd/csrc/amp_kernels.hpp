// HIP kernels of one AMP-PCG iteration (Alg. 3), in the paper's order:
//   k_precond   y = omega r (u_r), z = M^{-1} y (u_z), rho = r^T z   -- "zamx" + "innerProd"
//   k_pupdate   p = z + beta p (u_z)                                 -- "axpy"
//   k_spmv      q = A p (u_r), gamma = q^T p                          -- "Ax"
//   k_update    x += alpha p (FP64), r -= alpha q (u_r), delta        -- "updatePCG"
// plus k_init (r0 = b - A x0) and k_true_res (FP64 b - A x, residual
// replacement).  Every kernel reads the precisions of the current iteration
// from the device-resident controller and dispatches with a uniform branch,
// so precision switches never need the host.  Scalars (rho, gamma, delta)
// are finished by the last work-group to arrive, which also runs the
// controller step.
#pragma once

#include "amp_device.hpp"

namespace amp {

// Pointers of every working vector, indexed by precision slot
// (0: FP64, 1: FP32, 2: FP16).  Vectors are padded to np elements.
struct Bufs {
    double *x;
    const double *b;
    void *r[3], *z[3], *p[3], *q[3];
    const void *dinv[3];
    double *part;   // 2 * GMAX partial sums
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

#define AMP_GRID_STRIDE(i, np)                                                            \
    for (int64_t i = ((int64_t)blockIdx.x * NT + threadIdx.x) * VEC; i < (np);           \
         i += (int64_t)gridDim.x * NT * VEC)

// ----------------------------------------------------------------------------
// controller epilogues (single thread of the last work-group)
// ----------------------------------------------------------------------------

__device__ inline void finish_iteration(Ctrl *c, double delta_new, double maxr_new) {
    const int it = c->iters;
    c->maxr_prev = c->maxr;
    c->maxr = maxr_new;
    c->delta = delta_new;
    c->ring[it % kRing] = delta_new;
    if (c->delta_history) c->delta_history[it] = delta_new;
    if (delta_new <= c->tol_b) {
        c->status = c->verify ? NEED_VERIFY : CONVERGED;
        return;
    }
    if (!isfinite(delta_new)) {
        c->status = BREAKDOWN;
        return;
    }
    if (it >= c->maxit) {
        c->status = MAXIT;
        return;
    }
    prepare_iteration(*c, it);
}

// ----------------------------------------------------------------------------
// sliced-ELL row products
// ----------------------------------------------------------------------------

// FP64 values, FP64 accumulation: sum_j a_ij p_j in slot order.
template <typename TP>
__device__ __forceinline__ double row_dot64(const Sell &A, int64_t base, int w, int64_t row,
                                            const TP *p) {
    double acc = 0.0;
    for (int j = 0; j < w; ++j) {
        const int64_t s = base + (int64_t)j * SLICE;
        acc += A.v64[s] * (double)p[A.col[s]];
    }
    return acc;
}

// FP32 values, FP32 accumulation.  DIFF: off-diagonal slots contribute
// a_ij (p_j - p_i) in slot order, then the diagonal slot's row sum s_i
// contributes s_i p_i; otherwise the textbook sum_j a_ij p_j.
template <typename TP, bool DIFF>
__device__ __forceinline__ float row_dot32(const Sell &A, int64_t base, int w, int64_t row,
                                           const TP *p) {
    float acc = 0.0f;
    if (DIFF) {
        const float pi = (float)p[row];
        float dterm = 0.0f;
        for (int j = 0; j < w; ++j) {
            const int64_t s = base + (int64_t)j * SLICE;
            const int32_t cj = A.col[s];
            const float v = A.v32[s];
            const float pj = (float)p[cj];
            if (cj == row) dterm = v * pj;
            else acc += v * (pj - pi);
        }
        acc = dterm + acc;
    } else {
        for (int j = 0; j < w; ++j) {
            const int64_t s = base + (int64_t)j * SLICE;
            acc += A.v32p[s] * (float)p[A.col[s]];
        }
    }
    return acc;
}

#define AMP_SLICE_LOOP(A, row, base, w)                                                   \
    const int lane_ = threadIdx.x % WAVE;                                                  \
    const int64_t wave0_ = (int64_t)blockIdx.x * (NT / WAVE) + threadIdx.x / WAVE;         \
    const int64_t wstride_ = (int64_t)gridDim.x * (NT / WAVE);                             \
    for (int64_t sl_ = wave0_; sl_ < (A).nslices; sl_ += wstride_)                         \
        for (int64_t base = (A).sptr[sl_] + lane_, row = sl_ * SLICE + lane_,             \
                     w = ((A).sptr[sl_ + 1] - (A).sptr[sl_]) / SLICE, once_ = 1;           \
             once_; once_ = 0)

// ----------------------------------------------------------------------------
// k_init: r0 = b - A x0 in FP64, ||b||^2, ||r0||^2, max|r0|
// ----------------------------------------------------------------------------

__global__ void __launch_bounds__(NT) k_init(Sell A, Bufs B, Ctrl *c) {
    double sb = 0.0, sr = 0.0, mr = 0.0;
    double *r = (double *)B.r[0];
    AMP_SLICE_LOOP(A, row, base, w) {
        const double t = B.b[row] - row_dot64(A, base, (int)w, row, B.x);
        r[row] = t;
        sb += B.b[row] * B.b[row];
        sr += t * t;
        mr = fmax(mr, fabs(t));
    }
    block_max_to(&c->maxbits[0], mr);
    double v[2] = {block_sum(sb), block_sum(sr)};
    if (arrive_last(c, B.part, v, 2)) {
        const double tb = finish_sum(B.part);
        const double tr = finish_sum(B.part + gridDim.x);
        if (threadIdx.x == 0) {
            c->counter = 0;
            c->bnorm = sqrt(tb);
            c->tol_b = c->tol * c->bnorm;
            c->delta = sqrt(tr);
            c->maxr = bits_to_double(c->maxbits[0]);
            c->maxr_prev = c->maxr;
            c->maxbits[0] = 0;
            c->ring[0] = c->delta;
            if (c->delta_history) c->delta_history[0] = c->delta;
            if (c->delta <= c->tol_b) c->status = CONVERGED;
            else if (c->maxit <= 0) c->status = MAXIT;
            else prepare_iteration(*c, 0);
        }
    }
}

// ----------------------------------------------------------------------------
// k_precond (Jacobi / identity): z = dinv (.) fl_uz(fl_ur(omega r)), rho = r^T z
// ----------------------------------------------------------------------------

template <int RS, int UR, int UZ>
__device__ __forceinline__ void precond_body(const Ctrl *c, const Bufs &B, int64_t np, double &rho,
                                             double &mz) {
    typedef typename Prec<RS>::T TRS;
    typedef typename Prec<UR>::T TR;
    typedef typename Prec<UZ>::T TZ;
    typedef typename Prec<UZ>::C CZ;
    const TRS *r = (const TRS *)B.r[pslot(RS)];
    TR *rn = (TR *)B.r[pslot(UR)];
    TZ *z = (TZ *)B.z[pslot(UZ)];
    const TZ *dv = (const TZ *)B.dinv[pslot(UZ)];
    const TR w = (TR)c->omega_eff;
    AMP_GRID_STRIDE(i, np) {
        const V4<TRS> rv = ld4(r, i);
        const V4<TZ> dd = ld4(dv, i);
        V4<TZ> zz;
        V4<TR> rr;
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
            const TR re = (TR)rv.v[e];
            rr.v[e] = re;
            const TZ y = (TZ)(re * w);                 // computed in u_r, stored in u_z
            const TZ ze = (TZ)((CZ)y * (CZ)dd.v[e]);   // computed and stored in u_z
            zz.v[e] = ze;
            rho += (double)re * (double)ze;
            mz = fmax(mz, fabs((double)ze));
        }
        st4(z, i, zz);
        if (RS != UR) st4(rn, i, rr);
    }
}

__global__ void __launch_bounds__(NT) k_precond(Bufs B, int64_t np, Ctrl *c) {
    if (c->status != RUNNING) return;
    const int rs = c->r_store, ur = c->ur, uz = c->uz;
    double rho = 0.0, mz = 0.0;
#define AMP_PC(RS, UR, UZ) precond_body<RS, UR, UZ>(c, B, np, rho, mz)
#define AMP_PC_Z(RS, UR)            \
    if (uz == 64) AMP_PC(RS, UR, 64); \
    else if (uz == 32) AMP_PC(RS, UR, 32); \
    else AMP_PC(RS, UR, 16);
    if (rs == 64 && ur == 64) { AMP_PC_Z(64, 64) }
    else if (rs == 64) { AMP_PC_Z(64, 32) }
    else { AMP_PC_Z(32, 32) }
#undef AMP_PC_Z
#undef AMP_PC
    block_max_to(&c->maxbits[1], mz);
    double v[1] = {block_sum(rho)};
    if (arrive_last(c, B.part, v, 1)) {
        const double t = finish_sum(B.part);
        if (threadIdx.x == 0) {
            c->counter = 0;
            c->r_store = c->ur;
            c->maxz = bits_to_double(c->maxbits[1]);
            c->maxbits[1] = 0;
            const double rp = c->rho;
            c->rho_prev = rp;
            c->rho = t;
            c->beta = (c->k > 0) ? t / rp : 0.0;
            if (!(t > 0.0) || !isfinite(c->beta)) c->status = BREAKDOWN;
        }
    }
}

// ----------------------------------------------------------------------------
// k_pupdate: p_k = z_k + beta p_{k-1} in u_z (p_{k-1} held in p_store)
// ----------------------------------------------------------------------------

template <int PS, int UZ>
__device__ __forceinline__ void pupdate_body(const Ctrl *c, const Bufs &B, int64_t np, double &mp) {
    typedef typename Prec<PS>::T TPS;
    typedef typename Prec<UZ>::T TZ;
    typedef typename Prec<UZ>::C CZ;
    const TPS *po = (const TPS *)B.p[pslot(PS)];
    TZ *pn = (TZ *)B.p[pslot(UZ)];
    const TZ *z = (const TZ *)B.z[pslot(UZ)];
    const bool first = (c->k == 0);
    const CZ beta = (CZ)c->beta;
    AMP_GRID_STRIDE(i, np) {
        const V4<TZ> zz = ld4(z, i);
        V4<TZ> pp;
        if (first) {
            pp = zz;
        } else {
            const V4<TPS> qo = ld4(po, i);
#pragma unroll
            for (int e = 0; e < VEC; ++e) pp.v[e] = (TZ)((CZ)zz.v[e] + beta * (CZ)qo.v[e]);
        }
#pragma unroll
        for (int e = 0; e < VEC; ++e) mp = fmax(mp, fabs((double)pp.v[e]));
        st4(pn, i, pp);
    }
}

__global__ void __launch_bounds__(NT) k_pupdate(Bufs B, int64_t np, Ctrl *c) {
    if (c->status != RUNNING) return;
    const int ps = (c->k == 0) ? c->uz : c->p_store, uz = c->uz;
    double mp = 0.0;
    if (ps == 64) {
        if (uz == 64) pupdate_body<64, 64>(c, B, np, mp);
        else if (uz == 32) pupdate_body<64, 32>(c, B, np, mp);
        else pupdate_body<64, 16>(c, B, np, mp);
    } else if (ps == 32) {
        if (uz == 32) pupdate_body<32, 32>(c, B, np, mp);
        else pupdate_body<32, 16>(c, B, np, mp);
    } else {
        pupdate_body<16, 16>(c, B, np, mp);
    }
    block_max_to(&c->maxbits[2], mp);
}

// ----------------------------------------------------------------------------
// k_spmv: q = A p (u_r), gamma = q^T p (FP64)
// ----------------------------------------------------------------------------

template <int UP, int UR, bool DIFF>
__device__ __forceinline__ void spmv_body(const Sell &A, const Bufs &B, double &gam) {
    typedef typename Prec<UP>::T TP;
    typedef typename Prec<UR>::T TQ;
    const TP *p = (const TP *)B.p[pslot(UP)];
    TQ *q = (TQ *)B.q[pslot(UR)];
    AMP_SLICE_LOOP(A, row, base, w) {
        TQ qv;
        if (UR == 64) qv = (TQ)row_dot64(A, base, (int)w, row, p);
        else qv = (TQ)row_dot32<TP, DIFF>(A, base, (int)w, row, p);
        q[row] = qv;
        gam += (double)qv * (double)p[row];
    }
}

template <int UP, int UR, bool DIFF>
__global__ void __launch_bounds__(NT) k_spmv_fixed(Sell A, Bufs B, double *gamma_out, Ctrl *c) {
    double gam = 0.0;
    spmv_body<UP, UR, DIFF>(A, B, gam);
    double v[1] = {block_sum(gam)};
    if (arrive_last(c, B.part, v, 1)) {
        const double t = finish_sum(B.part);
        if (threadIdx.x == 0) {
            c->counter = 0;
            if (gamma_out) *gamma_out = t;
        }
    }
}

__global__ void __launch_bounds__(NT) k_spmv(Sell A, Bufs B, int diff, Ctrl *c) {
    if (c->status != RUNNING) return;
    const int up = c->uz, ur = c->ur;
    double gam = 0.0;
    if (ur == 64) {
        if (up == 64) spmv_body<64, 64, false>(A, B, gam);
        else if (up == 32) spmv_body<32, 64, false>(A, B, gam);
        else spmv_body<16, 64, false>(A, B, gam);
    } else if (diff) {
        if (up == 64) spmv_body<64, 32, true>(A, B, gam);
        else if (up == 32) spmv_body<32, 32, true>(A, B, gam);
        else spmv_body<16, 32, true>(A, B, gam);
    } else {
        if (up == 64) spmv_body<64, 32, false>(A, B, gam);
        else if (up == 32) spmv_body<32, 32, false>(A, B, gam);
        else spmv_body<16, 32, false>(A, B, gam);
    }
    double v[1] = {block_sum(gam)};
    if (arrive_last(c, B.part, v, 1)) {
        const double t = finish_sum(B.part);
        if (threadIdx.x == 0) {
            c->counter = 0;
            c->gamma = t;
            c->alpha = c->rho / t;
            if (!(t > 0.0) || !isfinite(c->alpha)) c->status = BREAKDOWN;
        }
    }
}

// ----------------------------------------------------------------------------
// k_update: x += alpha p (FP64), r -= alpha q (u_r), delta = ||r||
// ----------------------------------------------------------------------------

template <int UP, int UR>
__device__ __forceinline__ void update_body(const Ctrl *c, const Bufs &B, int64_t np, double &dd,
                                            double &mr) {
    typedef typename Prec<UP>::T TP;
    typedef typename Prec<UR>::T TR;
    const TP *p = (const TP *)B.p[pslot(UP)];
    TR *r = (TR *)B.r[pslot(UR)];
    const TR *q = (const TR *)B.q[pslot(UR)];
    const double alpha = c->alpha;
    const TR a = (TR)alpha;
    AMP_GRID_STRIDE(i, np) {
        const V4<TP> pv = ld4(p, i);
        V4<double> xv = ld4(B.x, i);
        V4<TR> rv = ld4(r, i);
        const V4<TR> qv = ld4(q, i);
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
            xv.v[e] = xv.v[e] + alpha * (double)pv.v[e];
            const TR rn = (TR)(rv.v[e] - a * qv.v[e]);
            rv.v[e] = rn;
            dd += (double)rn * (double)rn;
            mr = fmax(mr, fabs((double)rn));
        }
        st4(B.x, i, xv);
        st4(r, i, rv);
    }
}

__global__ void __launch_bounds__(NT) k_update(Bufs B, int64_t np, Ctrl *c) {
    if (c->status != RUNNING) return;
    const int up = c->uz, ur = c->ur;
    double dd = 0.0, mr = 0.0;
    if (ur == 64) {
        if (up == 64) update_body<64, 64>(c, B, np, dd, mr);
        else if (up == 32) update_body<32, 64>(c, B, np, dd, mr);
        else update_body<16, 64>(c, B, np, dd, mr);
    } else {
        if (up == 64) update_body<64, 32>(c, B, np, dd, mr);
        else if (up == 32) update_body<32, 32>(c, B, np, dd, mr);
        else update_body<16, 32>(c, B, np, dd, mr);
    }
    block_max_to(&c->maxbits[0], mr);
    double v[1] = {block_sum(dd)};
    if (arrive_last(c, B.part, v, 1)) {
        const double t = finish_sum(B.part);
        if (threadIdx.x == 0) {
            c->counter = 0;
            const double mrr = bits_to_double(c->maxbits[0]);
            c->maxbits[0] = 0;
            c->maxp = bits_to_double(c->maxbits[2]);
            c->maxbits[2] = 0;
            c->p_store = c->uz;
            c->iters = c->k + 1;
            if (c->rr_period > 0 && c->iters % c->rr_period == 0) {
                c->rr_pending = 1;     // k_true_res (mode 1) completes the iteration
            } else {
                finish_iteration(c, sqrt(t), mrr);
            }
        }
    }
}

// ----------------------------------------------------------------------------
// k_true_res: t = b - A x (FP64).  mode 0: termination check (with
// replacement of r by t when the check fails); mode 1: periodic replacement
// that completes the iteration (runs only when k_update deferred to it).
// r is written as fl_{r_store}(t).
// ----------------------------------------------------------------------------

template <int RS>
__device__ __forceinline__ void true_res_body(const Sell &A, const Bufs &B, double &st, double &ss,
                                              double &mr) {
    typedef typename Prec<RS>::T TR;
    TR *r = (TR *)B.r[pslot(RS)];
    AMP_SLICE_LOOP(A, row, base, w) {
        const double t = B.b[row] - row_dot64(A, base, (int)w, row, B.x);
        const TR tr = (TR)t;
        r[row] = tr;
        st += t * t;
        ss += (double)tr * (double)tr;
        mr = fmax(mr, fabs((double)tr));
    }
}

__global__ void __launch_bounds__(NT) k_true_res(Sell A, Bufs B, int mode, Ctrl *c) {
    if (mode == 0 && c->status != NEED_VERIFY) return;
    if (mode == 1 && (c->status != RUNNING || c->rr_pending == 0)) return;
    double st = 0.0, ss = 0.0, mr = 0.0;
    if (c->r_store == 64) true_res_body<64>(A, B, st, ss, mr);
    else true_res_body<32>(A, B, st, ss, mr);
    block_max_to(&c->maxbits[3], mr);
    double v[2] = {block_sum(st), block_sum(ss)};
    if (arrive_last(c, B.part, v, 2)) {
        const double tt = finish_sum(B.part);
        const double ts = finish_sum(B.part + gridDim.x);
        if (threadIdx.x == 0) {
            c->counter = 0;
            const double mrr = bits_to_double(c->maxbits[3]);
            c->maxbits[3] = 0;
            c->true_res = sqrt(tt);
            if (mode == 1) {
                c->rr_pending = 0;
                c->n_repl += 1;
                finish_iteration(c, sqrt(ts), mrr);
            } else if (c->true_res <= c->tol_b) {
                c->status = CONVERGED;
            } else if (c->n_repl >= c->max_repl) {
                c->status = MAXIT;
            } else {
                c->n_repl += 1;
                const double dn = sqrt(ts);
                const int it = c->iters;
                c->delta = dn;
                c->maxr = mrr;
                c->ring[it % kRing] = dn;
                if (c->delta_history) c->delta_history[it] = dn;
                if (it >= c->maxit) {
                    c->status = MAXIT;
                } else {
                    c->status = RUNNING;
                    prepare_iteration(*c, it);
                }
            }
        }
    }
}

// ----------------------------------------------------------------------------
// standalone preconditioner application (tests / measurement)
// ----------------------------------------------------------------------------

template <int UR, int UZ>
__global__ void __launch_bounds__(NT) k_precond_fixed(Bufs B, int64_t np, double omega_eff,
                                                      double *rho_out, Ctrl *c) {
    typedef typename Prec<UR>::T TR;
    typedef typename Prec<UZ>::T TZ;
    typedef typename Prec<UZ>::C CZ;
    const TR *r = (const TR *)B.r[pslot(UR)];
    TZ *z = (TZ *)B.z[pslot(UZ)];
    const TZ *dv = (const TZ *)B.dinv[pslot(UZ)];
    const TR w = (TR)omega_eff;
    double rho = 0.0;
    AMP_GRID_STRIDE(i, np) {
        const V4<TR> rv = ld4(r, i);
        const V4<TZ> dd = ld4(dv, i);
        V4<TZ> zz;
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
            const TZ y = (TZ)(rv.v[e] * w);
            zz.v[e] = (TZ)((CZ)y * (CZ)dd.v[e]);
            rho += (double)rv.v[e] * (double)zz.v[e];
        }
        st4(z, i, zz);
    }
    double v[1] = {block_sum(rho)};
    if (arrive_last(c, B.part, v, 1)) {
        const double t = finish_sum(B.part);
        if (threadIdx.x == 0) {
            c->counter = 0;
            if (rho_out) *rho_out = t;
        }
    }
}

}  // namespace amp
