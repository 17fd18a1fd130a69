// Chebyshev polynomial preconditioner: z = D^{-1/2} s(B) D^{-1/2} y with
// B = D^{-1/2} A D^{-1/2} stored in FP16 on A's sliced-ELL pattern, s the
// degree-(m-1) polynomial whose residual polynomial 1 - t s(t) is the scaled
// Chebyshev polynomial T_m((theta - t)/delta) / T_m(theta/delta) on
// [lam_lo, lam_hi], evaluated by the three-term Chebyshev iteration for
// B w = v from w = 0:
//   res_0 = v, dir_0 = v / theta, w_0 = 0;  for k = 0..m-2:
//   w_{k+1} = w_k + dir_k,  res_{k+1} = res_k - B dir_k,
//   dir_{k+1} = c1_k dir_k + c2_k res_{k+1};   w_m = w_{m-1} + dir_{m-1}.
// Work vectors are held in the arithmetic precision of u_z (FP64, or FP32
// for u_z = FP32 / FP16); B products accumulate in that precision; z is
// rounded to u_z.  One streaming kernel forms v, then m-1 product kernels
// each take one step; the last one also forms z and the partials of rho.
#pragma once

#include "amp_kernels.hpp"

namespace amp {

constexpr int kChebMax = 16;

struct Cheb {
    const SliceRec *srec;
    const int64_t *sptr;
    const int32_t *col;
    const int32_t *soff, *offs;
    const half_t *b16;       // B's values in FP16
    const double *isq64;     // D^{-1/2}
    const float *isq32;
    void *v, *res, *w;       // work vectors (np doubles each, read as float for FP32)
    void *dir[2];
    int64_t np, nslices;
    int32_t *step_iter;      // nullable: iteration each timed step launch performed (-1: passed through)
    int step_launch;         // index of this launch in step_iter
    int degree;
    double inv_theta;
    double c1[kChebMax], c2[kChebMax];
};

// y = fl_uz(fl_ur(omega r)); v = isq (.) y in the work precision C.
template <int RS, int UR, int UZ>
__device__ __forceinline__ void cheb_v_body(const St &s, const Bufs &B, const Cheb &P, Wg wg) {
    typedef typename Prec<RS>::T TRS;
    typedef typename Prec<UR>::T TR;
    typedef typename Prec<UZ>::T TZ;
    typedef typename Prec<UZ>::C CZ;
    const TRS *r = (const TRS *)B.r[pslot(RS)];
    TR *rn = (TR *)B.r[pslot(UR)];
    CZ *v = (CZ *)P.v;
    const CZ *isq = (UZ == 64) ? (const CZ *)P.isq64 : (const CZ *)P.isq32;
    const TR w = (TR)s.omega_eff;
    AMP_STREAM_LOOP(i, P.np, wg) {
        const V4<TRS> rv = ld4(r, i);
        const V4<CZ> iv = ld4(isq, i);
        V4<CZ> vv;
        V4<TR> rr;
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
            const TR re = (TR)rv.v[e];
            rr.v[e] = re;
            const TZ y = narrow<TZ>(re * w);
            vv.v[e] = iv.v[e] * (CZ)y;
        }
        st4(v, i, vv);
        if (RS != UR) st4(rn, i, rr);
    }
}

// First kernel of a Chebyshev application inside the iteration: controller
// prologue (like k_precond), then v.  standalone != 0 skips the prologue and
// uses the incoming state's precisions and omega as given.
__global__ void __launch_bounds__(NT) k_cheb_init(Cfg c, Bufs B, Cheb P, int standalone, const St *in, St *out,
                                                  Sell A) {
    __shared__ St s;
    const Wg wg = grid_wg();
    ResIn ri;
    if (!standalone) res_loads(res_early(c, B), ri);
    load_state(s, in);
    if (s.status != RUNNING) {
        if (!standalone) stop_flush(s, B, P.np, wg);
        store_state(s, out, wg);
        return;
    }
    if (!standalone) {
        consume_residual(s, c, B, wg, ri);
        __syncthreads();
        if (s.status != RUNNING) {   // the solve stops here: x gets its pending step
            stop_flush(s, B, P.np, wg);
            store_state(s, out, wg);
            return;
        }
    }
    int rs = s.r_store;
    const int ur = s.ur, uz = s.uz;
    if (!standalone && switch_replaces(c, s)) {   // r_k := fl32(b - A x_k)
        switch_replace(A, B, s, P.np, wg);
        rs = 32;
        if (threadIdx.x == 0) s.n_repl += 1;
    }
#define AMP_CV(RS, UR, UZ) cheb_v_body<RS, UR, UZ>(s, B, P, wg)
#define AMP_CV_Z(RS, UR)                  \
    if (uz == 64) AMP_CV(RS, UR, 64);       \
    else if (uz == 32) AMP_CV(RS, UR, 32);  \
    else AMP_CV(RS, UR, 16);
    if (rs == 64 && ur == 64) { AMP_CV_Z(64, 64) }
    else if (rs == 64) { AMP_CV_Z(64, 32) }
    else { AMP_CV_Z(32, 32) }
#undef AMP_CV_Z
#undef AMP_CV
    const bool conv = (s.k > 0 && s.p_store != uz);
    if (conv) {
        if (s.p_store == 64 && uz == 32) convert_p<64, 32>(B, s.pbuf, P.np, wg);
        else if (s.p_store == 64) convert_p<64, 16>(B, s.pbuf, P.np, wg);
        else convert_p<32, 16>(B, s.pbuf, P.np, wg);
    }
    if (threadIdx.x == 0) {
        s.r_store = s.ur;
        if (conv) s.p_store = uz;
    }
    store_state(s, out, wg);
}

// One step k of the recurrence for this work-group's slices.
// RLAST: 0 for an inner step; for the last step, the precision of r (the
// step then forms z and the partials of rho = r^T z).
template <int UZ, bool FIRST, int RLAST, int BS>
__device__ __forceinline__ void cheb_step_body(const St &s, const Bufs &B, const Cheb &P, Wg wg, int k, int din,
                                               double &rho, double &mz) {
    typedef typename Prec<UZ>::T TZ;
    typedef typename Prec<UZ>::C CZ;
    const CZ *v = (const CZ *)P.v;
    CZ *res = (CZ *)P.res;
    CZ *w = (CZ *)P.w;
    const CZ *dk = (const CZ *)P.dir[din];
    CZ *dn = (CZ *)P.dir[din ^ 1];
    const CZ inv_theta = (CZ)P.inv_theta;
    const CZ c1 = (CZ)P.c1[k], c2 = (CZ)P.c2[k];
    const CZ *isq = (UZ == 64) ? (const CZ *)P.isq64 : (const CZ *)P.isq32;
    TZ *z = (TZ *)B.z[pslot(UZ)];
    typedef typename Prec<(RLAST == 64 ? 64 : 32)>::T TRL;
    const TRL *rl = (const TRL *)B.r[pslot(RLAST == 64 ? 64 : 32)];
    const bool first = FIRST;
    constexpr bool last = RLAST != 0;
    auto dval = [&](int64_t j) -> CZ {
        if (FIRST) return v[j] * inv_theta;
        return dk[j];
    };
    AMP_SLICE_LOOP(P, sl, wg, BS) {
        progress_prio(sl - slo_, shi_ - slo_);
        AMP_SLICE_ROW(P, sl, lane, row, base, wd, BS);
        // the row's own operands are loaded before the product, so their
        // latency overlaps it
        const CZ d0 = dval(row);
        const CZ wk = first ? (CZ)0 + d0 : w[row];
        const CZ rk = first ? v[row] : res[row];
        CZ isq_r = (CZ)0;
        double rr = 0.0;
        if (last) {
            isq_r = isq[row];
            rr = (double)rl[row];
        }
        CZ acc = (CZ)0;
        // two chunks of slots per pass: all their value loads and gathers are
        // issued before the first product is added (slots past the width
        // repeat a valid slot's loads and add nothing; the sum runs in slot
        // order)
        with_rec_cols(rec_, P.col, P.offs, P.np, sl, lane, [&](const auto &sc) {
            for (int j0 = 0; j0 < wd; j0 += 2 * kChunk) {
                int32_t cc[2 * kChunk];
                bool dg[2 * kChunk];
                CZ bv[2 * kChunk], dj[2 * kChunk];
                sc.chunk(j0, wd, cc, dg);
                sc.chunk(j0 + kChunk < wd ? j0 + kChunk : j0, wd, cc + kChunk, dg + kChunk);
#pragma unroll
                for (int u = 0; u < 2 * kChunk; ++u) {
                    const int j = j0 + u < wd ? j0 + u : wd - 1;
                    bv[u] = (CZ)P.b16[base + (int64_t)j * SLICE];
                    dj[u] = dval(cc[u]);
                }
#pragma unroll
                for (int u = 0; u < 2 * kChunk; ++u) {
                    const CZ t = acc + bv[u] * dj[u];
                    acc = (j0 + u < wd) ? t : acc;
                }
            }
        });
        const CZ w1 = first ? wk : wk + d0;
        const CZ r1 = rk - acc;
        const CZ d1 = c1 * d0 + c2 * r1;
        if (!last) {
            w[row] = w1;
            res[row] = r1;
            dn[row] = d1;
        } else {
            const CZ wm = w1 + d1;
            const TZ zz = (TZ)(isq_r * wm);
            z[row] = zz;
            rho += rr * (double)zz;
            mz = fmax(mz, fabs((double)zz));
        }
    }
}

__global__ void __launch_bounds__(NTS) k_cheb_step(Bufs B, Cheb P, int k, int first, int last, int din,
                                                  const St *in, St *out) {
    __shared__ St s;
    const Wg wg = grid_wg();
    load_state(s, in);
    if (s.status != RUNNING) {
        store_state(s, out, wg);
        return;
    }
    if (P.step_iter && wg.lb == 0 && threadIdx.x == 0) P.step_iter[P.step_launch] = s.k;
    double rho = 0.0, mz = 0.0;
#define AMP_CS_L(UZ, RL)                                                                \
    do {                                                                                \
        if (first) cheb_step_body<UZ, true, RL, NTS>(s, B, P, wg, k, din, rho, mz);     \
        else cheb_step_body<UZ, false, RL, NTS>(s, B, P, wg, k, din, rho, mz);          \
    } while (0)
#define AMP_CS(UZ)                                                      \
    do {                                                                \
        if (!last) AMP_CS_L(UZ, 0);                                     \
        else if (s.ur == 64) AMP_CS_L(UZ, 64);                          \
        else AMP_CS_L(UZ, 32);                                          \
    } while (0)
    if (s.uz == 64) AMP_CS(64);
    else if (s.uz == 32) AMP_CS(32);
    else AMP_CS(16);
#undef AMP_CS
#undef AMP_CS_L
    if (last) {
        double v2[2] = {rho, mz};
        block_reduce<1, 1, NTS>(v2);
        rho = v2[0];
        mz = v2[1];
        if (threadIdx.x == 0) {
            B.part_pre[wg.lb] = rho;
            B.part_pre[GMAX + wg.lb] = mz;
        }
    }
    store_state(s, out, wg);
}

// Degree 1: z = fl_uz(isq (.) (v / theta)), no product with B.
template <int UZ>
__device__ __forceinline__ void cheb_deg1_body(const St &s, const Bufs &B, const Cheb &P, Wg wg, double &rho,
                                               double &mz) {
    typedef typename Prec<UZ>::T TZ;
    typedef typename Prec<UZ>::C CZ;
    const CZ *v = (const CZ *)P.v;
    const CZ *isq = (UZ == 64) ? (const CZ *)P.isq64 : (const CZ *)P.isq32;
    const CZ inv_theta = (CZ)P.inv_theta;
    TZ *z = (TZ *)B.z[pslot(UZ)];
    AMP_STREAM_LOOP(i, P.np, wg) {
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
            const CZ d0 = v[i + e] * inv_theta;
            const CZ wm = (CZ)0 + d0;
            const TZ zz = (TZ)(isq[i + e] * wm);
            z[i + e] = zz;
            const double rr = (s.ur == 64) ? ((const double *)B.r[0])[i + e] : (double)((const float *)B.r[1])[i + e];
            rho += rr * (double)zz;
            mz = fmax(mz, fabs((double)zz));
        }
    }
}

__global__ void __launch_bounds__(NT) k_cheb_deg1(Bufs B, Cheb P, const St *in, St *out) {
    __shared__ St s;
    const Wg wg = grid_wg();
    load_state(s, in);
    if (s.status != RUNNING) {
        store_state(s, out, wg);
        return;
    }
    double rho = 0.0, mz = 0.0;
    if (s.uz == 64) cheb_deg1_body<64>(s, B, P, wg, rho, mz);
    else if (s.uz == 32) cheb_deg1_body<32>(s, B, P, wg, rho, mz);
    else cheb_deg1_body<16>(s, B, P, wg, rho, mz);
    double v2[2] = {rho, mz};
    block_reduce<1, 1>(v2);
    rho = v2[0];
    mz = v2[1];
    if (threadIdx.x == 0) {
        B.part_pre[wg.lb] = rho;
        B.part_pre[GMAX + wg.lb] = mz;
    }
    store_state(s, out, wg);
}

// Setup: B's FP16 values on A's slots, b_ij = fl16((a_ij isq_i) isq_j);
// isq = 1/sqrt(diag).  Partials of max isq for the scaling gain.
__global__ void __launch_bounds__(NT) k_cheb_isq(const double *diag, int64_t n, int64_t np, double *isq64,
                                                 float *isq32, double *part) {
    double m = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < np; i += (int64_t)gridDim.x * NT) {
        const double v = (i < n) ? 1.0 / sqrt(diag[i]) : 0.0;
        isq64[i] = v;
        isq32[i] = (float)v;
        m = fmax(m, v);
    }
    m = block_max(m);
    if (threadIdx.x == 0) part[blockIdx.x] = m;
}

__global__ void __launch_bounds__(NTS) k_cheb_values(Sell A, const double *isq64, half_t *b16) {
    int64_t slo_, shi_;
    block_range(A.nslices, 1, xcd_block(), gridDim.x, slo_, shi_);
    const int64_t sfirst_ = slo_ + __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
    uint32_t nrec_ = rec_word(A.srec, sfirst_, shi_);
    for (int64_t sl = sfirst_; sl < shi_; sl += NTS / WAVE) {
        AMP_SLICE_ROW(A, sl, lane, row, base, w, NTS);
        const double si = isq64[row];
        AMP_WITH_COLS(A, sl, lane, sc) {
            for (int j0 = 0; j0 < w; j0 += kChunk) {
                int32_t cc[kChunk];
                bool dg[kChunk];
                sc.chunk(j0, w, cc, dg);
                for (int u = 0; u < kChunk && j0 + u < w; ++u) {
                    const int64_t sidx = base + (int64_t)(j0 + u) * SLICE;
                    b16[sidx] = narrow<half_t>((A.v64[sidx] * si) * isq64[cc[u]]);
                }
            }
        });
    }
}

}  // namespace amp
