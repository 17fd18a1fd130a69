// Chebyshev polynomial preconditioner: z = D^{-1/2} s(B) D^{-1/2} y with
// B = D^{-1/2} A D^{-1/2} stored in FP16 on A's sliced-ELL pattern, s the
// degree-(m-1) polynomial whose residual polynomial 1 - t s(t) is the scaled
// Chebyshev polynomial T_m((theta - t)/delta) / T_m(theta/delta) on
// [lam_lo, lam_hi], evaluated by the Chebyshev iteration for B w = v from
// w = 0 written on its iterates (with d_k = x_{k+1} - x_k and
// res_k = v - B x_k it is the direction form d_k = c1 d_{k-1} + c2 res_k):
//   x_0 = 0, x_1 = v / theta;  for k = 1..m-1:
//   x_{k+1} = x_k + c1_{k-1} (x_k - x_{k-1}) + c2_{k-1} (v - B x_k);  w = x_m.
// A step reads the gathered x_k, v and x_{k-1} of its row and writes
// x_{k+1} over x_{k-1}: 16 bytes per row in FP32 where the direction form
// moves 24 (x_1 is v / theta, so the first two steps read less).  Work
// vectors are held in the arithmetic precision of u_z (FP64, or FP32 for
// u_z = FP32 / FP16); B products accumulate in that precision; z is rounded
// to u_z.  One streaming kernel forms v, then m-1 product kernels each take
// one step; the last one also forms z and the partials of rho.
//
// The gathered vectors (v and the two iterate buffers) of each precision are separate allocations
// with a zero margin of `guard` elements before and after (guard >= the
// largest |column offset| of any offset-mode slice).  An offset-mode slot
// then reads its neighbour at row + offset without a range test: a slot
// whose neighbour lies outside [0, np) has B value 0 and reads a zero of the
// margin.  Each such gather addresses a wave-uniform base (vector + offset)
// plus one per-lane row offset shared by all slots, and each FP16 value load
// the slice's uniform base plus the lane's offset.
#pragma once

#include "amp_kernels.hpp"

namespace amp {

constexpr int kChebMax = 16;

// Threads of the polynomial-step kernel and the minimum waves per SIMD it
// is compiled for (8 caps it at 64 VGPRs: 8 work-groups' worth of loads in
// flight per CU instead of 4).
#ifndef AMP_NTC
#define AMP_NTC 512
#endif
constexpr int NTC = AMP_NTC;
#ifndef AMP_CHEB_WAVES
#define AMP_CHEB_WAVES 8
#endif
// 1: slices dealt to waves round-robin within each XCD's share
// (xcd_wave_slices); 0: contiguous ranges per work-group
#ifndef AMP_CHEB_STRIDED
#define AMP_CHEB_STRIDED 1
#endif

struct Cheb {
    const SliceRec *srec;
    const int64_t *sptr;
    const int32_t *col;
    const int32_t *soff, *offs;
    KOffs koffs;             // offs, for the scalar reads of the step kernel
    const half_t *b16;       // B's values in FP16
    const double *isq64;     // D^{-1/2}
    const float *isq32;
    // work vectors by precision (0: FP64, 1: FP32), np entries each, with
    // the zero margins described above: v, and the two iterate buffers
    void *v[2];
    void *dir[2][2];
    int64_t np, nslices;
    int64_t guard;           // zero margin of v and dir, in elements
    int nt;                  // 1: B and the rows' own vectors loaded with a non-temporal hint (B exceeds kMallBytes)
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
    CZ *v = (CZ *)P.v[UZ == 64 ? 0 : 1];
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
// NTL: B and the row's own vector entries (read once per launch) are loaded
// with a non-temporal hint; for a B larger than the memory-side cache.
template <int UZ, bool FIRST, int RLAST, int BS, bool NTL>
__device__ __forceinline__ void cheb_step_body(const St &s, const Bufs &B, const Cheb &P, Wg wg, double c1d,
                                               double c2d, int din, double &rho, double &mz) {
    typedef typename Prec<UZ>::T TZ;
    typedef typename Prec<UZ>::C CZ;
    constexpr int cp = (UZ == 64) ? 0 : 1;
    const CZ *v = (const CZ *)P.v[cp];
    // step kk (0-based) of the iterate form: x_{kk+1} is gathered (kk = 0:
    // v / theta); x_{kk} is read and x_{kk+2} written in the other buffer.
    // din bit 0: kk odd (x_{kk+1} in dir[0]); bit 1: kk = 1 (x_{kk} = x_1 =
    // v / theta, formed from v).  (Selects, not indexing: an argument array
    // indexed at run time would be copied to private memory.)
    const bool odd = (din & 1) != 0, prev_from_v = (din & 2) != 0;
    const CZ *xk_buf = (const CZ *)(odd ? P.dir[cp][0] : P.dir[cp][1]);
    CZ *xw = (CZ *)(odd ? P.dir[cp][1] : P.dir[cp][0]);
    const CZ *g = FIRST ? v : xk_buf;   // the gathered vector
    const CZ inv_theta = (CZ)P.inv_theta;
    const CZ c1 = (CZ)c1d, c2 = (CZ)c2d;
    const CZ *isq = (UZ == 64) ? (const CZ *)P.isq64 : (const CZ *)P.isq32;
    TZ *z = (TZ *)B.z[pslot(UZ)];
    typedef typename Prec<(RLAST == 64 ? 64 : 32)>::T TRL;
    const TRL *rl = (const TRL *)B.r[pslot(RLAST == 64 ? 64 : 32)];
    constexpr bool last = RLAST != 0;
    // the direction at a gathered entry (the first step's is v / theta)
    auto dfrom = [&](CZ gv) -> CZ { return FIRST ? gv * inv_theta : gv; };
#if AMP_CHEB_STRIDED
    int64_t sfirst_, sstep_, shi_;
    xcd_wave_slices(P.nslices, wg, BS / WAVE, __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE), sfirst_, sstep_,
                    shi_);
    uint32_t nrec_ = rec_word(P.srec, sfirst_, shi_);
    for (int64_t sl = sfirst_; sl < shi_; sl += sstep_) {
        progress_prio(sl - sfirst_, shi_ - sfirst_);
        const SliceRec rec_ = rec_from(nrec_);
        nrec_ = rec_word(P.srec, sl + sstep_, shi_);
        const int lane = threadIdx.x % WAVE;
        const int64_t row = sl * SLICE + lane, base = rec_.ptr + lane;
        const int wd = rec_.width;
#else
    AMP_SLICE_LOOP(P, sl, wg, BS) {
        progress_prio(sl - slo_, shi_ - slo_);
        AMP_SLICE_ROW(P, sl, lane, row, base, wd, BS);
#endif
        // the row's own operands are loaded before the product, so their
        // latency overlaps it
        const uint32_t ru = (uint32_t)row;   // row < np <= 2^29: 32-bit byte offsets
        const CZ gi = at32(g, ru);
        const CZ xk = dfrom(gi);                           // x_k of the row
        const CZ vi = FIRST ? gi : at32t<NTL>(v, ru);
        CZ xkm1;                                           // x_{k-1} of the row
        if (FIRST) xkm1 = (CZ)0;
        else if (prev_from_v) xkm1 = vi * inv_theta;
        else xkm1 = at32t<NTL>((const CZ *)xw, ru);
        CZ isq_r = (CZ)0;
        double rr = 0.0;
        if (last) {
            isq_r = at32t<NTL>(isq, ru);
            rr = (double)at32t<NTL>(rl, ru);
        }
        CZ acc = (CZ)0;
        // two chunks of slots per pass: all their value loads and gathers are
        // issued before the first product is added (slots past the width
        // repeat a valid slot's loads and add nothing; the sum runs in slot
        // order)
        if (rec_.soff >= 0) {
            // the gathered entry of slot j is gb[rowg + offset_j]: gb is the
            // start of the vector's leading margin, rowg = row + guard, so the
            // index is never negative and one 32-bit add forms each offset
            const KOffs ol = P.koffs + rec_.soff;
            const half_t *bsl = P.b16 + rec_.ptr;   // the slice's values, slot j at bsl[64 j + lane]
            const CZ *gb = g - P.guard;
            const uint32_t rowg = (uint32_t)(row + P.guard);
            for (int j0 = 0; j0 < wd; j0 += 2 * kChunk) {
                const bool full = j0 + 2 * kChunk <= wd;
                const int j1 = j0 + kChunk < wd ? j0 + kChunk : j0;
                OffChunk oa, ob;   // scalar loads
#pragma unroll
                for (int u = 0; u < kChunk; ++u) {
                    oa.o[u] = ol[j0 + u];
                    ob.o[u] = ol[j1 + u];
                }
                half_t bv[2 * kChunk];   // converted at use: two values per register while in flight
                CZ dj[2 * kChunk];
                if (full) {
#pragma unroll
                    for (int u = 0; u < kChunk; ++u) {
                        bv[u] = at32t<NTL>(bsl, (uint32_t)(lane + (j0 + u) * SLICE));
                        bv[kChunk + u] = at32t<NTL>(bsl, (uint32_t)(lane + (j0 + kChunk + u) * SLICE));
                        dj[u] = at32(gb, rowg + (uint32_t)oa.o[u]);
                        dj[kChunk + u] = at32(gb, rowg + (uint32_t)ob.o[u]);
                    }
#pragma unroll
                    for (int u = 0; u < 2 * kChunk; ++u) acc = acc + (CZ)bv[u] * dfrom(dj[u]);
                } else {
#pragma unroll
                    for (int u = 0; u < kChunk; ++u) {
                        const int ja = j0 + u < wd ? j0 + u : wd - 1, jb = j1 + u < wd ? j1 + u : wd - 1;
                        bv[u] = at32t<NTL>(bsl, (uint32_t)(lane + ja * SLICE));
                        bv[kChunk + u] = at32t<NTL>(bsl, (uint32_t)(lane + jb * SLICE));
                        dj[u] = at32(gb, rowg + (uint32_t)oa.o[u]);
                        dj[kChunk + u] = at32(gb, rowg + (uint32_t)ob.o[u]);
                    }
#pragma unroll
                    for (int u = 0; u < 2 * kChunk; ++u) {
                        const CZ t = acc + (CZ)bv[u] * dfrom(dj[u]);
                        acc = (j0 + u < wd) ? t : acc;
                    }
                }
            }
        } else {
            // index mode (general sparsity, not the stencil workloads): one
            // chunk of slots per pass keeps the register budget of the
            // offset-mode loop
            const IdxCols sc{P.col + rec_.ptr + lane, row};
            for (int j0 = 0; j0 < wd; j0 += kChunk) {
                int32_t cc[kChunk];
                bool dg[kChunk];
                half_t bv[kChunk];
                CZ dj[kChunk];
                sc.chunk(j0, wd, cc, dg);
#pragma unroll
                for (int u = 0; u < kChunk; ++u) {
                    const int j = j0 + u < wd ? j0 + u : wd - 1;
                    bv[u] = P.b16[base + (int64_t)j * SLICE];
                    dj[u] = at32(g, (uint32_t)cc[u]);
                }
#pragma unroll
                for (int u = 0; u < kChunk; ++u) {
                    const CZ t = acc + (CZ)bv[u] * dfrom(dj[u]);
                    acc = (j0 + u < wd) ? t : acc;
                }
            }
        }
        const CZ r1 = vi - acc;
        const CZ xn = (xk + c1 * (xk - xkm1)) + c2 * r1;   // x_{k+1}
        if (!last) {
            st32(xw, ru, xn);
        } else {
            const TZ zz = (TZ)(isq_r * xn);
            st32(z, ru, zz);
            rho += rr * (double)zz;
            mz = fmax(mz, fabs((double)zz));
        }
    }
}

// One launch of step k.  STEP: 0 the first step (k = 0), 1 an inner step,
// 2 the last step (forms z and the partials of rho), 3 both first and last
// (degree 2).  UZF: the u_z of every iteration when the solve's options fix
// it (u0 = FP16; or no u_z threshold can be crossed), so that only that
// precision's path is compiled and the kernel needs fewer registers; 0
// reads u_z from the state.  A state whose u_z differs from UZF can only
// come from a non-finite residual (the selector's comparisons fail): it
// ends the solve as a breakdown.
// c1, c2: the recurrence coefficients of step k.
// (every FP32 work-vector variant is compiled for 8 waves per SIMD, at
// most 64 VGPRs; the last step, which also carries the rho reduction and
// both r precisions, then spills a few registers and is still faster than
// at 6 waves without spills; the FP64 work-vector variants for 4)
template <int UZF, int STEP, bool NTL>
__global__ void __launch_bounds__(NTC, (UZF == 16 || UZF == 32) ? AMP_CHEB_WAVES : 4)
    k_cheb_step(Bufs B, Cheb P, double c1, double c2, int din, const St *in, St *out) {
    constexpr bool FIRST = STEP == 0 || STEP == 3, LAST = STEP >= 2;
    __shared__ St s;
    const Wg wg = grid_wg();
    load_state(s, in);
    if (s.status != RUNNING) {
        store_state(s, out, wg);
        return;
    }
    if (UZF != 0 && s.uz != UZF) {
        __syncthreads();
        if (threadIdx.x == 0) s.status = BREAKDOWN;
        store_state(s, out, wg);
        return;
    }
    if (P.step_iter && wg.lb == 0 && threadIdx.x == 0) P.step_iter[P.step_launch] = s.k;
    double rho = 0.0, mz = 0.0;
#define AMP_CS(UZ)                                                                                  \
    do {                                                                                            \
        if (!LAST) cheb_step_body<UZ, FIRST, 0, NTC, NTL>(s, B, P, wg, c1, c2, din, rho, mz);            \
        else if (s.ur == 64) cheb_step_body<UZ, FIRST, 64, NTC, NTL>(s, B, P, wg, c1, c2, din, rho, mz); \
        else cheb_step_body<UZ, FIRST, 32, NTC, NTL>(s, B, P, wg, c1, c2, din, rho, mz);                 \
    } while (0)
    if constexpr (UZF == 64) AMP_CS(64);
    else if constexpr (UZF == 32) AMP_CS(32);
    else if constexpr (UZF == 16) AMP_CS(16);
    else {
        if (s.uz == 64) AMP_CS(64);
        else if (s.uz == 32) AMP_CS(32);
        else AMP_CS(16);
    }
#undef AMP_CS
    if (LAST) {
        double v2[2] = {rho, mz};
        block_reduce<1, 1, NTC>(v2);
        rho = v2[0];
        mz = v2[1];
        if (threadIdx.x == 0) {
            B.part_pre[wg.lb] = rho;
            B.part_pre[GMAX + wg.lb] = mz;
        }
    }
    store_state(s, out, wg);
}

typedef void (*ChebStepFn)(Bufs, Cheb, double, double, int, const St *, St *);

// The step kernel for (UZF, STEP, non-temporal loads).
inline ChebStepFn cheb_step_fn(int uzf, int step, bool nt) {
#define AMP_F(U, N)                                     \
    switch (step) {                                     \
        case 0: return k_cheb_step<U, 0, N>;            \
        case 1: return k_cheb_step<U, 1, N>;            \
        case 2: return k_cheb_step<U, 2, N>;            \
        default: return k_cheb_step<U, 3, N>;           \
    }
#define AMP_FN(U)              \
    if (nt) { AMP_F(U, true) } \
    else { AMP_F(U, false) }
    switch (uzf) {
        case 16: AMP_FN(16)
        case 32: AMP_FN(32)
        case 64: AMP_FN(64)
        default: AMP_FN(0)
    }
#undef AMP_FN
#undef AMP_F
}

// Degree 1: z = fl_uz(isq (.) (v / theta)), no product with B.
template <int UZ>
__device__ __forceinline__ void cheb_deg1_body(const St &s, const Bufs &B, const Cheb &P, Wg wg, double &rho,
                                               double &mz) {
    typedef typename Prec<UZ>::T TZ;
    typedef typename Prec<UZ>::C CZ;
    const CZ *v = (const CZ *)P.v[UZ == 64 ? 0 : 1];
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
