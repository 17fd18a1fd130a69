// p-multigrid preconditioner (Section 5.3, Ex. linear conv2) for the
// matrix-free hexahedral operator: a V-cycle over polynomial orders
// N_0 > N_1 > ... on the same mesh, each level the operator rediscretised at
// its order, smoothed by a Chebyshev-accelerated Jacobi polynomial, with a
// higher-degree Chebyshev-Jacobi polynomial as the coarse solve.
//
// V-cycle for f on level l: x = S f; x += P V_{l+1}(P^T (f - A x));
// x += S (f - A x).  S = s(D^-1 A) D^-1 is the Chebyshev iteration for
// D^-1 A x = D^-1 f from x = 0 on [lo, hi]:
//   x_1 = D^-1 f / theta;  x_{k+1} = x_k + c1 (x_k - x_{k-1}) + c2 D^-1 (f - A x_k).
// P interpolates the coarse function at the fine GLL points element by
// element (1-D matrix J[a][b] = l_b(x_a) along each direction); every element
// holding a fine node gives it the same value, so only the node's owner
// element writes it.  P^T: each element sums J^T of its fine values weighted
// by 1 / (number of elements sharing the node) into the coarse nodes by
// atomic adds (exact: P[f][c] is nonzero only when every element holding f
// also holds c).
//
// Every kernel takes the precision of the cycle from the solve's state (FP64
// when u_z is FP64, else FP32; nothing at all once the solve has stopped) or,
// standalone, from an argument.  Work vectors of both precisions exist; only
// the active one is touched.
#pragma once

#include <type_traits>

#include "amp_hex.hpp"
#include "amp_controller.hpp"

namespace amp {

constexpr int kPmgLevels = 4;    // most levels of a cycle
constexpr int kPmgDegMax = 32;   // highest smoother / coarse polynomial degree
constexpr int NTV = 256;         // threads of the vector kernels
constexpr int kPmgPartMax = 1024;

// Precision of a cycle launch: 64 or 32, or 0 when the solve has stopped.
__device__ __forceinline__ int pmg_prec(const St *st, int prec) {
    if (st) {
        if (st->status != RUNNING) return 0;
        return st->uz == 64 ? 64 : 32;
    }
    return prec;
}

// One elementwise pass of the smoother.  Pointers by precision (0: FP64,
// 1: FP32).  first: x_1 = a D^-1 g with g = rhs, or, when gout is set,
// g = rhs - ax stored to gout (the post-smoother's right-hand side);
// otherwise x_{k+1} = x_k + c1 (x_k - x_{k-1}) + c2 D^-1 (rhs - ax) with
// x_{k-1} = 0 when prev is null.  The result is stored to out, or added to
// acc.  ax is cleared after it is read (the next product sums into it).
// vcur / vprev: x_k / x_{k-1} is the pre-smoother's first iterate
// a1 D^-1 rhs, formed here instead of read (it is never stored).
struct PmgVecOp {
    const void *dinv[2];
    const void *rhs[2];
    void *ax[2];
    const void *cur[2];
    const void *prev[2];
    void *out[2];
    void *gout[2];
    void *acc[2];
    int64_t n;
    double a, c1, c2, a1;
    int first, vcur, vprev;
};

template <typename T>
__device__ __forceinline__ void pmg_vec_body(const PmgVecOp &o, int s) {
    const T *dinv = (const T *)o.dinv[s];
    const T *rhs = (const T *)o.rhs[s];
    T *ax = (T *)o.ax[s];
    const T *cur = (const T *)o.cur[s];
    const T *prev = (const T *)o.prev[s];
    T *out = (T *)o.out[s];
    T *gout = (T *)o.gout[s];
    T *acc = (T *)o.acc[s];
    const T a = (T)o.a, c1 = (T)o.c1, c2 = (T)o.c2;
    for (int64_t i = (int64_t)blockIdx.x * NTV + threadIdx.x; i < o.n; i += (int64_t)gridDim.x * NTV) {
        T xn;
        if (o.first) {
            T g = rhs[i];
            if (gout) {
                g = g - ax[i];
                gout[i] = g;
            }
            xn = a * (dinv[i] * g);
        } else {
            const T x1 = (o.vcur || o.vprev) ? (T)o.a1 * (dinv[i] * rhs[i]) : (T)0;
            const T xk = o.vcur ? x1 : cur[i];
            const T xp = o.vprev ? x1 : (prev ? prev[i] : (T)0);
            xn = (xk + c1 * (xk - xp)) + c2 * (dinv[i] * (rhs[i] - ax[i]));
        }
        if (acc) acc[i] = acc[i] + xn;
        else out[i] = xn;
        ax[i] = (T)0;
    }
}

__global__ void __launch_bounds__(NTV) k_pmg_vec(PmgVecOp o, const St *st, int prec) {
    const int p = pmg_prec(st, prec);
    if (p == 64) pmg_vec_body<double>(o, 0);
    else if (p == 32) pmg_vec_body<float>(o, 1);
}

// a = 0 on n entries of the active precision.
__global__ void __launch_bounds__(NTV) k_pmg_clear(void *a64, void *a32, int64_t n, const St *st, int prec) {
    const int p = pmg_prec(st, prec);
    for (int64_t i = (int64_t)blockIdx.x * NTV + threadIdx.x; i < n; i += (int64_t)gridDim.x * NTV) {
        if (p == 64) ((double *)a64)[i] = 0.0;
        else if (p == 32) ((float *)a32)[i] = 0.0f;
    }
}

// out += A u on one level (atomic assembly into out, cleared by the launch
// before), several elements per wave: lanes
// [s NP, (s+1) NP) of a wave take element slot s (NP = (N+1)^2 lanes, one per
// grid line (i, j) of the element, as in the solve's element kernel), four
// waves per work-group, so the orders below 7 keep every lane busy (order 3:
// 4 elements per wave, order 1: 16).  Instantiated per precision P: the
// launch does nothing unless the cycle runs in P (the host launches only
// the matching variant when the solve's u_z is fixed).  D is read from LDS.
// vf non-null: u = va D^-1 vf (vd holds D^-1), the pre-smoother's first
// iterate formed at the gather instead of read.
constexpr int NTA = 256;
// minimum waves per SIMD the product is compiled for (its VGPR budget)
#ifndef PMG_WAVES
#define PMG_WAVES(N, P) ((N) == 7 ? ((P) == 64 ? 2 : 4) : 4)
#endif

template <int N, int P>
__global__ void __launch_bounds__(NTA) __attribute__((amdgpu_waves_per_eu(PMG_WAVES(N, P))))
    k_pmg_ax_packed(HexView h, int64_t E, const void *uv, void *ov, const void *vf, const void *vd, double va,
                    const St *st, int prec) {
    typedef typename std::conditional<P == 64, double, float>::type T;
    constexpr int N1 = N + 1, NP = N1 * N1, NN = NP * N1;
    constexpr int EPW = WAVE / NP, S = (NTA / WAVE) * EPW;   // elements per wave, per work-group
    if (pmg_prec(st, prec) != P) return;   // uniform over the launch
    __shared__ T Lu[S * NN], Lfr[S * NN], Lfs[S * NN];
    __shared__ T LD[NP];
    const T *u = (const T *)uv;
    const T *vfp = (const T *)vf, *vdp = (const T *)vd;
    T *o = (T *)ov;
    const int tid = threadIdx.x, lane = tid % WAVE;
    const int slot = (tid / WAVE) * EPW + lane / NP;
    const int l = lane % NP;
    const bool inwave = lane < EPW * NP;   // every lane when NP divides 64
    const int64_t e = (int64_t)xcd_block() * S + slot;
    const bool active = inwave && e < E;
    const int64_t ev = active ? e : E - 1;   // a valid element for the geometry
    const int ex = (int)(ev % h.ex), ey = (int)((ev / h.ex) % h.ey), ez = (int)(ev / ((int64_t)h.ex * h.ey));
    const int i = l % N1, j = l / N1;
    const double *xg = h.tab, *wg = h.tab + N1, *Dg = h.tab + 2 * N1;
    for (int t = tid; t < NP; t += NTA) LD[t] = (T)Dg[t];
    T* const U = Lu + slot * NN;
    T* const FR = Lfr + slot * NN;
    T* const FS = Lfs + slot * NN;
    T uu[N1];
    int32_t dof[N1];
#pragma unroll
    for (int k = 0; k < N1; ++k) {
        dof[k] = active ? (int32_t)hex_dof<N>(h, ex * N + i, ey * N + j, ez * N + k) : -1;
        uu[k] = (dof[k] < 0) ? (T)0 : vfp ? (T)va * (vdp[dof[k]] * vfp[dof[k]]) : u[dof[k]];
        if (inwave) U[k * NP + l] = uu[k];
    }
    double X[2][2][2][3];
    hex_corners(h, ex, ey, ez, X);
    const T r = (T)xg[i], sv = (T)xg[j];
    const T hr[2] = {(T)0.5 * ((T)1 - r), (T)0.5 * ((T)1 + r)};
    const T hs[2] = {(T)0.5 * ((T)1 - sv), (T)0.5 * ((T)1 + sv)};
    // dx/dr and dx/ds are linear in t along the line, dx/dt constant
    T Pr[2][3], Ps[2][3], Jt[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            Pr[c][d] = hex_fma((T)0.5 * ((T)X[c][0][1][d] - (T)X[c][0][0][d]), hs[0],
                               (T)0.5 * ((T)X[c][1][1][d] - (T)X[c][1][0][d]) * hs[1]);
            Ps[c][d] = hex_fma((T)0.5 * ((T)X[c][1][0][d] - (T)X[c][0][0][d]), hr[0],
                               (T)0.5 * ((T)X[c][1][1][d] - (T)X[c][0][1][d]) * hr[1]);
        }
        T jt = 0;
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int a = 0; a < 2; ++a)
                jt = hex_fma((T)0.5 * ((T)X[1][b][a][d] - (T)X[0][b][a][d]), hr[a] * hs[b], jt);
        Jt[d] = jt;
    }
    const T wij = (T)wg[i] * (T)wg[j];
    __syncthreads();
    T ft[N1], au[N1];
#pragma unroll
    for (int k = 0; k < N1; ++k) {
        T ur = 0, us = 0, ut = 0;
#pragma unroll
        for (int m = 0; m < N1; ++m) {
            ur = hex_fma(LD[i * N1 + m], U[k * NP + j * N1 + m], ur);
            us = hex_fma(LD[j * N1 + m], U[k * NP + m * N1 + i], us);
            ut = hex_fma((T)Dg[k * N1 + m], uu[m], ut);
        }
        const T t = (T)xg[k];
        const T ht0 = (T)0.5 * ((T)1 - t), ht1 = (T)0.5 * ((T)1 + t);
        T J[3][3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            J[d][0] = hex_fma(Pr[0][d], ht0, Pr[1][d] * ht1);
            J[d][1] = hex_fma(Ps[0][d], ht0, Ps[1][d] * ht1);
            J[d][2] = Jt[d];
        }
        T C[3][3];   // cofactors: J^-T = C / det
        C[0][0] = J[1][1] * J[2][2] - J[1][2] * J[2][1];
        C[0][1] = J[1][2] * J[2][0] - J[1][0] * J[2][2];
        C[0][2] = J[1][0] * J[2][1] - J[1][1] * J[2][0];
        C[1][0] = J[0][2] * J[2][1] - J[0][1] * J[2][2];
        C[1][1] = J[0][0] * J[2][2] - J[0][2] * J[2][0];
        C[1][2] = J[0][1] * J[2][0] - J[0][0] * J[2][1];
        C[2][0] = J[0][1] * J[1][2] - J[0][2] * J[1][1];
        C[2][1] = J[0][2] * J[1][0] - J[0][0] * J[1][2];
        C[2][2] = J[0][0] * J[1][1] - J[0][1] * J[1][0];
        const T det = J[0][0] * C[0][0] + J[0][1] * C[0][1] + J[0][2] * C[0][2];
        const T w = wij * (T)wg[k];
        const T f = w / det;
        const T g0 = hex_fma(C[0][0], ur, hex_fma(C[0][1], us, C[0][2] * ut));
        const T g1 = hex_fma(C[1][0], ur, hex_fma(C[1][1], us, C[1][2] * ut));
        const T g2 = hex_fma(C[2][0], ur, hex_fma(C[2][1], us, C[2][2] * ut));
        if (inwave) {
            FR[k * NP + l] = f * hex_fma(C[0][0], g0, hex_fma(C[1][0], g1, C[2][0] * g2));
            FS[k * NP + l] = f * hex_fma(C[0][1], g0, hex_fma(C[1][1], g1, C[2][1] * g2));
        }
        ft[k] = f * hex_fma(C[0][2], g0, hex_fma(C[1][2], g1, C[2][2] * g2));
        au[k] = w * det * (T)h.lam * uu[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < N1; ++k) {
        T a = au[k];
#pragma unroll
        for (int m = 0; m < N1; ++m) {
            a = hex_fma(LD[m * N1 + i], FR[k * NP + j * N1 + m], a);
            a = hex_fma(LD[m * N1 + j], FS[k * NP + m * N1 + i], a);
            a = hex_fma((T)Dg[m * N1 + k], ft[m], a);
        }
        if (dof[k] >= 0) unsafeAtomicAdd(o + dof[k], a);
    }
}

// Transfer kernels: one wave per element, XW elements per work-group;
// instantiated per precision P like the products (a launch whose P is not
// the cycle's returns at once).
constexpr int XW = 4;
constexpr int NTX = XW * WAVE;

// Contraction of one direction of an element's tensor by the element's
// wave: dst[o][c][i] = sum_m J(m, c) src[o][m][i] (TRANS: J(m, c) = J[m][c],
// the restriction; else J(m, c) = J[c][m], the interpolation), for `outer`
// x `cm` x `inner` outputs, src `outer` x `sm` x `inner`.
template <typename T, bool TRANS>
__device__ __forceinline__ void pmg_contract(const double *J, int jc, const T *src, T *dst, int outer, int sm,
                                             int cm, int inner, int lane) {
    const int total = outer * cm * inner;
    for (int t = lane; t < total; t += WAVE) {
        const int i = t % inner, c = (t / inner) % cm, o = t / (inner * cm);
        T acc = 0;
        for (int m = 0; m < sm; ++m) {
            const T w = TRANS ? (T)J[m * jc + c] : (T)J[c * jc + m];
            acc = acc + w * src[(o * sm + m) * inner + i];
        }
        dst[(o * cm + c) * inner + i] = acc;
    }
}

// The element of this wave (e = work-group * XW + wave; valid when e < E).
__device__ __forceinline__ bool pmg_xfer_element(const HexView &h, int64_t E, int &ex, int &ey, int &ez) {
    const int64_t e = (int64_t)xcd_block() * XW + threadIdx.x / WAVE;
    const int64_t ev = e < E ? e : E - 1;
    ex = (int)(ev % h.ex);
    ey = (int)((ev / h.ex) % h.ey);
    ez = (int)(ev / ((int64_t)h.ex * h.ey));
    return e < E;
}

// fc += P^T (f - ax) for the waves' elements.  J: (NF+1) x (NC+1) row-major,
// J[a][b] = l_b(x_a).
template <int NF, int NC, int P>
__global__ void __launch_bounds__(NTX) k_pmg_restrict(HexView hf, HexView hc, const double *J, int64_t E,
                                                      const void *fv, const void *axv, void *fcv, const St *st,
                                                      int prec) {
    typedef typename std::conditional<P == 64, double, float>::type T;
    constexpr int F1 = NF + 1, C1 = NC + 1, FN = F1 * F1 * F1;
    if (pmg_prec(st, prec) != P) return;   // uniform over the launch
    __shared__ T Us[XW * FN], T1s[XW * F1 * F1 * C1], T2s[XW * F1 * C1 * C1];
    const int w = threadIdx.x / WAVE, lane = threadIdx.x % WAVE;
    T *U = Us + w * FN, *T1 = T1s + w * F1 * F1 * C1, *T2 = T2s + w * F1 * C1 * C1;
    const T *f = (const T *)fv, *ax = (const T *)axv;
    T *fc = (T *)fcv;
    int ex, ey, ez;
    const bool valid = pmg_xfer_element(hf, E, ex, ey, ez);
    for (int t = lane; t < FN; t += WAVE) {
        const int i = t % F1, j = (t / F1) % F1, k = t / (F1 * F1);
        const int64_t dof = valid ? hex_dof<NF>(hf, ex * NF + i, ey * NF + j, ez * NF + k) : -1;
        T v = 0;
        if (dof >= 0) {
            // a node on an element face, edge or corner off the boundary is
            // shared by 2, 4 or 8 elements
            const int mult = ((i == 0 || i == NF) ? 2 : 1) * ((j == 0 || j == NF) ? 2 : 1) * ((k == 0 || k == NF) ? 2 : 1);
            v = (f[dof] - ax[dof]) / (T)mult;
        }
        U[t] = v;
    }
    __syncthreads();
    pmg_contract<T, true>(J, C1, U, T1, F1 * F1, F1, C1, 1, lane);      // i -> c
    __syncthreads();
    pmg_contract<T, true>(J, C1, T1, T2, F1, F1, C1, C1, lane);         // j -> b
    __syncthreads();
    for (int t = lane; t < C1 * C1 * C1; t += WAVE) {                   // k -> a
        const int c = t % C1, b = (t / C1) % C1, a = t / (C1 * C1);
        T acc = 0;
        for (int k = 0; k < F1; ++k) acc = acc + (T)J[k * C1 + a] * T2[(k * C1 + b) * C1 + c];
        const int64_t cd = valid ? hex_dof<NC>(hc, ex * NC + c, ey * NC + b, ez * NC + a) : -1;
        if (cd >= 0) unsafeAtomicAdd(fc + cd, acc);
    }
}

// x += P xc at the fine nodes each wave's element owns; ax = 0 there (the
// product that follows sums into it).
template <int NF, int NC, int P>
__global__ void __launch_bounds__(NTX) k_pmg_prolong(HexView hf, HexView hc, const double *J, int64_t E,
                                                     const void *xcv, void *xv, void *axv, const St *st, int prec) {
    typedef typename std::conditional<P == 64, double, float>::type T;
    constexpr int F1 = NF + 1, C1 = NC + 1, CN = C1 * C1 * C1;
    if (pmg_prec(st, prec) != P) return;   // uniform over the launch
    __shared__ T Ucs[XW * CN], V1s[XW * C1 * C1 * F1], V2s[XW * C1 * F1 * F1];
    const int w = threadIdx.x / WAVE, lane = threadIdx.x % WAVE;
    T *Uc = Ucs + w * CN, *V1 = V1s + w * C1 * C1 * F1, *V2 = V2s + w * C1 * F1 * F1;
    const T *xc = (const T *)xcv;
    T *x = (T *)xv, *ax = (T *)axv;
    int ex, ey, ez;
    const bool valid = pmg_xfer_element(hf, E, ex, ey, ez);
    for (int t = lane; t < CN; t += WAVE) {
        const int c = t % C1, b = (t / C1) % C1, a = t / (C1 * C1);
        const int64_t cd = valid ? hex_dof<NC>(hc, ex * NC + c, ey * NC + b, ez * NC + a) : -1;
        Uc[t] = (cd >= 0) ? xc[cd] : (T)0;
    }
    __syncthreads();
    pmg_contract<T, false>(J, C1, Uc, V1, C1 * C1, C1, F1, 1, lane);   // c -> i
    __syncthreads();
    pmg_contract<T, false>(J, C1, V1, V2, C1, C1, F1, F1, lane);       // b -> j
    __syncthreads();
    if (!valid) return;   // after the last barrier
    for (int t = lane; t < F1 * F1 * F1; t += WAVE) {                  // a -> k
        const int i = t % F1, j = (t / F1) % F1, k = t / (F1 * F1);
        if (!hex_owner<NF>(hf, ex, ey, ez, i, j, k)) continue;
        const int64_t dof = hex_dof<NF>(hf, ex * NF + i, ey * NF + j, ez * NF + k);
        if (dof < 0) continue;
        T acc = 0;
        for (int a = 0; a < C1; ++a) acc = acc + (T)J[k * C1 + a] * V2[(a * F1 + j) * F1 + i];
        x[dof] = x[dof] + acc;
        ax[dof] = (T)0;
    }
}

// Standalone entry and exit: f = fl_prec(r); z = x (FP64).
__global__ void __launch_bounds__(NTV) k_pmg_in(const double *r, void *f64, void *f32, int64_t n, int prec) {
    for (int64_t i = (int64_t)blockIdx.x * NTV + threadIdx.x; i < n; i += (int64_t)gridDim.x * NTV) {
        if (prec == 64) ((double *)f64)[i] = r[i];
        else ((float *)f32)[i] = (float)r[i];
    }
}
__global__ void __launch_bounds__(NTV) k_pmg_out(const void *x64, const void *x32, double *z, int64_t n, int prec) {
    for (int64_t i = (int64_t)blockIdx.x * NTV + threadIdx.x; i < n; i += (int64_t)gridDim.x * NTV)
        z[i] = (prec == 64) ? ((const double *)x64)[i] : (double)((const float *)x32)[i];
}

// dinv = 1 / diag (both precisions); err |= 1 where diag <= 0 or is not finite.
__global__ void __launch_bounds__(NTV) k_pmg_dinv(const double *diag, double *d64, float *d32, int64_t n, int *err) {
    for (int64_t i = (int64_t)blockIdx.x * NTV + threadIdx.x; i < n; i += (int64_t)gridDim.x * NTV) {
        const double d = diag[i];
        if (!(d > 0.0) || !isfinite(d)) atomicOr(err, 1);
        const double v = 1.0 / d;
        d64[i] = v;
        d32[i] = (float)v;
    }
}

// Power iteration for rho = lambda_max(D^-1 A) (FP64).  Start vector: a
// counter-based hash of the index mapped to [0.5, 1.5).
__global__ void __launch_bounds__(NTV) k_pmg_start(double *v, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * NTV + threadIdx.x; i < n; i += (int64_t)gridDim.x * NTV) {
        uint64_t z = (uint64_t)i + 0x9E3779B97F4A7C15ull;   // splitmix64 finaliser
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        z ^= z >> 31;
        v[i] = 0.5 + (double)(z >> 11) * 0x1.0p-53;
    }
}

// With ax = A v: part[2 b] = sum v ax, part[2 b + 1] = sum v^2 / dinv over
// this work-group's entries (v^T A v and v^T D v: their ratio is the
// Rayleigh quotient of D^-1 A in the D inner product); v = scale D^-1 ax;
// ax = 0.
__global__ void __launch_bounds__(NTV) k_pmg_power(double *v, double *ax, const double *dinv, int64_t n,
                                                   double scale, double *part) {
    __shared__ double sh[2][NTV];
    double num = 0.0, den = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * NTV + threadIdx.x; i < n; i += (int64_t)gridDim.x * NTV) {
        const double vi = v[i], ai = ax[i];
        num += vi * ai;
        den += vi * vi / dinv[i];
        v[i] = scale * (dinv[i] * ai);
        ax[i] = 0.0;
    }
    sh[0][threadIdx.x] = num;
    sh[1][threadIdx.x] = den;
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = 0.0, b = 0.0;
        for (int t = 0; t < NTV; ++t) {
            a += sh[0][t];
            b += sh[1][t];
        }
        part[2 * blockIdx.x] = a;
        part[2 * blockIdx.x + 1] = b;
    }
}

// part[b] = max |x| over this work-group's entries (FP64).
__global__ void __launch_bounds__(NTV) k_pmg_maxabs(const double *x, int64_t n, double *part) {
    __shared__ double sh[NTV];
    double m = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * NTV + threadIdx.x; i < n; i += (int64_t)gridDim.x * NTV)
        m = fmax(m, fabs(x[i]));
    sh[threadIdx.x] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int k = 0; k < NTV; ++k) t = fmax(t, sh[k]);
        part[blockIdx.x] = t;
    }
}

}  // namespace amp
