// Matrix-free order-N hexahedral screened Poisson operator (Section 5.5,
// Ex. jac libp): q = A p with A = sum over elements of D^T G D + lambda M on
// the GLL points of each element, the geometric factors of each element's
// trilinear map formed at every quadrature point from its 8 vertices (24
// values per element) instead of being stored, and mu = p^T q.
//
// Mesh: a box of Ex x Ey x Ez elements; global nodes on the
// (N Ex + 1) x (N Ey + 1) x (N Ez + 1) grid (x fastest), local node (i, j, k)
// of element (ex, ey, ez) is grid node (ex N + i, ey N + j, ez N + k); the
// unknowns are the grid nodes off the boundary (homogeneous Dirichlet), in
// grid order.  No index arrays: every map is arithmetic.
//
// One wave per element, lane (i, j) owning the grid line (i, j, 0..N)
// (hex_wave_apply).  The element's p values are gathered to LDS; the
// reference gradient, G (from the Jacobian of the trilinear map at each
// point, formed in registers) and the transposed derivative follow the
// line.  Results are summed into q (zeroed
// first) by atomic adds: shared face, edge and corner nodes receive 2 to 8
// contributions in an order that is not fixed, so q is exact to rounding but
// not bitwise reproducible there.  mu comes from per-element partials p_e^T (A_e
// p_e) summed in element order (deterministic).
//
// Precision: UP is the storage of p (64, 32 or 16), UR the arithmetic and
// storage of q (64 or 32); the geometric factors and contractions run in UR.
// Contractions are written as fused multiply-adds (this operator is bound by
// arithmetic, not by the one-rounding-per-operation rules of the solver's
// vector kernels).
#pragma once

#include "amp_device.hpp"

namespace amp {

constexpr int kHexMaxOrder = 7;

// Device view of an operator handle.
struct HexView {
    int ex, ey, ez;            // elements per direction
    int64_t n;                 // unknowns: (N ex - 1)(N ey - 1)(N ez - 1)
    const double *verts;       // ((ex+1)(ey+1)(ez+1), 3), x fastest
    const double *tab;         // GLL nodes [N+1], weights [N+1], D [(N+1)^2] (D[m][j] = l_j'(x_m))
    double lam;
};

template <typename T>
__device__ __forceinline__ T hex_fma(T a, T b, T c) {
    return __builtin_fma(a, b, c);
}
template <>
__device__ __forceinline__ float hex_fma<float>(float a, float b, float c) {
    return __builtin_fmaf(a, b, c);
}

// The unknown index of grid node (gx, gy, gz), or -1 on the boundary.
template <int N>
__device__ __forceinline__ int64_t hex_dof(const HexView &h, int gx, int gy, int gz) {
    const int mx = N * h.ex, my = N * h.ey, mz = N * h.ez;
    if (gx <= 0 || gy <= 0 || gz <= 0 || gx >= mx || gy >= my || gz >= mz) return -1;
    return (int64_t)(gx - 1) + (int64_t)(mx - 1) * ((int64_t)(gy - 1) + (int64_t)(my - 1) * (gz - 1));
}

// Geometric factors at reference point (r, s, t) of the element whose
// corner (a, b, c) is X[c][b][a][d]: G = w det(J) J^-1 J^-T (six entries,
// rr rs rt ss st tt) and w det(J).  J^-1 = adj(J) / det(J), so
// G = (w / det(J)) adj(J) adj(J)^T.
template <typename T>
__device__ __forceinline__ void hex_geometry(const double (&X)[2][2][2][3], T r, T s, T t, T w, T (&G)[6],
                                             T &wdet) {
    const T hr[2] = {(T)0.5 * ((T)1 - r), (T)0.5 * ((T)1 + r)};
    const T hs[2] = {(T)0.5 * ((T)1 - s), (T)0.5 * ((T)1 + s)};
    const T ht[2] = {(T)0.5 * ((T)1 - t), (T)0.5 * ((T)1 + t)};
    T J[3][3];   // J[d][q] = dx_d / d(r, s, t)_q
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        T jr = 0, js = 0, jt = 0;
#pragma unroll
        for (int c = 0; c < 2; ++c)
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                // x_d(r) along the r-line at (s, t) corner pair (b, c), etc.
                jr = hex_fma((T)0.5 * ((T)X[c][b][1][d] - (T)X[c][b][0][d]), hs[b] * ht[c], jr);
                js = hex_fma((T)0.5 * ((T)X[c][1][b][d] - (T)X[c][0][b][d]), hr[b] * ht[c], js);
                jt = hex_fma((T)0.5 * ((T)X[1][c][b][d] - (T)X[0][c][b][d]), hr[b] * hs[c], jt);
            }
        J[d][0] = jr;
        J[d][1] = js;
        J[d][2] = jt;
    }
    // cofactors C[d][q] (adj(J) = C^T)
    T C[3][3];
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
    wdet = w * det;
    const T f = w / det;
    // (J^-1)[q][d] = C[d][q] / det:  G[p][q] = (w / det) sum_d C[d][p] C[d][q]
    G[0] = f * (C[0][0] * C[0][0] + C[1][0] * C[1][0] + C[2][0] * C[2][0]);
    G[1] = f * (C[0][0] * C[0][1] + C[1][0] * C[1][1] + C[2][0] * C[2][1]);
    G[2] = f * (C[0][0] * C[0][2] + C[1][0] * C[1][2] + C[2][0] * C[2][2]);
    G[3] = f * (C[0][1] * C[0][1] + C[1][1] * C[1][1] + C[2][1] * C[2][1]);
    G[4] = f * (C[0][1] * C[0][2] + C[1][1] * C[1][2] + C[2][1] * C[2][2]);
    G[5] = f * (C[0][2] * C[0][2] + C[1][2] * C[1][2] + C[2][2] * C[2][2]);
}

// The element's corner coordinates (wave-uniform loads).
__device__ __forceinline__ void hex_corners(const HexView &h, int ex, int ey, int ez, double (&X)[2][2][2][3]) {
    const int vx = h.ex + 1, vy = h.ey + 1;
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int a = 0; a < 2; ++a) {
                const int64_t v = (int64_t)(ex + a) + (int64_t)vx * ((ey + b) + (int64_t)vy * (ez + c));
#pragma unroll
                for (int d = 0; d < 3; ++d) X[c][b][a][d] = h.verts[3 * v + d];
            }
}

// The element of this work-group (blocks dealt so that consecutive
// elements, which share nodes, run on the same XCD).
__device__ __forceinline__ void hex_element(const HexView &h, int &ex, int &ey, int &ez) {
    const int e = xcd_block();
    ex = e % h.ex;
    ey = (e / h.ex) % h.ey;
    ez = e / (h.ex * h.ey);
}

// LDS of one element application (one wave): p on the element's nodes and
// the r- and s-fluxes.
template <int N, typename T>
struct HexLds {
    static constexpr int NN = (N + 1) * (N + 1) * (N + 1);
    T u[NN], fr[NN], fs[NN];
    T D[(N + 1) * (N + 1)];   // D[m][j] = l_j'(x_m)
};

// A_e u_e for element (ex, ey, ez) by the calling wave: lane l < (N+1)^2
// owns the grid line (i, j) = (l mod (N+1), l div (N+1)) of nodes
// (i, j, 0..N); its values, t-derivatives and t-fluxes stay in registers,
// so only the r- and s-contractions read LDS.  The Jacobian's
// k-independent parts are formed once per line: dx/dr and dx/ds are linear
// in t, dx/dt does not depend on t.
//   fetch(k, dof) -> T   the line's value at node k (called for dof >= 0;
//                        boundary nodes hold 0)
//   emit(k, dof, a, u)   the line's result a = (A_e u_e) at node k and its
//                        value u (called for dof >= 0)
// Every thread of the work-group calls this the same number of times
// (active = false where a wave has no element this time; (ex, ey, ez) must
// still name a valid element): it contains two work-group barriers.
// DREG: D's rows and columns for the lane's own i and j in registers (64
// of the FP64 kernel's VGPRs; faster where the kernel is not limited by
// registers), else read from the work-group's LDS copy.
template <int N, typename T, bool DREG, typename Fetch, typename Emit>
__device__ __forceinline__ void hex_wave_apply(const HexView &h, bool active, int ex, int ey, int ez,
                                               HexLds<N, T> &L, Fetch fetch, Emit emit) {
    constexpr int N1 = N + 1, NP = N1 * N1;
    static_assert(NP <= WAVE, "one wave per element");
    const int lane = threadIdx.x % WAVE;
    const bool line = active && lane < NP;
    const int i = lane % N1, j = (lane / N1) % N1;
    const double *xg = h.tab, *wg = h.tab + N1, *Dg = h.tab + 2 * N1;
    T u[N1];
    int32_t dof[N1];   // unknowns number below 2^31
#pragma unroll
    for (int k = 0; k < N1; ++k) {
        dof[k] = line ? (int32_t)hex_dof<N>(h, ex * N + i, ey * N + j, ez * N + k) : -1;
        u[k] = (dof[k] >= 0) ? fetch(k, (int64_t)dof[k]) : (T)0;
        if (line) L.u[k * NP + lane] = u[k];
    }
    // D for the loop's k is wave-uniform; for the lane's i and j see DREG
    T Di[N1], Dj[N1], DTi[N1], DTj[N1];
    if constexpr (DREG) {
#pragma unroll
        for (int m = 0; m < N1; ++m) {
            Di[m] = (T)Dg[i * N1 + m];
            Dj[m] = (T)Dg[j * N1 + m];
            DTi[m] = (T)Dg[m * N1 + i];
            DTj[m] = (T)Dg[m * N1 + j];
        }
    } else {
        for (int e = lane; e < N1 * N1; e += WAVE) L.D[e] = (T)Dg[e];
    }
    auto d_row = [&](const T *reg, int a, int m) -> T {   // D[a][m]
        if constexpr (DREG) return reg[m];
        else return L.D[a * N1 + m];
    };
    auto d_col = [&](const T *reg, int a, int m) -> T {   // D[m][a]
        if constexpr (DREG) return reg[m];
        else return L.D[m * N1 + a];
    };
    // Jacobian pieces of the line (i, j): dx_d/dr = Pr0[d] ht0 + Pr1[d] ht1,
    // dx_d/ds = Ps0[d] ht0 + Ps1[d] ht1, dx_d/dt = Jt[d]
    double X[2][2][2][3];
    hex_corners(h, ex, ey, ez, X);   // (ex, ey, ez) is a valid element also when !active
    const T r = (T)xg[i], s = (T)xg[j];
    const T hr[2] = {(T)0.5 * ((T)1 - r), (T)0.5 * ((T)1 + r)};
    const T hs[2] = {(T)0.5 * ((T)1 - s), (T)0.5 * ((T)1 + s)};
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
            ur = hex_fma(d_row(Di, i, m), L.u[k * NP + j * N1 + m], ur);
            us = hex_fma(d_row(Dj, j, m), L.u[k * NP + m * N1 + i], us);
            ut = hex_fma((T)Dg[k * N1 + m], u[m], ut);
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
        T C[3][3];
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
        // grad_x u = J^-T (ur, us, ut) = C (ur, us, ut) / det; the fluxes are
        // G (ur, us, ut) = (w / det) C^T C (ur, us, ut)
        const T g0 = hex_fma(C[0][0], ur, hex_fma(C[0][1], us, C[0][2] * ut));
        const T g1 = hex_fma(C[1][0], ur, hex_fma(C[1][1], us, C[1][2] * ut));
        const T g2 = hex_fma(C[2][0], ur, hex_fma(C[2][1], us, C[2][2] * ut));
        if (line) {
            L.fr[k * NP + lane] = f * hex_fma(C[0][0], g0, hex_fma(C[1][0], g1, C[2][0] * g2));
            L.fs[k * NP + lane] = f * hex_fma(C[0][1], g0, hex_fma(C[1][1], g1, C[2][1] * g2));
        }
        ft[k] = f * hex_fma(C[0][2], g0, hex_fma(C[1][2], g1, C[2][2] * g2));
        au[k] = w * det * (T)h.lam * u[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < N1; ++k) {
        T a = au[k];
#pragma unroll
        for (int m = 0; m < N1; ++m) {
            a = hex_fma(d_col(DTi, i, m), L.fr[k * NP + j * N1 + m], a);
            a = hex_fma(d_col(DTj, j, m), L.fs[k * NP + m * N1 + i], a);
            a = hex_fma((T)Dg[m * N1 + k], ft[m], a);
        }
        if (dof[k] >= 0) emit(k, (int64_t)dof[k], a, u[k]);
    }
}

// Whether local node (i, j, k) of element (ex, ey, ez) is the one copy of
// its grid node that writes per-node results: the element with the lowest
// index along each direction that contains it.
template <int N>
__device__ __forceinline__ bool hex_owner(const HexView &h, int ex, int ey, int ez, int i, int j, int k) {
    return (i < N || ex == h.ex - 1) && (j < N || ey == h.ey - 1) && (k < N || ez == h.ez - 1);
}

// q += A_e p_e for this work-group's element; part[e] = p_e^T (A_e p_e).
// One wave per work-group and element.  Shared nodes are summed into q by
// atomic adds in no fixed order (a plain store for the nodes inside the
// element, whose only contributor it is, measured 2.3x slower: the divergent
// branch around the atomic).
template <int N, int UP, int UR>
__global__ void __launch_bounds__((N + 1) * (N + 1))
    k_hex_ax(HexView h, const void *pv, void *qv, double *part) {
    typedef typename Prec<UP>::T TP;
    typedef typename Prec<UR>::T T;
    constexpr int NP = (N + 1) * (N + 1);
    __shared__ HexLds<N, T> L;
    __shared__ double s_mu[NP];
    const TP *p = (const TP *)pv;
    T *q = (T *)qv;
    int ex, ey, ez;
    hex_element(h, ex, ey, ez);
    double mu = 0.0;
    hex_wave_apply<N, T, false>(h, true, ex, ey, ez, L, [&](int, int64_t dof) { return (T)p[dof]; },
                         [&](int, int64_t dof, T a, T u) {
                             unsafeAtomicAdd(q + dof, a);
                             mu += (double)u * (double)a;
                         });
    // per-element partial, summed over the lines in lane order
    s_mu[threadIdx.x] = mu;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int l = 0; l < NP; ++l) t += s_mu[l];
        part[(int64_t)ez * h.ex * h.ey + (int64_t)ey * h.ex + ex] = t;
    }
}

// diag += the diagonal of A_e (FP64): for local node (a, b, c) the reference
// gradient of its basis function is nonzero only on the three grid lines
// through it, so A_e's diagonal entry is sum_m D[m][a]^2 G_rr(m, b, c) +
// sum_m D[m][b]^2 G_ss(a, m, c) + sum_m D[m][c]^2 G_tt(a, b, m) + 2 D[a][a]
// D[b][b] G_rs + 2 D[a][a] D[c][c] G_rt + 2 D[b][b] D[c][c] G_st (at the node
// itself) + lambda w det(J).
template <int N>
__global__ void __launch_bounds__((N + 1) * (N + 1) * (N + 1)) k_hex_diag(HexView h, double *diag) {
    constexpr int N1 = N + 1, NN = N1 * N1 * N1;
    __shared__ double s_g[3][NN];
    const int tid = threadIdx.x;
    const int i = tid % N1, j = (tid / N1) % N1, k = tid / (N1 * N1);
    int ex, ey, ez;
    hex_element(h, ex, ey, ez);
    const double *xg = h.tab, *wg = h.tab + N1, *D = h.tab + 2 * N1;
    double X[2][2][2][3];
    hex_corners(h, ex, ey, ez, X);
    double G[6], wdet;
    hex_geometry<double>(X, xg[i], xg[j], xg[k], wg[i] * wg[j] * wg[k], G, wdet);
    s_g[0][tid] = G[0];
    s_g[1][tid] = G[3];
    s_g[2][tid] = G[5];
    __syncthreads();
    double d = h.lam * wdet;
    for (int m = 0; m < N1; ++m) {
        d += D[m * N1 + i] * D[m * N1 + i] * s_g[0][(k * N1 + j) * N1 + m];
        d += D[m * N1 + j] * D[m * N1 + j] * s_g[1][(k * N1 + m) * N1 + i];
        d += D[m * N1 + k] * D[m * N1 + k] * s_g[2][(m * N1 + j) * N1 + i];
    }
    const double di = D[i * N1 + i], dj = D[j * N1 + j], dk = D[k * N1 + k];
    d += 2.0 * di * dj * G[1] + 2.0 * di * dk * G[2] + 2.0 * dj * dk * G[4];
    const int64_t dof = hex_dof<N>(h, ex * N + i, ey * N + j, ez * N + k);
    if (dof >= 0) unsafeAtomicAdd(diag + dof, d);
}

template <typename T>
__global__ void k_hex_zero(T *a, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        a[i] = (T)0;
}

// out[0] = sum of part[0 .. n): thread t sums part[t], part[t + 1024], ...
// (coalesced), then thread 0 adds the 1024 sums in thread order -- a fixed
// order, so the result is reproducible.
constexpr int kHexSumThreads = 1024;
__global__ void __launch_bounds__(kHexSumThreads) k_hex_sum(const double *part, int64_t n, double *out) {
    __shared__ double sh[kHexSumThreads];
    double s = 0.0;
    // eight loads in flight per thread, added in index order
    constexpr int U = 8;
    int64_t e = threadIdx.x;
    for (; e + (U - 1) * kHexSumThreads < n; e += U * kHexSumThreads) {
        double v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = part[e + u * kHexSumThreads];
#pragma unroll
        for (int u = 0; u < U; ++u) s += v[u];
    }
    for (; e < n; e += kHexSumThreads) s += part[e];
    sh[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < kHexSumThreads; ++w) t += sh[w];
        out[0] = t;
    }
}

}  // namespace amp
