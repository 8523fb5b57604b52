// Discrete adjoint of the LBM time step for gfx950.
//
// Forward model (two-lattice state g^n, f^n = S g^n):
//   f^{n+1} = S C(f^n; tau, F),  u^n = sum_a e_a f^n_a + F/2  (rho0 = 1),
// with C the node collision and S the propagation with bounce-back, a
// permutation.  Given lambda^{n+1} = dJ/df^{n+1}, one adjoint step is
//   lambda*_a(x) = lambda^{n+1}_a(x + e_a)   (lambda^{n+1}_abar(x) at a wall:
//                                           S^T = S^-1, a pull from x + e_a)
//   lambda^n     = (dC/df)^T lambda*,  taubar += (dC/dtau)^T lambda*,
//                                      Fbar   += (dC/dF)^T lambda*.
// The transposed collision Jacobian has a closed form through four weighted
// moments of lambda* at the node (w_a weights, u the node velocity):
//   m0 = sum w l,  m1 = sum w l e,  m2 = sum w l (e.u) e,  m3 = sum w l (e.F) e,
//   A  = 3 m1 + 9 m2 - 3 m0 u,       B  = 9 m3 - 3 m0 F,
//   lambda^n_b = (1 - omega) l_b + omega m0 + (omega A + (1 - omega/2) B) . e_b,
//   taubar    += -omega^2 sum_a l_a (feq_a - f_a - G_a/2),
//   Fbar      += A + (1 - omega/2) B / 2,
// from feq_a = w_a (rho + 3 e.u + 4.5 (e.u)^2 - 1.5 u.u) (derivative
// w_a (3 e + 9 (e.u) e - 3 u) in u), G_a = w_a (3 (e - u).F + 9 (e.u)(e.F))
// and du/df_b = e_b, du/dF = I/2, domega/dtau = -omega^2.  The same
// expressions hold for the deviation storages (the update is affine in f).
//
// Compressible model (feq_a = rho phi_a(u), u = (sum e f + F/2)/rho, so
// du/df_b = (e_b - u)/rho and du/dF = I/(2 rho)): with
//   P = sum l_a phi_a = m0 (1 - 1.5 u.u) + 3 m1.u + 4.5 m2.u,
//   lambda^n_b = (1 - omega) l_b + omega P + (omega A + (1 - omega/2) B/rho) . (e_b - u),
//   Fbar      += A + (1 - omega/2) B / (2 rho),
// and taubar as above with this feq.
//
// Walls of the nodal scheme make the forward state B(S C(f)) with B the
// copy of Eq. (bb) on wall nodes; its transpose (k_adjoint_nodal_bt) folds
// the adjoint of each unknown population into the opposite one before every
// adjoint step and before the init map.
//
// lambda fields use the tiled layout of the stored state (slot()) in the
// arithmetic type of the storage, with the same streaming hints as the
// forward step.  taubar and Fbar accumulate per workgroup in FP64 into a
// fixed slot per workgroup, summed at the end in a fixed order.
#pragma once

#include "kernels.hpp"

namespace imexlbm {

template <class C>
struct AdjArgs {
    Dims g;
    int bx_shift;
    C omega;
    C F[3];
    C half;  // 1 - omega/2
};

constexpr int kAccSlots = 4;  // taubar, Fbar_x, Fbar_y, Fbar_z

// Sums v[0..3] over the workgroup (fixed tree) and adds the result to the
// workgroup's slots of acc.  Every work-item of the group must call it.
__device__ __forceinline__ void block_accumulate(double (&v)[kAccSlots], double* __restrict__ acc)
{
    __shared__ double s[kAccSlots][256];
    const int t = threadIdx.x;
    for (int c = 0; c < kAccSlots; ++c) s[c][t] = v[c];
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (t < h)
            for (int c = 0; c < kAccSlots; ++c) s[c][t] += s[c][t + h];
        __syncthreads();
    }
    if (t == 0) {
        const size_t b = blockIdx.x + size_t(gridDim.x) * (blockIdx.y + size_t(gridDim.y) * blockIdx.z);
        for (int c = 0; c < kAccSlots; ++c) acc[b * kAccSlots + c] += s[c][0];
    }
}

// One adjoint step: reads the forward state g^n (two-lattice layout) and
// lambda^{n+1}, writes lambda^n, accumulates taubar and Fbar.
template <int L, class S, bool WALLS, bool FORCE, bool COMP>
__global__ LBM_STEP_BOUNDS void k_adjoint_step(const S* __restrict__ g,
                                                      const typename Store<S>::C* __restrict__ lam_in,
                                                      typename Store<S>::C* __restrict__ lam_out,
                                                      double* __restrict__ acc,
                                                      AdjArgs<typename Store<S>::C> p)
{
    using C = typename Store<S>::C;
    constexpr int Q = Lattice<L>::Q;
    int x, y, z;
    const bool inside = node_of_item(p.g, p.bx_shift, x, y, z);
    const bool active = inside && !(WALLS && is_solid(p.g, x, y, z));
    double part[kAccSlots] = {0.0, 0.0, 0.0, 0.0};
    if (inside) {
        const int TS = p.g.S;
        const unsigned own = unsigned(x) + unsigned(p.g.nx) * (unsigned(y) + unsigned(p.g.ny) * unsigned(z));
        if (!active) {
            for (int a = 0; a < Q; ++a) lam_out[slot<Q>(a, own, TS)] = C(0);
        } else {
            unsigned idx[Q];
            bool wall[Q];
            // lambda*: pull from x + e_a.
            link_nodes<L, WALLS, +1>(p.g, x, y, z, idx, wall);
            C ls[Q];
            static_for<Q>([&](auto ac) {
                constexpr int a = decltype(ac)::value;
                constexpr int abar = Lattice<L>::opp(a);
                constexpr bool aligned = kLattice<L>.e[a][0] == 0;
                ls[a] = get<aligned>(lam_in + ((WALLS && wall[a]) ? slot<Q>(abar, own, TS) : slot<Q>(a, idx[a], TS)));
            });
            // f^n: pull from x - e_a in the stored state.
            link_nodes<L, WALLS, -1>(p.g, x, y, z, idx, wall);
            C f[Q];
            static_for<Q>([&](auto ac) {
                constexpr int a = decltype(ac)::value;
                constexpr bool aligned = kLattice<L>.e[a][0] == 0;
                f[a] = Store<S>::load(get<aligned>(g + gather_offset<L>(kPull, a, own, idx[a], WALLS && wall[a], TS)));
            });
            if constexpr (WALLS) nodal_fill<L>(p.g, x, y, z, f);
            const Moments<L, C> m = node_moments<L, C, FORCE, COMP, Store<S>::kDeviation>(f, p.F);
            const C usq = m.ux * m.ux + m.uy * m.uy + m.uz * m.uz;
            C uF = C(0);
            if constexpr (FORCE) uF = m.ux * p.F[0] + m.uy * p.F[1] + m.uz * p.F[2];
            C m0 = C(0), m1[3] = {C(0), C(0), C(0)}, m2[3] = {C(0), C(0), C(0)},
              m3[3] = {C(0), C(0), C(0)};
            C tsum = C(0);  // sum_a l_a (feq_a - f_a - G_a/2)
            static_for<Q>([&](auto ac) {
                constexpr int a = decltype(ac)::value;
                constexpr int ex = kLattice<L>.e[a][0], ey = kLattice<L>.e[a][1], ez = kLattice<L>.e[a][2];
                const C w = C(kLattice<L>.w[a]);
                const C wl = w * ls[a];
                const C edu = eterm<ex>(m.ux) + eterm<ey>(m.uy) + eterm<ez>(m.uz);
                m0 += wl;
                m1[0] += eterm<ex>(wl);
                m1[1] += eterm<ey>(wl);
                m1[2] += eterm<ez>(wl);
                const C wle = wl * edu;
                m2[0] += eterm<ex>(wle);
                m2[1] += eterm<ey>(wle);
                m2[2] += eterm<ez>(wle);
                const C q = C(3) * edu + C(4.5) * edu * edu - C(1.5) * usq;
                const C feq = w * (m.rho + (COMP ? m.rf * q : q));
                C gterm = C(0);
                if constexpr (FORCE) {
                    const C eF = eterm<ex>(p.F[0]) + eterm<ey>(p.F[1]) + eterm<ez>(p.F[2]);
                    const C wlF = wl * eF;
                    m3[0] += eterm<ex>(wlF);
                    m3[1] += eterm<ey>(wlF);
                    m3[2] += eterm<ez>(wlF);
                    gterm = C(0.5) * w * (C(3) * (eF - uF) + C(9) * edu * eF);
                }
                tsum += ls[a] * (feq - f[a] - gterm);
            });
            const C u[3] = {m.ux, m.uy, m.uz};
            const C binv = COMP ? C(1) / m.rf : C(1);  // du/dj = I/rho
            C A[3], B[3], V[3];
            for (int d = 0; d < 3; ++d) {
                A[d] = C(3) * m1[d] + C(9) * m2[d] - C(3) * m0 * u[d];
                B[d] = FORCE ? C(9) * m3[d] - C(3) * m0 * p.F[d] : C(0);
                V[d] = p.omega * A[d] + p.half * B[d] * binv;
            }
            C base = p.omega * m0;
            if constexpr (COMP) {
                const C P = m0 * (C(1) - C(1.5) * usq) + C(3) * (m1[0] * u[0] + m1[1] * u[1] + m1[2] * u[2]) +
                            C(4.5) * (m2[0] * u[0] + m2[1] * u[1] + m2[2] * u[2]);
                base = p.omega * P - (V[0] * u[0] + V[1] * u[1] + V[2] * u[2]);
            }
            const C keep = C(1) - p.omega;
            const auto ws = WaveStores<C>::template make<Q>(lam_out, own, p.g);
            static_for<Q>([&](auto ac) {
                constexpr int b = decltype(ac)::value;
                constexpr int ex = kLattice<L>.e[b][0], ey = kLattice<L>.e[b][1], ez = kLattice<L>.e[b][2];
                ws.put(slot<Q>(b, own, TS),
                       C(keep * ls[b] + base + (eterm<ex>(V[0]) + eterm<ey>(V[1]) + eterm<ez>(V[2]))));
            });
            part[0] = -double(p.omega) * double(p.omega) * double(tsum);
            for (int d = 0; d < kDim<L>; ++d)
                part[1 + d] = double(A[d]) + 0.5 * double(p.half) * double(B[d]) * double(binv);
        }
    }
    block_accumulate(part, acc);
}

// Output map: lambda^n_a = e_a . ubar (rho0 = 1) from ubar = dJ/du^n, and
// Fbar += ubar/2 (u^n carries F/2).  In the compressible model (COMP) u^n
// = (sum e f + F/2)/rho of the final state fN (two-lattice layout):
// lambda^n_a = ubar . (e_a - u)/rho and Fbar += ubar/(2 rho).  Solid nodes
// get lambda = 0.
template <int L, class S, bool WALLS, bool COMP>
__global__ __launch_bounds__(256) void k_adjoint_seed(const double* __restrict__ ubar,
                                                      const S* __restrict__ fN,
                                                      typename Store<S>::C* __restrict__ lam,
                                                      double* __restrict__ acc, IoArgs p)
{
    using C = typename Store<S>::C;
    constexpr int Q = Lattice<L>::Q;
    const Dims& g = p.g;
    int x, y, z;
    const bool inside = node_of_item(g, p.bx_shift, x, y, z);
    double part[kAccSlots] = {0.0, 0.0, 0.0, 0.0};
    if (inside) {
        const unsigned N = g.N;
        const unsigned own = unsigned(x) + unsigned(g.nx) * (unsigned(y) + unsigned(g.ny) * unsigned(z));
        const bool fluid = !(WALLS && is_solid(g, x, y, z));
        double ub[3] = {0.0, 0.0, 0.0};
        if (fluid)
            for (int d = 0; d < kDim<L>; ++d) ub[d] = ubar[size_t(d) * N + own];
        double shift = 0.0, scale = 1.0;  // lambda_a = scale (e_a . ubar) - shift
        if (COMP && fluid) {
            C fn[Q];
            gather_node<L, S, WALLS>(fN, p, x, y, z, own, fn);
            double sum, rho, u[3];
            node_rho_u<L, S>(fn, p, sum, rho, u);
            scale = 1.0 / rho;
            shift = (ub[0] * u[0] + ub[1] * u[1] + ub[2] * u[2]) * scale;
        }
        static_for<Q>([&](auto ac) {
            constexpr int a = decltype(ac)::value;
            constexpr auto& LT = kLattice<L>;
            const double eu = eterm<LT.e[a][0]>(ub[0]) + eterm<LT.e[a][1]>(ub[1]) + eterm<LT.e[a][2]>(ub[2]);
            lam[slot<Q>(a, own, g.S)] = C(COMP ? scale * eu - shift : eu);
        });
        for (int d = 0; d < kDim<L>; ++d) part[1 + d] = 0.5 * ub[d] * scale;
    }
    block_accumulate(part, acc);
}

// Transpose of Eq. (bb) on the walls of the nodal scheme: on each wall node,
// the adjoint of every unknown population is added to the opposite one and
// cleared.  One work-item per node of the two wall planes.
template <int L, class C>
__global__ __launch_bounds__(256) void k_adjoint_nodal_bt(C* __restrict__ lam, Dims g)
{
    constexpr int Q = Lattice<L>::Q;
    const int ax = g.nodal;
    const int n[3] = {g.nx, g.ny, g.nz};
    const int u = ax == 0 ? 1 : 0, v = ax == 2 ? 1 : 2;  // the two other axes
    const unsigned plane = unsigned(n[u]) * unsigned(n[v]);
    const unsigned i = blockIdx.x * 256u + threadIdx.x;
    if (i >= 2 * plane) return;
    const unsigned k = i % plane;
    int c[3];
    c[ax] = i < plane ? 0 : n[ax] - 1;
    c[u] = int(k % unsigned(n[u]));
    c[v] = int(k / unsigned(n[u]));
    if (is_solid(g, c[0], c[1], c[2])) return;
    const unsigned own = node_index(g, c[0], c[1], c[2]);
    const int side = c[ax] == 0 ? 1 : -1;
    static_for<Q>([&](auto ac) {
        constexpr int a = decltype(ac)::value;
        constexpr auto& LT = kLattice<L>;
        if constexpr (LT.e[a][0] != 0 || LT.e[a][1] != 0 || LT.e[a][2] != 0) {
            const int e = ax == 0 ? LT.e[a][0] : (ax == 1 ? LT.e[a][1] : LT.e[a][2]);
            if (e == side) {
                C* la = lam + slot<Q>(a, own, g.S);
                C* lb = lam + slot<Q>(Lattice<L>::opp(a), own, g.S);
                *lb = *lb + *la;
                *la = C(0);
            }
        }
    });
}

// Init map: f^0_a = w_a (rho + 3 e.u0 + 4.5 (e.u0)^2 - 1.5 u0.u0) + noise, so
// u0bar = sum_a lambda^0_a w_a (3 e_a + 9 (e_a.u0) e_a - 3 u0); the
// compressible equilibrium carries the extra factor rho0 of the node.
template <int L, class S, bool WALLS, bool COMP>
__global__ __launch_bounds__(256) void k_adjoint_init_map(const typename Store<S>::C* __restrict__ lam,
                                                          const double* __restrict__ rho0,
                                                          const double* __restrict__ u0,
                                                          double* __restrict__ u0bar, Dims g,
                                                          int bx_shift)
{
    constexpr int Q = Lattice<L>::Q;
    int x, y, z;
    if (!node_of_item(g, bx_shift, x, y, z)) return;
    const unsigned N = g.N;
    const unsigned own = unsigned(x) + unsigned(g.nx) * (unsigned(y) + unsigned(g.ny) * unsigned(z));
    if (WALLS && is_solid(g, x, y, z)) {
        for (int d = 0; d < 3; ++d) u0bar[size_t(d) * N + own] = 0.0;
        return;
    }
    const double u[3] = {u0[own], u0[size_t(N) + own], kDim<L> == 3 ? u0[2 * size_t(N) + own] : 0.0};
    double m0 = 0.0, m1[3] = {0.0, 0.0, 0.0}, m2[3] = {0.0, 0.0, 0.0};
    static_for<Q>([&](auto ac) {
        constexpr int a = decltype(ac)::value;
        constexpr auto& LT = kLattice<L>;
        const double wl = LT.w[a] * double(lam[slot<Q>(a, own, g.S)]);
        const double edu = eterm<LT.e[a][0]>(u[0]) + eterm<LT.e[a][1]>(u[1]) + eterm<LT.e[a][2]>(u[2]);
        m0 += wl;
        m1[0] += eterm<LT.e[a][0]>(wl);
        m1[1] += eterm<LT.e[a][1]>(wl);
        m1[2] += eterm<LT.e[a][2]>(wl);
        m2[0] += eterm<LT.e[a][0]>(wl * edu);
        m2[1] += eterm<LT.e[a][1]>(wl * edu);
        m2[2] += eterm<LT.e[a][2]>(wl * edu);
    });
    const double r = COMP ? rho0[own] : 1.0;
    for (int d = 0; d < 3; ++d)
        u0bar[size_t(d) * N + own] = d < kDim<L> ? r * (3.0 * m1[d] + 9.0 * m2[d] - 3.0 * m0 * u[d]) : 0.0;
}

// Sums the per-workgroup slots in workgroup order (one workgroup).
[[maybe_unused]] static __global__ __launch_bounds__(256) void k_adjoint_sum(const double* __restrict__ acc, size_t nblocks,
                                                     double* __restrict__ out)
{
    __shared__ double s[kAccSlots][256];
    const int t = threadIdx.x;
    double v[kAccSlots] = {0.0, 0.0, 0.0, 0.0};
    for (size_t b = t; b < nblocks; b += 256)
        for (int c = 0; c < kAccSlots; ++c) v[c] += acc[b * kAccSlots + c];
    for (int c = 0; c < kAccSlots; ++c) s[c][t] = v[c];
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (t < h)
            for (int c = 0; c < kAccSlots; ++c) s[c][t] += s[c][t + h];
        __syncthreads();
    }
    if (t == 0)
        for (int c = 0; c < kAccSlots; ++c) out[c] = s[c][0];
}

[[maybe_unused]] static __global__ __launch_bounds__(256) void k_fill_zero(double* __restrict__ p, size_t n)
{
    const size_t i = blockIdx.x * size_t(256) + threadIdx.x;
    if (i < n) p[i] = 0.0;
}

}  // namespace imexlbm
