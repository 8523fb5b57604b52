// Several time steps of a fully periodic D2Q9 box in one launch (two-lattice
// pattern, temporal blocking in LDS).
//
// A 256-item workgroup holds a 16 x 16 region of nodes, one per work-item,
// loads the stored state of that region once and runs kFuseSteps = 4 steps
// on it: each step puts the post-collision values into LDS, pulls f_a(x)
// from x - e_a in LDS (Eq. (propagation)) and collides (Eq. (collision),
// the collide() of the one-step kernels).  A node's value after 4 steps
// depends only on nodes within 4 links (Chebyshev distance), so the inner
// 8 x 8 nodes are exact and are the ones stored; the ring around them is
// recomputed by the neighbouring workgroups, which replaces a grid-wide
// barrier by redundant arithmetic.  Region nodes take their coordinates
// modulo the box, so boxes smaller than a region wrap the same way.  With a
// reduced-precision storage every step rounds its result through the storage
// type, as a store and reload would, so the state after 4 steps is bit for
// bit that of 4 one-step launches.
//
// Why: a small box is latency-bound with one launch per step (128 x 128
// nodes: 64 workgroups, ~3-4 us per step, most of it one dependent
// load-collide-store chain), and on large boxes the 4 steps per pass move
// (read 72 + write 18) B per FP64 update instead of 144.  Measured on
// MI355X, FP64: 128^2 13,370 vs 3,900-5,700 MLUPS; 4096^2 62,765 vs
// 42,913 MLUPS (two-node one-step kernel).  4 steps per pass beat 2, 3, 5
// and 6 on every box from 64^2 to 4096^2 (the redundant ring costs 4x the
// arithmetic at 4 steps and 16x at 6).
#pragma once

#include "kernels.hpp"

namespace imexlbm {

constexpr int kFuseEdge = 16;  // region edge: kFuseEdge^2 = 256 work-items
constexpr int kFuseSteps = 4;  // steps per launch (halo width)
constexpr int kFuseInner = kFuseEdge - 2 * kFuseSteps;

template <class S, bool FORCE, bool COMP, bool NT>
__global__ __launch_bounds__(256) void k_step_ab_fused2d(const S* __restrict__ src, S* __restrict__ dst,
                                                         StepArgs<typename Store<S>::C> p)
{
    using C = typename Store<S>::C;
    constexpr int L = 0, Q = Lattice<L>::Q, E = kFuseEdge, H = kFuseSteps, I = kFuseInner;
    __shared__ C sh[Q][E][E];
    const Dims& g = p.g;
    const int lx = int(threadIdx.x) & (E - 1), ly = int(threadIdx.x) / E;
    int gx = (int(blockIdx.x) * I - H + lx) % g.nx;
    int gy = (int(blockIdx.y) * I - H + ly) % g.ny;
    gx += gx < 0 ? g.nx : 0;
    gy += gy < 0 ? g.ny : 0;
    const int TS = g.S;
    const unsigned node = unsigned(gx) + unsigned(g.nx) * unsigned(gy);
    C f[Q];
    static_for<Q>([&](auto ac) {
        constexpr int a = decltype(ac)::value;
        f[a] = Store<S>::load(src[slot<Q>(a, node, TS)]);
    });
    for (int s = 0; s < H; ++s) {
        static_for<Q>([&](auto ac) {
            constexpr int a = decltype(ac)::value;
            sh[a][ly][lx] = f[a];
        });
        __syncthreads();
        // Pull; a region-edge node reads a clamped (stale) neighbour, which
        // only reaches nodes outside the stored inner block.
        static_for<Q>([&](auto ac) {
            constexpr int a = decltype(ac)::value;
            constexpr int ex = kLattice<L>.e[a][0], ey = kLattice<L>.e[a][1];
            int sx = lx - ex, sy = ly - ey;
            if constexpr (ex == 1) sx = sx < 0 ? 0 : sx;
            if constexpr (ex == -1) sx = sx > E - 1 ? E - 1 : sx;
            if constexpr (ey == 1) sy = sy < 0 ? 0 : sy;
            if constexpr (ey == -1) sy = sy > E - 1 ? E - 1 : sy;
            f[a] = sh[a][sy][sx];
        });
        __syncthreads();
        collide<L, C, FORCE, COMP, Store<S>::kDeviation>(f, p.c);
        if constexpr (!std::is_same_v<S, C>) {
            static_for<Q>([&](auto ac) {
                constexpr int a = decltype(ac)::value;
                f[a] = Store<S>::load(Store<S>::save(f[a]));
            });
        }
    }
    const int ix = lx - H, iy = ly - H;
    if (ix < 0 || ix >= I || iy < 0 || iy >= I) return;
    const int ox = int(blockIdx.x) * I + ix, oy = int(blockIdx.y) * I + iy;
    if (ox >= g.nx || oy >= g.ny) return;
    const unsigned own = unsigned(ox) + unsigned(g.nx) * unsigned(oy);
    static_for<Q>([&](auto ac) {
        constexpr int a = decltype(ac)::value;
        put<NT>(dst + slot<Q>(a, own, TS), Store<S>::save(f[a]));
    });
}

}  // namespace imexlbm
