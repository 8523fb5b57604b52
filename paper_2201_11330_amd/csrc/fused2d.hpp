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

// Placement of the workgroups (one per inner block; gx x gy blocks).  With
// tw = 0 the launch is a gx x gy grid.  Otherwise it is one-dimensional and
// XCD-aware: the hardware hands workgroup i to XCD i % 8, and the k-th
// workgroup of an XCD takes block k % (tw*th) of that XCD's (k / (tw*th))-th
// tile of tw x th blocks, so the neighbouring regions whose rings overlap
// are read through the same L2.  Padding workgroups (past the last tile or
// the box) exit at once.
struct FuseMap {
    int gx, gy;        // inner blocks along x and y
    int tw, th;        // blocks per tile (0: plain 2D grid)
    int tiles_x, tiles;
};

__device__ __forceinline__ bool fuse_block(const FuseMap& m, int& bx, int& by)
{
    if (m.tw == 0) {
        bx = int(blockIdx.x);
        by = int(blockIdx.y);
        return true;
    }
    const int id = int(blockIdx.x), per_tile = m.tw * m.th;
    const int k = id >> 3, t = (k / per_tile) * 8 + (id & 7), w = k % per_tile;
    if (t >= m.tiles) return false;
    bx = (t % m.tiles_x) * m.tw + w % m.tw;
    by = (t / m.tiles_x) * m.th + w / m.tw;
    return bx < m.gx && by < m.gy;
}

// XCD-aware placement from this many inner blocks up, in tiles of 8 x 8
// blocks.  Measured on MI355X (FP64): +3 to +21 % from 576 blocks (192^2)
// to 65,536 (2048^2), most on ragged boxes; at 256 blocks (128^2) the
// padding to whole tiles costs 15 %.  Tiles of 16 x 16 blocks were no better
// from 4096 blocks up and worse below.
constexpr int kFuseXcdMinBlocks = 512;
constexpr int kFuseXcdTile = 8;

// The placement of an nx x ny box: tiles of tile x tile blocks (0: plain
// grid), and the launch grid that goes with it.
inline FuseMap fuse_plan(int nx, int ny, int tile, dim3* grid)
{
    FuseMap m{};
    m.gx = (nx + kFuseInner - 1) / kFuseInner;
    m.gy = (ny + kFuseInner - 1) / kFuseInner;
    if (tile <= 0) {
        *grid = dim3(unsigned(m.gx), unsigned(m.gy), 1);
        return m;
    }
    m.tw = m.th = tile;
    m.tiles_x = (m.gx + tile - 1) / tile;
    m.tiles = m.tiles_x * ((m.gy + tile - 1) / tile);
    *grid = dim3(unsigned((m.tiles + 7) / 8) * 8u * unsigned(tile * tile), 1, 1);
    return m;
}

template <class S, bool FORCE, bool COMP, bool NT>
__global__ __launch_bounds__(256) void k_step_ab_fused2d(const S* __restrict__ src, S* __restrict__ dst,
                                                         StepArgs<typename Store<S>::C> p, FuseMap m)
{
    using C = typename Store<S>::C;
    constexpr int L = 0, Q = Lattice<L>::Q, E = kFuseEdge, H = kFuseSteps, I = kFuseInner;
    int bx, by;
    if (!fuse_block(m, bx, by)) return;  // uniform over the workgroup
    __shared__ C sh[Q][E][E];
    const Dims& g = p.g;
    const int lx = int(threadIdx.x) & (E - 1), ly = int(threadIdx.x) / E;
    int gx = (bx * I - H + lx) % g.nx;
    int gy = (by * I - H + ly) % g.ny;
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
    const int ox = bx * I + ix, oy = by * I + iy;
    if (ox >= g.nx || oy >= g.ny) return;
    const unsigned own = unsigned(ox) + unsigned(g.nx) * unsigned(oy);
    static_for<Q>([&](auto ac) {
        constexpr int a = decltype(ac)::value;
        put<NT>(dst + slot<Q>(a, own, TS), Store<S>::save(f[a]));
    });
}

}  // namespace imexlbm
