// Several time steps of a fully periodic D2Q9 box in one launch (two-lattice
// pattern, temporal blocking in LDS).
//
// A 256-item workgroup holds an E x E region of nodes (E = 16: one node per
// work-item; E = 32: four), loads the stored state of that region once and
// runs kFuseSteps = 4 steps on it: each step puts the post-collision values
// into LDS, pulls f_a(x) from x - e_a in LDS (Eq. (propagation)) and
// collides (Eq. (collision), the collide() of the one-step kernels).  A
// node's value after 4 steps depends only on nodes within 4 links (Chebyshev
// distance), so the inner (E - 8) x (E - 8) nodes are exact and are the ones
// stored; the ring around them is recomputed by the neighbouring workgroups,
// which replaces a grid-wide barrier by redundant arithmetic.  Region nodes
// take their coordinates modulo the box, so boxes smaller than a region wrap
// the same way.  With a reduced-precision storage every step rounds its
// result through the storage type, as a store and reload would, so the state
// after 4 steps is bit for bit that of 4 one-step launches.
//
// Why: a small box is latency-bound with one launch per step (128 x 128
// nodes: 64 workgroups, ~3-4 us per step, most of it one dependent
// load-collide-store chain), and on large boxes a launch reads and writes
// the state once per 4 steps (36 B per FP64 update instead of 144) at the
// price of the ring's arithmetic: 4x the useful collisions with E = 16,
// 1.78x with E = 32.  Measured on MI355X, FP64: 128^2 12,800-13,300 vs
// 3,900-5,800 MLUPS (one step per launch); 4096^2 95,000 vs 42,900 MLUPS
// (E = 32 vs the two-node one-step kernel).  4 steps per pass beat 2, 3, 5
// and 6 on every box from 64^2 to 4096^2.
#pragma once

#include "kernels.hpp"

namespace imexlbm {

constexpr int kFuseSteps = 4;  // steps per launch (halo width)

// Inner (stored) nodes per region edge.
template <int E>
inline constexpr int kFuseInnerOf = E - 2 * kFuseSteps;

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

// Choice of region and placement, measured on MI355X (FP64):
//  * E = 32 (72 KB of LDS per workgroup, 2 waves per SIMD) from
//    kFuseBigMinBlocks of its 24 x 24 blocks up, on a plain grid: x1.09 at
//    384^2 (256 blocks), x1.17-1.26 at 512^2, x1.36 at 1000 x 777, x1.38 at
//    1024^2, x1.47 at 4096^2 over E = 16; with fewer blocks it fills too few
//    CUs (x0.84 at 320^2, 196 blocks; x0.73 at 256^2).  Its XCD-aware
//    placement was slower (x0.92-0.99).
//  * E = 16 otherwise, XCD-aware in tiles of 8 x 8 blocks from
//    kFuseXcdMinBlocks of its 8 x 8 blocks up: +3 to +21 % from 192^2 to
//    2048^2, most on ragged boxes; at 256 blocks (128^2) the padding to
//    whole tiles costs 15 %.  Tiles of 16 x 16 blocks were no better.
constexpr int kFuseBigMinBlocks = 256;
constexpr int kFuseXcdMinBlocks = 512;
constexpr int kFuseXcdTile = 8;

// The placement of an nx x ny box in blocks of `inner` x `inner` stored
// nodes: tiles of tile x tile blocks (0: plain grid), and the launch grid
// that goes with it.
inline FuseMap fuse_plan(int nx, int ny, int inner, int tile, dim3* grid)
{
    FuseMap m{};
    m.gx = (nx + inner - 1) / inner;
    m.gy = (ny + inner - 1) / inner;
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

template <int E, class S, bool FORCE, bool COMP, bool NT>
__global__ __launch_bounds__(256) void k_step_ab_fused2d(const S* __restrict__ src, S* __restrict__ dst,
                                                         StepArgs<typename Store<S>::C> p, FuseMap m)
{
    using C = typename Store<S>::C;
    constexpr int L = 0, Q = Lattice<L>::Q, H = kFuseSteps, I = kFuseInnerOf<E>;
    constexpr int NE = E / 16, NPT = NE * NE;  // nodes per work-item: (tx + 16i, ty + 16j)
    static_assert(E % 16 == 0 && I >= 1, "region edge must be a multiple of 16 and exceed the ring");
    int bx, by;
    if (!fuse_block(m, bx, by)) return;  // uniform over the workgroup
    __shared__ C sh[Q][E][E];
    const Dims& g = p.g;
    const int tx = int(threadIdx.x) & 15, ty = int(threadIdx.x) >> 4;
    const int TS = g.S;
    C f[NPT][Q];
#pragma unroll
    for (int j = 0; j < NPT; ++j) {
        const int lx = tx + 16 * (j % NE), ly = ty + 16 * (j / NE);
        int gx = (bx * I - H + lx) % g.nx;
        int gy = (by * I - H + ly) % g.ny;
        gx += gx < 0 ? g.nx : 0;
        gy += gy < 0 ? g.ny : 0;
        const unsigned node = unsigned(gx) + unsigned(g.nx) * unsigned(gy);
        static_for<Q>([&](auto ac) {
            constexpr int a = decltype(ac)::value;
            f[j][a] = Store<S>::load(src[slot<Q>(a, node, TS)]);
        });
    }
    for (int s = 0; s < H; ++s) {
#pragma unroll
        for (int j = 0; j < NPT; ++j) {
            const int lx = tx + 16 * (j % NE), ly = ty + 16 * (j / NE);
            static_for<Q>([&](auto ac) {
                constexpr int a = decltype(ac)::value;
                sh[a][ly][lx] = f[j][a];
            });
        }
        __syncthreads();
        // Pull; a region-edge node reads a clamped (stale) neighbour, which
        // only reaches nodes outside the stored inner block.
#pragma unroll
        for (int j = 0; j < NPT; ++j) {
            const int lx = tx + 16 * (j % NE), ly = ty + 16 * (j / NE);
            static_for<Q>([&](auto ac) {
                constexpr int a = decltype(ac)::value;
                constexpr int ex = kLattice<L>.e[a][0], ey = kLattice<L>.e[a][1];
                int sx = lx - ex, sy = ly - ey;
                if constexpr (ex == 1) sx = sx < 0 ? 0 : sx;
                if constexpr (ex == -1) sx = sx > E - 1 ? E - 1 : sx;
                if constexpr (ey == 1) sy = sy < 0 ? 0 : sy;
                if constexpr (ey == -1) sy = sy > E - 1 ? E - 1 : sy;
                f[j][a] = sh[a][sy][sx];
            });
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < NPT; ++j) {
            collide<L, C, FORCE, COMP, Store<S>::kDeviation>(f[j], p.c);
            if constexpr (!std::is_same_v<S, C>) {
                static_for<Q>([&](auto ac) {
                    constexpr int a = decltype(ac)::value;
                    f[j][a] = Store<S>::load(Store<S>::save(f[j][a]));
                });
            }
        }
    }
#pragma unroll
    for (int j = 0; j < NPT; ++j) {
        const int lx = tx + 16 * (j % NE), ly = ty + 16 * (j / NE);
        const int ix = lx - H, iy = ly - H;
        if (ix < 0 || ix >= I || iy < 0 || iy >= I) continue;
        const int ox = bx * I + ix, oy = by * I + iy;
        if (ox >= g.nx || oy >= g.ny) continue;
        const unsigned own = unsigned(ox) + unsigned(g.nx) * unsigned(oy);
        // Non-temporal global stores: the nt | sc1 buffer stores of the
        // one-step kernels measured slower here (128^2: 11,950 vs 12,500-
        // 13,300 MLUPS; 4096^2: 83,900 vs 89,600-91,000), the written state
        // being read again, largely from cache, by the next launch.
        static_for<Q>([&](auto ac) {
            constexpr int a = decltype(ac)::value;
            put<NT>(dst + slot<Q>(a, own, TS), Store<S>::save(f[j][a]));
        });
    }
}

}  // namespace imexlbm
