// Full-order MPM transfers on gfx950 (paper Section 2.2, Algorithm 1):
// particle-to-grid scatter, grid update with boundary band, grid-to-particle
// gather with deformation-gradient update, and the cell sort.
//
// Two P2G paths:
//  * unsorted: one thread per particle, 3^d x (d+1) float atomics into the
//    grid (L2 atomics) -- correct for any particle order;
//  * sorted (MR_SORTED): one workgroup per 4x4x4 (2D: 8x8) tile of stencil
//    base cells, whose particles the cell sort made contiguous and ordered
//    slot-major (all first particles of the tile's cells, then all second
//    ones, ...), so that the lanes of a wave sit in distinct cells.  The
//    workgroup accumulates its particles into an LDS copy of the tile's node
//    region (tile plus stencil reach plus one cell of drift margin on each
//    side) with plain LDS read-modify-write, then flushes the region to HBM
//    with one global atomic per non-zero node channel.  Particles that drifted beyond
//    the margin since the sort fall back to global atomics.
#include "mpm_kernels.h"

namespace mr {

// zero fill by a kernel rather than hipMemsetAsync, so that every launch of
// the full-order path can be captured in a graph (memset nodes are avoided
// there); count in 32-bit words
__global__ void zero_words_kernel(uint32_t *p, int64_t words)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < words;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

inline void zero_words(void *p, int64_t words, hipStream_t st)
{
    if (words <= 0) return;
    const int64_t blocks = (words + 255) / 256;
    zero_words_kernel<<<(unsigned)(blocks < 4096 ? blocks : 4096), 256, 0, st>>>(
        reinterpret_cast<uint32_t *>(p), words);
}

}  // namespace mr

#include <stdio.h>

namespace mr {

// ---------------------------------------------------------------------------
// particle access helpers (SoA, component-major)

template <int D>
struct PartPtrs {
    const float *x, *v, *C, *F, *m, *V0;
    float m_u, V0_u;
    int64_t n;
};

template <int D>
__device__ __forceinline__ void load_payload(const PartPtrs<D> &pp, int64_t p, bool apic,
                                             int model, float mu, float la, float dt,
                                             const GridK &g, Stencil<D> &st, P2GPayload<D> &pl,
                                             bool &ok)
{
    const int64_t n = pp.n;
    float xp[D], vp[D], Fp[D * D], tau[D * D];
#pragma unroll
    for (int a = 0; a < D; ++a) {
        xp[a] = pp.x[a * n + p];
        vp[a] = pp.v[a * n + p];
    }
#pragma unroll
    for (int k = 0; k < D * D; ++k) Fp[k] = pp.F[k * n + p];
    ok = make_stencil<D>(g, xp, st);
    ok = kirchhoff<D>(model, mu, la, Fp, tau) && ok;
    float m = pp.m ? pp.m[p] : pp.m_u;
    float V0 = pp.V0 ? pp.V0[p] : pp.V0_u;
    pl.m = m;
#pragma unroll
    for (int a = 0; a < D; ++a) pl.mv[a] = m * vp[a];
    float sc = dt * V0;
#pragma unroll
    for (int k = 0; k < D * D; ++k) {
        pl.mC[k] = apic ? m * pp.C[k * n + p] : 0.0f;
        pl.S[k] = sc * tau[k];
    }
}

template <int D>
__device__ __forceinline__ void scatter_global(const GridK &g, const Stencil<D> &st,
                                               const P2GPayload<D> &pl, float *grid)
{
    const int oz = (D == 3) ? 3 : 1;
    for (int o2 = 0; o2 < oz; ++o2)
#pragma unroll
        for (int o1 = 0; o1 < 3; ++o1)
#pragma unroll
            for (int o0 = 0; o0 < 3; ++o0) {
                float mom[D];
                float mw = p2g_node<D>(g, st, pl, o0, o1, o2, mom);
                int64_t i = node_lin(g, st.base[0] + o0, st.base[1] + o1,
                                     D == 3 ? st.base[2] + o2 : 0);
                float *gp = grid + 4 * i;
                atomicAdd(gp, mw);
#pragma unroll
                for (int a = 0; a < D; ++a) atomicAdd(gp + 1 + a, mom[a]);
            }
}

template <int D>
__global__ void __launch_bounds__(256) p2g_atomic_kernel(GridK g, PartPtrs<D> pp,
                                                         const int32_t *subset, int64_t ns,
                                                         int apic, int model, float mu,
                                                         float la, float dt, float *grid,
                                                         int32_t *flag)
{
    int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= ns) return;
    int64_t p = subset ? (int64_t)subset[s] : s;
    Stencil<D> st;
    P2GPayload<D> pl;
    bool ok;
    load_payload<D>(pp, p, apic != 0, model, mu, la, dt, g, st, pl, ok);
    if (!ok) {
        raise_flag(flag, MR_FLAG_DOMAIN);
        return;
    }
    scatter_global<D>(g, st, pl, grid);
}

// ---------------------------------------------------------------------------
// tiling used by the cell sort and the sorted P2G

template <int D>
struct Tiling {
    static constexpr int TS = (D == 3) ? 4 : 8;          // cells per tile edge
    static constexpr int CELLS = (D == 3) ? 64 : 64;     // cells per tile
    static constexpr int R = TS + 4;                     // LDS node region edge
    static constexpr int RN = (D == 3) ? R * R * R : R * R;
};

struct TileGeom {
    int nt0, nt1, nt2;  // tiles per dimension
    int64_t ntiles;
};

template <int D>
inline TileGeom tile_geom(const GridK &g)
{
    // valid base cells are 0 .. n-3 per dimension
    TileGeom t;
    int TS = Tiling<D>::TS;
    t.nt0 = (int)ceil_div(g.n0 - 2, TS);
    t.nt1 = (int)ceil_div(g.n1 - 2, TS);
    t.nt2 = D == 3 ? (int)ceil_div(g.n2 - 2, TS) : 1;
    t.ntiles = (int64_t)t.nt0 * t.nt1 * t.nt2;
    return t;
}

// tile-major cell key: tile * CELLS + local cell (x fastest); -1 if outside
template <int D>
__device__ __forceinline__ int32_t cell_key(const GridK &g, const TileGeom &tg, const float *xp)
{
    const int TS = Tiling<D>::TS;
    const int n[3] = {g.n0, g.n1, g.n2};
    int b[3] = {0, 0, 0};
    bool ok = true;
#pragma unroll
    for (int a = 0; a < D; ++a) {
        float bf = floorf(xp[a] * g.inv_dx - 0.5f);
        ok = ok && (bf >= 0.0f) && (bf + 2.0f <= (float)(n[a] - 1));
        b[a] = ok ? (int)bf : 0;
    }
    if (!ok) return -1;
    int t = (b[0] / TS) + tg.nt0 * ((b[1] / TS) + tg.nt1 * (D == 3 ? b[2] / TS : 0));
    int c = (b[0] % TS) + TS * ((b[1] % TS) + (D == 3 ? TS * (b[2] % TS) : 0));
    return t * Tiling<D>::CELLS + c;
}

template <int D>
__global__ void cell_key_kernel(GridK g, TileGeom tg, const float *x, int64_t n, int32_t *keys,
                                int32_t *counts, int32_t *flag)
{
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    float xp[D];
#pragma unroll
    for (int a = 0; a < D; ++a) xp[a] = x[a * n + p];
    int32_t k = cell_key<D>(g, tg, xp);
    if (k < 0) {
        raise_flag(flag, MR_FLAG_DOMAIN);
        k = (int32_t)(tg.ntiles * Tiling<D>::CELLS);  // overflow bucket at the end
    }
    keys[p] = k;
    if (counts) atomicAdd(counts + k, 1);
}

// --- exclusive scan of int32 (three phases) ---------------------------------
constexpr int SCAN_BLOCK = 1024;

__device__ __forceinline__ int block_exclusive_scan(int v, int *sh, int &total)
{
    // sh: blockDim.x ints; Hillis-Steele over LDS (blockDim = SCAN_BLOCK)
    int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int off = 1; off < (int)blockDim.x; off <<= 1) {
        int add = (t >= off) ? sh[t - off] : 0;
        __syncthreads();
        sh[t] += add;
        __syncthreads();
    }
    total = sh[blockDim.x - 1];
    int incl = sh[t];
    __syncthreads();
    return incl - v;
}

__global__ void __launch_bounds__(SCAN_BLOCK) scan_blocks_kernel(const int32_t *in, int64_t n,
                                                                  int32_t *out, int32_t *block_sums)
{
    __shared__ int sh[SCAN_BLOCK];
    int64_t i = (int64_t)blockIdx.x * SCAN_BLOCK + threadIdx.x;
    int v = (i < n) ? in[i] : 0;
    int total;
    int ex = block_exclusive_scan(v, sh, total);
    if (i < n) out[i] = ex;
    if (threadIdx.x == 0) block_sums[blockIdx.x] = total;
}

// single workgroup: exclusive scan of nb block sums in place (serial chunks)
__global__ void __launch_bounds__(SCAN_BLOCK) scan_sums_kernel(int32_t *sums, int64_t nb,
                                                                int32_t *grand_total)
{
    __shared__ int sh[SCAN_BLOCK];
    int carry = 0;
    for (int64_t base = 0; base < nb; base += SCAN_BLOCK) {
        int64_t i = base + threadIdx.x;
        int v = (i < nb) ? sums[i] : 0;
        int total;
        int ex = block_exclusive_scan(v, sh, total);
        if (i < nb) sums[i] = ex + carry;
        carry += total;
    }
    if (threadIdx.x == 0 && grand_total) *grand_total = carry;
}

__global__ void scan_add_kernel(int32_t *out, int64_t n, const int32_t *block_sums)
{
    int64_t i = (int64_t)blockIdx.x * SCAN_BLOCK + threadIdx.x;
    if (i < n) out[i] += block_sums[blockIdx.x];
}

int32_t exclusive_scan(const int32_t *in, int64_t n, int32_t *out, int32_t *block_sums,
                       int32_t *grand_total, hipStream_t st)
{
    int64_t nb = ceil_div(n, SCAN_BLOCK);
    scan_blocks_kernel<<<(unsigned)nb, SCAN_BLOCK, 0, st>>>(in, n, out, block_sums);
    scan_sums_kernel<<<1, SCAN_BLOCK, 0, st>>>(block_sums, nb, grand_total);
    scan_add_kernel<<<(unsigned)nb, SCAN_BLOCK, 0, st>>>(out, n, block_sums);
    MR_LAUNCH_CHECK();
    return MR_OK;
}

// --- counting sort into cells, then stable order inside each cell ----------
__global__ void cell_scatter_kernel(const int32_t *keys, int64_t n, const int32_t *offsets,
                                    int32_t *fill, int32_t *cell_sorted)
{
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    int k = keys[p];
    int slot = offsets[k] + atomicAdd(fill + k, 1);
    cell_sorted[slot] = (int32_t)p;
}

// order of two particles inside a cell: by index (stable sort), or, in the
// canonical order of the deterministic mode, by position (the bit patterns
// of x, y, z, which order non-negative floats like their values) with the
// index only between particles at the same position
template <int D>
__device__ __forceinline__ bool cell_before(int32_t a, int32_t b, const float *x, int64_t n,
                                            bool canonical)
{
    if (canonical) {
#pragma unroll
        for (int k = 0; k < D; ++k) {
            const uint32_t ua = __float_as_uint(x[k * n + a]), ub = __float_as_uint(x[k * n + b]);
            if (ua != ub) return ua < ub;
        }
    }
    return a < b;
}

// insertion sort of each cell segment (restores the previous order among
// particles of one cell, or puts them in canonical order)
template <int D>
__global__ void cell_segment_sort_kernel(const int32_t *offsets, const int32_t *counts,
                                         int64_t ncells, int32_t *cell_sorted, const float *x,
                                         int64_t n, int canonical)
{
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncells) return;
    int s = offsets[c], len = counts[c];
    // cells hold a few tens of particles; a pathological pile-up (or the
    // overflow bucket of flagged particles) keeps its arrival order rather
    // than paying a quadratic sort in one thread
    if (len > 1024 || len < 2) return;
    if (!canonical && len <= 32) {
        // the common case: sort by index in registers (one load and one
        // store per element instead of a dependent chain of global accesses)
        int buf[32];
#pragma unroll
        for (int i = 0; i < 32; ++i)
            if (i < len) buf[i] = cell_sorted[s + i];
        for (int i = 1; i < len; ++i) {
            const int v = buf[i];
            int j = i - 1;
            while (j >= 0 && v < buf[j]) {
                buf[j + 1] = buf[j];
                --j;
            }
            buf[j + 1] = v;
        }
#pragma unroll
        for (int i = 0; i < 32; ++i)
            if (i < len) cell_sorted[s + i] = buf[i];
        return;
    }
    for (int i = 1; i < len; ++i) {
        int v = cell_sorted[s + i];
        int j = i - 1;
        while (j >= 0 && cell_before<D>(v, cell_sorted[s + j], x, n, canonical != 0)) {
            cell_sorted[s + j + 1] = cell_sorted[s + j];
            --j;
        }
        cell_sorted[s + j + 1] = v;
    }
}

// slot-major order inside a tile: the particle of rank k in local cell c goes
// to tile_start + sum_c' min(cnt[c'], k) + #{c' < c : cnt[c'] > k}.  One wave
// per tile, lane = local cell: for each rank k the cells holding a k-th
// particle are one ballot, whose population count is that slot's length and
// whose count below the lane is the cell's place in it.
template <int D>
__global__ void __launch_bounds__(64) tile_slot_kernel(const int32_t *offsets,
                                                       const int32_t *counts,
                                                       const int32_t *cell_sorted,
                                                       int32_t *perm, int64_t ntiles)
{
    static_assert(Tiling<D>::CELLS == 64, "one lane per local cell");
    const int64_t t = blockIdx.x;
    if (t >= ntiles) return;
    const int c = threadIdx.x;
    const int64_t cell = t * 64 + c;
    const int my_cnt = counts[cell];
    const int my_off = offsets[cell];
    int64_t pos0 = offsets[t * 64];                 // start of the tile's particles
    const uint64_t below = c == 0 ? 0ull : (~0ull >> (64 - c));
    for (int k = 0;; ++k) {
        const uint64_t has = __ballot(k < my_cnt);
        if (has == 0) break;
        if (k < my_cnt) perm[pos0 + __popcll(has & below)] = cell_sorted[my_off + k];
        pos0 += __popcll(has);
    }
}

// overflow bucket (particles outside the lattice): keep their order at the end
__global__ void tail_copy_kernel(const int32_t *cell_sorted, int32_t *perm, const int32_t *start,
                                 int64_t n)
{
    int64_t i = (int64_t)(*start) + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) perm[i] = cell_sorted[i];
}

__global__ void gather_plane_kernel(const float *__restrict__ src, float *__restrict__ dst,
                                    const int32_t *__restrict__ perm, int64_t n, int planes)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int64_t q = perm[i];
    // source and destination never overlap (a separate set or the copy
    // buffer), so the loads of all planes can be in flight together
    int k = 0;
    for (; k + 3 < planes; k += 4) {
        const float a0 = src[k * n + q], a1 = src[(k + 1) * n + q];
        const float a2 = src[(k + 2) * n + q], a3 = src[(k + 3) * n + q];
        dst[k * n + i] = a0;
        dst[(k + 1) * n + i] = a1;
        dst[(k + 2) * n + i] = a2;
        dst[(k + 3) * n + i] = a3;
    }
    for (; k < planes; ++k) dst[k * n + i] = src[k * n + q];
}

// ---------------------------------------------------------------------------
// sorted P2G: one wave per tile, one lane per home cell
//
// The cell sort orders each tile's particles slot-major: the first particle
// of every cell of the tile (in cell order), then the second ones, ...  A
// wave owns one tile and lane c owns local cell c: at rank k the active lanes
// (cells with more than k particles) read consecutive particles, so the loads
// are coalesced, and their stencil bases are distinct, so for any one stencil
// offset the 64 lanes touch 64 distinct nodes.  The wave accumulates into a
// private LDS copy of the tile's node region with plain float4
// read-modify-write (LDS float atomics are far slower on this part); the
// accesses of one wave are kept in program order by a compiler barrier after
// every node, which the in-order LDS pipeline then preserves across lanes.
// Particles that drifted out of their sort-time cell may share a base cell
// with another lane.  The sorted P2G defers them to a per-tile index list
// and scatters them after the slots, 64 at a time, with lanes claiming
// their base cell in an owner table and the losers retrying in a later
// round; the fused kernel (and a full list) claims inside the slot.  A
// particle whose stencil left the region entirely goes to HBM atomics.
// Region rows are unpadded in 3D (8 float4) and padded to 24 in 2D.

// tiles (one wave each) per workgroup of the tile kernels
#ifndef MR_TILE_WPB
#define MR_TILE_WPB 1
#endif
#ifndef MR_TILE_PREFETCH
#define MR_TILE_PREFETCH 0
#endif
// per-node ordering of the scatter arithmetic and row-wise G2P gathering:
// fewer live registers in exchange for less instruction-level overlap
#ifndef MR_TILE_ORDERED
#define MR_TILE_ORDERED 0
#endif

template <int D>
struct CellTile {
    static constexpr int TS = Tiling<D>::TS;        // cells per tile edge
    static constexpr int R = TS + 4;                // region nodes per edge
    static constexpr int RC = TS + 2;               // region cells per edge
    static constexpr int SY = (D == 3) ? R : 24;    // row stride (float4; 2D rows padded)
    static constexpr int SZ = (D == 3) ? SY * R : 0;
    static constexpr int RNP = (D == 3) ? SZ * R : SY * R;
    static constexpr int RCN = (D == 3) ? RC * RC * RC : RC * RC;
    static constexpr int WPB = MR_TILE_WPB;         // waves (tiles) per workgroup
};

__device__ __forceinline__ void lds_order() { asm volatile("" ::: "memory"); }

// Adds a 3D tile's LDS region (8 x 8 x 8 nodes from grid node (r0, r1, r2))
// to the grid with one atomic per non-zero node channel.  Lane l takes
// channel l % 4 of the nodes with x index l / 4 % 8 in rows l / 32 + 2 j of
// every z layer, so one atomic instruction covers 16 nodes: two rows of 8
// nodes, two contiguous 128-byte stretches of the grid.  (With a node per
// lane an instruction touched eight stretches, and the kernel wrote four
// times the bytes back to HBM: 69 vs 17 MB per launch on the 2.1M-particle
// scene, measured.)
__device__ __forceinline__ void flush_region_3d(const float4 *acc, int r0, int r1, int r2,
                                                const GridK &g, float *grid_out, int lane)
{
    using CT = CellTile<3>;
    static_assert(CT::R == 8, "flush mapping assumes 8-node region rows");
    const float *accf = reinterpret_cast<const float *>(acc);
    const int c = lane & 3, i0 = (lane >> 2) & 7, j0 = lane >> 5;
    const int gi = r0 + i0;
    if (gi < 0 || gi >= g.n0) return;
    for (int i2 = 0; i2 < CT::R; ++i2) {
        const int gk = r2 + i2;
        if (gk < 0 || gk >= g.n2) continue;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int i1 = j0 + 2 * j, gj = r1 + i1;
            const int slot = i0 + CT::SY * i1 + CT::SZ * i2;
            if (gj < 0 || gj >= g.n1 || accf[4 * slot] == 0.0f) continue;   // massless: skip
            atomicAdd(grid_out + 4 * node_lin(g, gi, gj, gk) + c, accf[4 * slot + c]);
        }
    }
}

// an empty asm that claims to modify the stencil and payload values (stops
// the compiler from hoisting what is computed from them out of a loop)
template <int D>
__device__ __forceinline__ void opaque_payload(Stencil<D> &st, P2GPayload<D> &pl)
{
#pragma unroll
    for (int a = 0; a < D; ++a) {
        asm volatile("" : "+v"(st.f[a]));
#pragma unroll
        for (int o = 0; o < 3; ++o) asm volatile("" : "+v"(st.w[a][o]), "+v"(st.dw[a][o]));
        asm volatile("" : "+v"(pl.mv[a]));
    }
    asm volatile("" : "+v"(pl.m));
#pragma unroll
    for (int q = 0; q < D * D; ++q) asm volatile("" : "+v"(pl.mC[q]), "+v"(pl.S[q]));
}

// waves per SIMD the tile kernels are compiled for (bounds their registers)
#ifndef MR_TILE_MIN_WAVES
#define MR_TILE_MIN_WAVES 1
#endif

// DET (sorted P2G, deterministic mode): base cells are claimed by the lowest
// lane (LDS atomic min), a particle whose stencil left the region raises
// MR_FLAG_DRIFT instead of scattering with atomics, and the region is stored
// whole to the tile's staging area (summed per node in tile order by
// det_combine_kernel) instead of being flushed with atomics.
// Workgroups are dispatched round-robin over the 8 XCDs, each with its own
// L2: block b runs on XCD b % 8.  In 3D with one tile per workgroup the 8
// tiles of a 2 x 2 x 2 brick run on one XCD, so the halo nodes they share
// are fetched into, and flushed from, one L2; consecutive bricks go to
// consecutive XCDs, which spreads the occupied tiles evenly.  Blocks b =
// 64 j + 8 w + x take tile w of brick 8 j + x (a bijection onto the
// bricks rounded up to a multiple of 8; tiles past the lattice get -1).
constexpr int XCDS = 8;

template <int D>
inline unsigned tile_blocks(const TileGeom &tg)
{
    if (D == 3 && MR_TILE_WPB == 1) {
        const int64_t nb = (int64_t)((tg.nt0 + 1) / 2) * ((tg.nt1 + 1) / 2) * ((tg.nt2 + 1) / 2);
        return (unsigned)(64 * ceil_div(nb, (int64_t)XCDS));
    }
    return (unsigned)ceil_div(tg.ntiles, (int64_t)MR_TILE_WPB);
}

template <int D>
__device__ __forceinline__ int64_t tile_of_block(const TileGeom &tg, int wave)
{
    if constexpr (D == 3 && MR_TILE_WPB == 1) {
        const int64_t b = blockIdx.x;
        const int64_t k = b / XCDS;
        const int w = (int)(k & 7);
        const int64_t brick = (k >> 3) * XCDS + (b % XCDS);
        const int nb0 = (tg.nt0 + 1) / 2, nb1 = (tg.nt1 + 1) / 2;
        const int t0 = 2 * (int)(brick % nb0) + (w & 1);
        const int t1 = 2 * (int)((brick / nb0) % nb1) + ((w >> 1) & 1);
        const int64_t t2 = 2 * (brick / ((int64_t)nb0 * nb1)) + (w >> 2);
        if (t0 >= tg.nt0 || t1 >= tg.nt1 || t2 >= tg.nt2) return -1;
        return t0 + (int64_t)tg.nt0 * (t1 + (int64_t)tg.nt1 * t2);
    } else {
        return (int64_t)blockIdx.x * MR_TILE_WPB + wave;
    }
}

template <int D, bool FUSED, bool DET = false>
__global__ void __launch_bounds__(64 * MR_TILE_WPB, MR_TILE_MIN_WAVES) tile_scatter_kernel(
    GridK g, TileGeom tg, float *x, float *v, float *C, float *F, const float *m, const float *V0,
    float m_u, float V0_u, int64_t n, const int32_t *offsets, const int32_t *counts, int apic,
    int model, float mu, float la, float dt, const float *grid_in, float *grid_out, float *v_out,
    float *C_out, int32_t *flag, float4 *stage = nullptr)
{
    using CT = CellTile<D>;
    // sorted P2G: particles that drifted out of their sort-time cell are
    // deferred to the end of the tile (index list), so the slots themselves
    // never need base-cell claims
    constexpr bool DEFER = !FUSED && !DET;
    constexpr int DEFER_CAP = DEFER ? 512 : 1;
    __shared__ float4 acc_all[CT::WPB][CT::RNP];
    __shared__ int owner_all[CT::WPB][CT::RCN];
    __shared__ int32_t defer_all[CT::WPB][DEFER_CAP];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    float4 *acc = acc_all[wave];
    int *owner = owner_all[wave];
    int32_t *deferred = defer_all[wave];
    int ndef = 0;                                   // wave-uniform
    const int64_t t = tile_of_block<D>(tg, wave);
    if (t < 0 || t >= tg.ntiles) return;           // wave-uniform; no block barriers below
    const int64_t c0 = offsets[t * Tiling<D>::CELLS];
    const int64_t c1 = offsets[(t + 1) * Tiling<D>::CELLS];
    if (c0 == c1) return;
    for (int i = lane; i < CT::RNP; i += 64) acc[i] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    lds_order();
    const int tt0 = (int)(t % tg.nt0);
    const int tt1 = (int)((t / tg.nt0) % tg.nt1);
    const int tt2 = D == 3 ? (int)(t / ((int64_t)tg.nt0 * tg.nt1)) : 0;
    const int r0 = tt0 * CT::TS - 1, r1 = tt1 * CT::TS - 1, r2 = D == 3 ? tt2 * CT::TS - 1 : 0;
    // home cell of this lane, relative to the region origin
    const int h0 = lane % CT::TS + 1;
    const int h1 = (lane / CT::TS) % CT::TS + 1;
    const int h2 = D == 3 ? lane / (CT::TS * CT::TS) + 1 : 0;
    const int cnt = counts[t * Tiling<D>::CELLS + lane];
    const float cscale = apic ? 4.0f * g.inv_dx * g.inv_dx : 0.0f;
    const float4 *gin4 = reinterpret_cast<const float4 *>(grid_in);
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    int64_t base = c0;
    // fused: the next slot's x and F are loaded while the current slot is
    // processed (slot k + 1 of a lane exists iff k + 1 < cnt, so its index is
    // known one slot ahead)
    float pre_x[FUSED && MR_TILE_PREFETCH ? D : 1], pre_F[FUSED && MR_TILE_PREFETCH ? D * D : 1];
    if (FUSED && MR_TILE_PREFETCH) {
        const uint64_t m0k = __ballot(0 < cnt);
        if (0 < cnt) {
            const int64_t p0 = base + __popcll(m0k & below);
#pragma unroll
            for (int a = 0; a < D; ++a) pre_x[a] = x[a * n + p0];
#pragma unroll
            for (int q = 0; q < D * D; ++q) pre_F[q] = F[q * n + p0];
        }
    }
    for (int k = 0;; ++k) {
        const bool act = k < cnt;
        const uint64_t mask = __ballot(act);
        if (mask == 0) break;
        const int64_t p = base + __popcll(mask & below);
        base += __popcll(mask);
        float cur_x[FUSED && MR_TILE_PREFETCH ? D : 1], cur_F[FUSED && MR_TILE_PREFETCH ? D * D : 1];
        if (FUSED && MR_TILE_PREFETCH) {
#pragma unroll
            for (int a = 0; a < D; ++a) cur_x[a] = pre_x[a];
#pragma unroll
            for (int q = 0; q < D * D; ++q) cur_F[q] = pre_F[q];
            const bool act1 = k + 1 < cnt;
            const uint64_t mask1 = __ballot(act1);
            if (act1) {
                const int64_t p1 = base + __popcll(mask1 & below);
#pragma unroll
                for (int a = 0; a < D; ++a) pre_x[a] = x[a * n + p1];
#pragma unroll
                for (int q = 0; q < D * D; ++q) pre_F[q] = F[q * n + p1];
            }
        }
        bool scat = false, inreg = false;
        Stencil<D> sn;
        P2GPayload<D> pl;
        int m0 = 0, m1 = 0, m2 = 0;
        if (act) {
            float xn[D], vp[D], Cp[D * D], Fn[D * D];
            bool ok = true;
            if (FUSED) {
                float xp[D], Fp[D * D];
                if (MR_TILE_PREFETCH) {
#pragma unroll
                    for (int a = 0; a < D; ++a) xp[a] = cur_x[a];
#pragma unroll
                    for (int q = 0; q < D * D; ++q) Fp[q] = cur_F[q];
                } else {
#pragma unroll
                    for (int a = 0; a < D; ++a) xp[a] = x[a * n + p];
#pragma unroll
                    for (int q = 0; q < D * D; ++q) Fp[q] = F[q * n + p];
                }
                Stencil<D> so;
                ok = make_stencil<D>(g, xp, so);
                if (ok) {
                    float Bp[D * D], gv[D * D];
                    auto fetch = [&](int o0, int o1, int o2) {
                        return gin4[node_lin(g, so.base[0] + o0, so.base[1] + o1,
                                             D == 3 ? so.base[2] + o2 : 0)];
                    };
                    g2p_separable<D, decltype(fetch) &, MR_TILE_ORDERED != 0>(g, so, fetch, vp, Bp,
                                                                             gv);
                    mr::update_F<D>(gv, Fp, dt, Fn);
#pragma unroll
                    for (int q = 0; q < D * D; ++q) Cp[q] = cscale * Bp[q];
#pragma unroll
                    for (int a = 0; a < D; ++a) xn[a] = xp[a] + dt * vp[a];
#pragma unroll
                    for (int a = 0; a < D; ++a) x[a * n + p] = xn[a];
#pragma unroll
                    for (int q = 0; q < D * D; ++q) F[q * n + p] = Fn[q];
                    if (v_out)
#pragma unroll
                        for (int a = 0; a < D; ++a) v_out[a * n + p] = vp[a];
                    if (C_out)
#pragma unroll
                        for (int q = 0; q < D * D; ++q) C_out[q * n + p] = Cp[q];
                }
            } else {
#pragma unroll
                for (int a = 0; a < D; ++a) {
                    xn[a] = x[a * n + p];
                    vp[a] = v[a * n + p];
                }
#pragma unroll
                for (int q = 0; q < D * D; ++q) {
                    Fn[q] = F[q * n + p];
                    Cp[q] = apic ? C[q * n + p] : 0.0f;
                }
            }
            float tau[D * D];
            if (ok) {
                ok = make_stencil<D>(g, xn, sn);
                ok = kirchhoff<D>(model, mu, la, Fn, tau) && ok;
            }
            if (!ok) {
                raise_flag(flag, MR_FLAG_DOMAIN);
            } else {
                const float mp = m ? m[p] : m_u;
                const float sc = dt * (V0 ? V0[p] : V0_u);
                pl.m = mp;
#pragma unroll
                for (int a = 0; a < D; ++a) pl.mv[a] = mp * vp[a];
#pragma unroll
                for (int q = 0; q < D * D; ++q) {
                    pl.mC[q] = mp * Cp[q];
                    pl.S[q] = sc * tau[q];
                }
                scat = true;
                m0 = sn.base[0] - r0;
                m1 = sn.base[1] - r1;
                m2 = D == 3 ? sn.base[2] - r2 : 0;
                inreg = m0 >= 0 && m0 < CT::RC && m1 >= 0 && m1 < CT::RC &&
                        (D == 2 || (m2 >= 0 && m2 < CT::RC));
                if (!inreg) {
                    if (DET)
                        raise_flag(flag, MR_FLAG_DRIFT);
                    else
                        scatter_global<D>(g, sn, pl, grid_out);
                }
            }
        }
        bool pending = scat && inreg;
        bool drifted = pending && (m0 != h0 || m1 != h1 || (D == 3 && m2 != h2));
        if (DEFER) {
            const uint64_t dm = __ballot(drifted);
            const int nd = __popcll(dm);
            if (nd != 0 && ndef + nd <= DEFER_CAP) {
                if (drifted) deferred[ndef + __popcll(dm & below)] = (int32_t)p;
                ndef += nd;
                pending = pending && !drifted;
                drifted = false;
            }
        }
        const bool any_drift = __ballot(drifted) != 0;
        const int key = m0 + CT::RC * (m1 + (D == 3 ? CT::RC * m2 : 0));
        const int nb = m0 + CT::SY * m1 + (D == 3 ? CT::SZ * m2 : 0);
        while (__ballot(pending) != 0) {
            bool go = pending;
            if (any_drift) {
                if (DET) {
                    if (pending) owner[key] = 64;
                    lds_order();
                    if (pending) atomicMin(owner + key, lane);
                } else if (pending) {
                    owner[key] = lane;
                }
                lds_order();
                go = pending && owner[key] == lane;
                lds_order();
            }
            if (go) {
                // sorted P2G: keep the node contributions inside the round
                // (computed node by node next to their updates) rather than
                // hoisted out of the retry loop and held in registers
                // (measured: faster there, no gain in the fused kernel)
                if (!FUSED) opaque_payload<D>(sn, pl);
                auto rmw = [&](int o0, int o1, int o2, float mw, float q0, float q1, float q2) {
                    float4 *a4 = acc + nb + o0 + CT::SY * o1 + (D == 3 ? CT::SZ * o2 : 0);
                    float4 q = *a4;
                    q.x += mw;
                    q.y += q0;
                    q.z += q1;
                    q.w += q2;
                    *a4 = q;
                    lds_order();
                };
                p2g_separable<D, decltype(rmw) &, MR_TILE_ORDERED != 0>(g, sn, pl, rmw);
                pending = false;
            }
        }
    }
    if (DEFER && ndef > 0) {
        // the deferred particles, 64 at a time: reload, form the payload
        // again and scatter in claim rounds (lanes sharing a base cell go
        // in turn; any two distinct base cells touch distinct nodes per
        // stencil offset)
        lds_order();
        for (int i0 = 0; i0 < ndef; i0 += 64) {
            bool pending = false;
            Stencil<D> sn;
            P2GPayload<D> pl;
            int key = 0, nb = 0;
            if (i0 + lane < ndef) {
                const int64_t p = deferred[i0 + lane];
                float xn[D], vp[D], Cp[D * D], Fn[D * D], tau[D * D];
#pragma unroll
                for (int a = 0; a < D; ++a) {
                    xn[a] = x[a * n + p];
                    vp[a] = v[a * n + p];
                }
#pragma unroll
                for (int q = 0; q < D * D; ++q) {
                    Fn[q] = F[q * n + p];
                    Cp[q] = apic ? C[q * n + p] : 0.0f;
                }
                // both succeeded when the particle was deferred
                make_stencil<D>(g, xn, sn);
                kirchhoff<D>(model, mu, la, Fn, tau);
                const float mp = m ? m[p] : m_u;
                const float sc = dt * (V0 ? V0[p] : V0_u);
                pl.m = mp;
#pragma unroll
                for (int a = 0; a < D; ++a) pl.mv[a] = mp * vp[a];
#pragma unroll
                for (int q = 0; q < D * D; ++q) {
                    pl.mC[q] = mp * Cp[q];
                    pl.S[q] = sc * tau[q];
                }
                const int m0 = sn.base[0] - r0, m1 = sn.base[1] - r1;
                const int m2 = D == 3 ? sn.base[2] - r2 : 0;
                key = m0 + CT::RC * (m1 + (D == 3 ? CT::RC * m2 : 0));
                nb = m0 + CT::SY * m1 + (D == 3 ? CT::SZ * m2 : 0);
                pending = true;
            }
            while (__ballot(pending) != 0) {
                if (pending) owner[key] = lane;
                lds_order();
                const bool go = pending && owner[key] == lane;
                lds_order();
                if (go) {
                    opaque_payload<D>(sn, pl);
                    auto rmw = [&](int o0, int o1, int o2, float mw, float q0, float q1, float q2) {
                        float4 *a4 = acc + nb + o0 + CT::SY * o1 + (D == 3 ? CT::SZ * o2 : 0);
                        float4 q = *a4;
                        q.x += mw;
                        q.y += q0;
                        q.z += q1;
                        q.w += q2;
                        *a4 = q;
                        lds_order();
                    };
                    p2g_separable<D, decltype(rmw) &, MR_TILE_ORDERED != 0>(g, sn, pl, rmw);
                    pending = false;
                }
            }
        }
    }
    lds_order();
    constexpr int RN = (D == 3) ? CT::R * CT::R * CT::R : CT::R * CT::R;
    if (DET) {
        // the whole region, zeros included, in region order
        float4 *dst = stage + t * RN;
        for (int li = lane; li < RN; li += 64) {
            const int i0 = li % CT::R, i1 = (li / CT::R) % CT::R, i2 = D == 3 ? li / (CT::R * CT::R) : 0;
            dst[li] = acc[i0 + CT::SY * i1 + (D == 3 ? CT::SZ * i2 : 0)];
        }
        return;
    }
    // flush the region: one global atomic per non-zero node channel
    if constexpr (D == 3) {
        flush_region_3d(acc, r0, r1, r2, g, grid_out, lane);
        return;
    }
    for (int li = lane; li < RN; li += 64) {
        const int i0 = li % CT::R, i1 = (li / CT::R) % CT::R, i2 = D == 3 ? li / (CT::R * CT::R) : 0;
        const float4 q = acc[i0 + CT::SY * i1 + (D == 3 ? CT::SZ * i2 : 0)];
        if (q.x == 0.0f) continue;
        const int gi = r0 + i0, gj = r1 + i1, gk = D == 3 ? r2 + i2 : 0;
        if (gi < 0 || gj < 0 || gk < 0 || gi >= g.n0 || gj >= g.n1 || gk >= g.n2) continue;
        float *gp = grid_out + 4 * node_lin(g, gi, gj, gk);
        atomicAdd(gp, q.x);
        atomicAdd(gp + 1, q.y);
        atomicAdd(gp + 2, q.z);
        if (D == 3) atomicAdd(gp + 3, q.w);
    }
}

// ---------------------------------------------------------------------------
// sorted P2G in 3D: per-cell sums in registers
//
// One wave per 4 x 4 x 4 tile, lane c = local cell c, as in the tile scatter
// above.  Every particle whose stencil base is still its sort-time (home)
// cell is summed into the lane's registers instead of into LDS node by node.
// A particle's contribution to stencil node o is, with the 1D weights w_b,
// their derivatives dw_b (per unit length) and u_b = w_b (o_b - f_b) dx,
//   mass   m w0 w1 w2
//   mom_a  w1 w2 Px_a[o0] + w0 (w2 Qy_a[o1] + w1 Rz_a[o2]),
//   Px_a = mv_a w0 + mC_a0 u0 - S_a0 dw0,  Qy_a = mC_a1 u1 - S_a1 dw1,
//   Rz_a = mC_a2 u2 - S_a2 dw2          (S = dt V0 tau),
// i.e. w (mv + mC (x_i - x_p)) - S grad w expanded per axis: one fused
// multiply-add per node for the mass, two per momentum channel.  The two
// lower z layers of the stencil (18 nodes x 4 channels) stay in registers
// over all of the lane's particles; the top layer (9 nodes) is added to the
// tile's LDS region particle by particle (ordered read-modify-write: lanes
// sit in distinct cells, so one instruction touches 64 distinct nodes) --
// all 27 in registers would not fit the register budget.  The kernel runs
// three waves per SIMD, which hides the loads of a slot behind the other
// waves' sums better than loading one slot ahead at two waves per SIMD did;
// a slot loads x and F first and v and C only after the stress, for the
// particles summed here, so that no more than 168 VGPRs are live (162-165,
// no spills: 117 vs 136 us on the 2.1M-particle scene; with spilled
// registers the scratch traffic also slowed the gather that follows).
// After the slots the lane adds its register sums to the region once;
// particles that left their home cell since the sort, and those of a cell
// beyond the tile's slot cap (its mean count per occupied cell, rounded
// up), are deferred (the first DEFER_CAP in LDS, the rest in the tile's own
// range of a spill array) and scattered into the region afterwards in claim
// rounds (those beyond the region with global atomics); the region is
// flushed with one atomic per non-zero node channel.  MODEL is the constitutive law (compiled separately, so that each
// law's registers are allocated on their own); PER_PARTICLE selects
// per-particle masses and volumes.  Cl is C, or any 9-plane array when the
// affine term is off (then scaled by 0), so the loads need no branch.
template <int MODEL, bool PER_PARTICLE>
__global__ void __launch_bounds__(64, 3) cell_sum_p2g_kernel(
    GridK g, TileGeom tg, const float *__restrict__ x, const float *__restrict__ v,
    const float *__restrict__ Cl, const float *__restrict__ F, const float *__restrict__ m,
    const float *__restrict__ V0, float m_u, float V0_u, int64_t n,
    const int32_t *__restrict__ offsets, const int32_t *__restrict__ counts, int apic, float mu,
    float la, float dt, float *grid_out, int32_t *spill, int32_t *flag)
{
    using CT = CellTile<3>;
    constexpr int DEFER_CAP = 512;                  // the rest spills
    __shared__ float4 acc[CT::RNP];
    __shared__ int owner[CT::RCN];
    __shared__ int32_t deferred[DEFER_CAP];
    const int lane = threadIdx.x;
    const int64_t t = tile_of_block<3>(tg, 0);
    if (t < 0 || t >= tg.ntiles) return;           // wave-uniform; no barriers below
    const int64_t c0 = offsets[t * Tiling<3>::CELLS];
    const int64_t c1 = offsets[(t + 1) * Tiling<3>::CELLS];
    if (c0 == c1) return;
    for (int i = lane; i < CT::RNP; i += 64) acc[i] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    lds_order();
    const int tt0 = (int)(t % tg.nt0);
    const int tt1 = (int)((t / tg.nt0) % tg.nt1);
    const int tt2 = (int)(t / ((int64_t)tg.nt0 * tg.nt1));
    const int r0 = tt0 * CT::TS - 1, r1 = tt1 * CT::TS - 1, r2 = tt2 * CT::TS - 1;
    const int h0 = lane % CT::TS + 1, h1 = (lane / CT::TS) % CT::TS + 1, h2 = lane / 16 + 1;
    const int cnt = counts[t * Tiling<3>::CELLS + lane];
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    // slots summed in registers: the tile's mean count per occupied cell,
    // rounded up, plus a slack; a cell's particles beyond it take the
    // deferred way, so a few crowded cells do not keep the whole wave in
    // slots where most lanes have nothing left.  The slack trades idle
    // lanes in the last slots against the dearer claim rounds, and the
    // stress sets the balance (2.1M-particle scene, 1,000 steps): with the
    // Neo-Hookean law slack 0 / 1 / 2 gave 118.6 / 116.7 / 118.0 us against
    // 120.9 us with no cap; with the fixed-corotated law's eigen-solve per
    // particle 178.2 / 182.1 / 188.8 against 196.9 us.
    constexpr int SLACK = MODEL == MR_FIXED_COROTATED ? 0 : 1;
    const int occ = __popcll(__ballot(cnt > 0));    // >= 1: c1 > c0
    const int cap = (int)((c1 - c0 + occ - 1) / occ) + SLACK;
    const float cscale = apic ? 1.0f : 0.0f;
    const int nb = h0 + CT::SY * h1 + CT::SZ * h2;  // the home stencil's base node
    float4 *top = acc + nb + 2 * CT::SZ;            // its top layer

    float sum[18][4];
#pragma unroll
    for (int q = 0; q < 18; ++q)
#pragma unroll
        for (int c = 0; c < 4; ++c) sum[q][c] = 0.0f;
    int ndef = 0;                                   // wave-uniform

    int64_t base = c0;
    uint64_t mask = __ballot(0 < cnt);
    for (int k = 0; mask != 0; ++k) {
        const bool act = k < cnt && k < cap;
        const int64_t p = base + __popcll(mask & below);
        float xp[3], Fp[9];
        float mp = m_u, Vp = V0_u;
        if (act) {
#pragma unroll
            for (int a = 0; a < 3; ++a) xp[a] = x[a * n + p];
#pragma unroll
            for (int q = 0; q < 9; ++q) Fp[q] = F[q * n + p];
            if (PER_PARTICLE) {
                mp = m[p];
                Vp = V0[p];
            }
        }
        base += __popcll(mask);
        const uint64_t mask1 = __ballot(k + 1 < cnt);
        bool drifted = k < cnt && k >= cap;             // beyond the cap
        if (act) {
            float w[3][3], dw[3][3], f[3];
            int b[3];
            bool ok = true;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const int na = a == 0 ? g.n0 : (a == 1 ? g.n1 : g.n2);
                b[a] = bspline(xp[a], g.inv_dx, na, w[a], dw[a], ok);
                f[a] = xp[a] * g.inv_dx - (float)b[a];
            }
            float tau[9];
            ok = kirchhoff<3>(MODEL, mu, la, Fp, tau) && ok;
            if (!ok) {
                raise_flag(flag, MR_FLAG_DOMAIN);
            } else if (b[0] - r0 == h0 && b[1] - r1 == h1 && b[2] - r2 == h2) {
                // v and C only for the particles summed here (the deferred
                // ones read theirs when they are scattered), and only once
                // the stress is done: fewer registers live across it
                float vp[3], Cp[9];
#pragma unroll
                for (int a = 0; a < 3; ++a) vp[a] = v[a * n + p];
#pragma unroll
                for (int q = 0; q < 9; ++q) Cp[q] = Cl[q * n + p];
                const float sc = dt * Vp;
                float P[3][3], Q[3][3], R[3][3];   // [a][o]
#pragma unroll
                for (int o = 0; o < 3; ++o) {
                    const float u0 = w[0][o] * (((float)o - f[0]) * g.dx);
                    const float u1 = w[1][o] * (((float)o - f[1]) * g.dx);
                    const float u2 = w[2][o] * (((float)o - f[2]) * g.dx);
#pragma unroll
                    for (int a = 0; a < 3; ++a) {
                        const float mca0 = cscale * mp * Cp[3 * a + 0];
                        const float mca1 = cscale * mp * Cp[3 * a + 1];
                        const float mca2 = cscale * mp * Cp[3 * a + 2];
                        P[a][o] = (mp * vp[a]) * w[0][o] + mca0 * u0 - (sc * tau[3 * a + 0]) * dw[0][o];
                        Q[a][o] = mca1 * u1 - (sc * tau[3 * a + 1]) * dw[1][o];
                        R[a][o] = mca2 * u2 - (sc * tau[3 * a + 2]) * dw[2][o];
                    }
                }
#pragma unroll
                for (int o2 = 0; o2 < 3; ++o2)
#pragma unroll
                    for (int o1 = 0; o1 < 3; ++o1) {
                        const float wyz = w[1][o1] * w[2][o2];
                        const float mwyz = mp * wyz;
                        float T[3];
#pragma unroll
                        for (int a = 0; a < 3; ++a) T[a] = Q[a][o1] * w[2][o2] + w[1][o1] * R[a][o2];
#pragma unroll
                        for (int o0 = 0; o0 < 3; ++o0) {
                            if (o2 < 2) {
                                float *s4 = sum[o0 + 3 * o1 + 9 * o2];
                                s4[0] = fmaf(mwyz, w[0][o0], s4[0]);
#pragma unroll
                                for (int a = 0; a < 3; ++a)
                                    s4[1 + a] = fmaf(w[0][o0], T[a], fmaf(P[a][o0], wyz, s4[1 + a]));
                            } else {
                                float4 *a4 = top + o0 + CT::SY * o1;
                                float4 q = *a4;
                                q.x = fmaf(mwyz, w[0][o0], q.x);
                                q.y = fmaf(w[0][o0], T[0], fmaf(P[0][o0], wyz, q.y));
                                q.z = fmaf(w[0][o0], T[1], fmaf(P[1][o0], wyz, q.z));
                                q.w = fmaf(w[0][o0], T[2], fmaf(P[2][o0], wyz, q.w));
                                *a4 = q;
                                lds_order();
                            }
                        }
                    }
            } else {
                drifted = true;
            }
        }
        // particles that left their home cell (or lie beyond the cap) wait
        // for the claim rounds after the slots (each is deferred once, so a
        // tile never defers more than its c1 - c0 particles)
        const uint64_t dm = __ballot(drifted);
        if (dm != 0) {
            if (drifted) {
                const int i = ndef + __popcll(dm & below);
                if (i < DEFER_CAP)
                    deferred[i] = (int32_t)p;
                else
                    spill[c0 + i - DEFER_CAP] = (int32_t)p;
            }
            ndef += __popcll(dm);
        }
        mask = mask1;
    }
    // the lanes' register sums (the two lower layers) into the region, in
    // program order after the top-layer updates
    lds_order();
    if (cnt > 0) {
#pragma unroll
        for (int o2 = 0; o2 < 2; ++o2)
#pragma unroll
            for (int o1 = 0; o1 < 3; ++o1)
#pragma unroll
                for (int o0 = 0; o0 < 3; ++o0) {
                    const float *s4 = sum[o0 + 3 * o1 + 9 * o2];
                    float4 *a4 = acc + nb + o0 + CT::SY * o1 + CT::SZ * o2;
                    float4 q = *a4;
                    q.x += s4[0];
                    q.y += s4[1];
                    q.z += s4[2];
                    q.w += s4[3];
                    *a4 = q;
                    lds_order();
                }
    }
    if (ndef > 0) {
        // the spilled indices were stored by this wave: complete and make its
        // stores visible before reading them back
        if (ndef > DEFER_CAP) __threadfence();
        // the deferred particles, 64 at a time: lanes sharing a base cell go
        // in turn (any two distinct base cells touch distinct nodes per
        // stencil offset)
        for (int i0 = 0; i0 < ndef; i0 += 64) {
            bool pending = false;
            Stencil<3> sn;
            P2GPayload<3> pl;
            int key = 0, nbd = 0;
            if (i0 + lane < ndef) {
                const int i = i0 + lane;
                const int64_t p = i < DEFER_CAP ? deferred[i] : spill[c0 + i - DEFER_CAP];
                float xn[3], vq[3], Cq[9], Fq[9], tau[9];
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    xn[a] = x[a * n + p];
                    vq[a] = v[a * n + p];
                }
#pragma unroll
                for (int q = 0; q < 9; ++q) {
                    Fq[q] = F[q * n + p];
                    Cq[q] = Cl[q * n + p];
                }
                // a drifted particle passed both checks in its slot; one
                // beyond the cap meets them here first
                const bool ok = make_stencil<3>(g, xn, sn) && kirchhoff<3>(MODEL, mu, la, Fq, tau);
                const float mp = PER_PARTICLE ? m[p] : m_u;
                const float sc = dt * (PER_PARTICLE ? V0[p] : V0_u);
                pl.m = mp;
#pragma unroll
                for (int a = 0; a < 3; ++a) pl.mv[a] = mp * vq[a];
#pragma unroll
                for (int q = 0; q < 9; ++q) {
                    pl.mC[q] = cscale * mp * Cq[q];
                    pl.S[q] = sc * tau[q];
                }
                const int m0 = sn.base[0] - r0, m1 = sn.base[1] - r1, m2 = sn.base[2] - r2;
                if (!ok) {
                    raise_flag(flag, MR_FLAG_DOMAIN);
                } else if (m0 >= 0 && m0 < CT::RC && m1 >= 0 && m1 < CT::RC && m2 >= 0 && m2 < CT::RC) {
                    key = m0 + CT::RC * (m1 + CT::RC * m2);
                    nbd = m0 + CT::SY * m1 + CT::SZ * m2;
                    pending = true;
                } else {
                    // left the region since the sort: global atomics
                    scatter_global<3>(g, sn, pl, grid_out);
                }
            }
            while (__ballot(pending) != 0) {
                if (pending) owner[key] = lane;
                lds_order();
                const bool go = pending && owner[key] == lane;
                lds_order();
                if (go) {
                    opaque_payload<3>(sn, pl);
                    auto rmw = [&](int o0, int o1, int o2, float mw, float q0, float q1, float q2) {
                        float4 *a4 = acc + nbd + o0 + CT::SY * o1 + CT::SZ * o2;
                        float4 q = *a4;
                        q.x += mw;
                        q.y += q0;
                        q.z += q1;
                        q.w += q2;
                        *a4 = q;
                        lds_order();
                    };
                    p2g_separable<3, decltype(rmw) &, MR_TILE_ORDERED != 0>(g, sn, pl, rmw);
                    pending = false;
                }
            }
        }
    }
    lds_order();
    // flush the region: one global atomic per non-zero node channel
    flush_region_3d(acc, r0, r1, r2, g, grid_out, lane);
}

// Deterministic mode: node i of the grid sums the staged regions of the
// tiles covering it (a tile's region spans nodes TS*tt - 1 .. TS*tt + TS + 2
// per axis) in ascending tile order, skipping empty tiles, and writes (or
// adds to) the grid.
template <int D>
__global__ void det_combine_kernel(GridK g, TileGeom tg, const int32_t *offsets,
                                   const float4 *stage, float *grid, int accumulate)
{
    using CT = CellTile<D>;
    constexpr int RN = (D == 3) ? CT::R * CT::R * CT::R : CT::R * CT::R;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nodes = (int64_t)g.n0 * g.n1 * (D == 3 ? g.n2 : 1);
    if (i >= nodes) return;
    const int c[3] = {(int)(i % g.n0), (int)((i / g.n0) % g.n1),
                      D == 3 ? (int)(i / ((int64_t)g.n0 * g.n1)) : 0};
    const int nt[3] = {tg.nt0, tg.nt1, tg.nt2};
    int lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
#pragma unroll
    for (int a = 0; a < D; ++a) {
        // tiles tt with TS tt - 1 <= c <= TS tt + R - 2
        int l = c[a] - (CT::R - 2);
        l = l <= 0 ? 0 : (l + CT::TS - 1) / CT::TS;
        int h = (c[a] + 1) / CT::TS;
        hi[a] = h < nt[a] - 1 ? h : nt[a] - 1;
        lo[a] = l;
    }
    float4 sum = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    for (int t2 = lo[2]; t2 <= hi[2]; ++t2)
        for (int t1 = lo[1]; t1 <= hi[1]; ++t1)
            for (int t0 = lo[0]; t0 <= hi[0]; ++t0) {
                const int64_t t = t0 + (int64_t)tg.nt0 * (t1 + (int64_t)tg.nt1 * t2);
                if (offsets[t * Tiling<D>::CELLS] == offsets[(t + 1) * Tiling<D>::CELLS]) continue;
                const int l0 = c[0] - (t0 * CT::TS - 1), l1 = c[1] - (t1 * CT::TS - 1);
                const int l2 = D == 3 ? c[2] - (t2 * CT::TS - 1) : 0;
                const float4 q = stage[t * RN + l0 + CT::R * (l1 + CT::R * l2)];
                sum.x += q.x;
                sum.y += q.y;
                sum.z += q.z;
                sum.w += q.w;
            }
    float4 *gp = reinterpret_cast<float4 *>(grid) + i;
    if (accumulate) {
        float4 o = *gp;
        sum = make_float4(o.x + sum.x, o.y + sum.y, o.z + sum.z, o.w + sum.w);
    }
    *gp = sum;
}

// ---------------------------------------------------------------------------
// grid update

template <int D>
__global__ void grid_update_kernel(GridK g, float dt, float *grid, const int32_t *active,
                                   int64_t count, float *clear = nullptr)
{
    int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= count) return;
    int64_t i = active ? (int64_t)active[s] : s;
    // the time loop clears the other grid buffer (the next scatter target)
    // in the same pass
    if (clear) reinterpret_cast<float4 *>(clear)[i] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    float4 *gp = reinterpret_cast<float4 *>(grid) + i;
    float4 q = *gp;
    if (!(q.x > 0.0f)) {
        // massless: v = 0; the untouched nodes of a scatter are zero already
        // (most of the grid), so only a non-zero node is written
        if (q.x != 0.0f || q.y != 0.0f || q.z != 0.0f || q.w != 0.0f)
            *gp = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        return;
    }
    float inv = 1.0f / q.x;
    float v[3];
    v[0] = q.y * inv + dt * g.g0;
    v[1] = q.z * inv + dt * g.g1;
    v[2] = (D == 3) ? q.w * inv + dt * g.g2 : 0.0f;
    int i0 = (int)(i % g.n0);
    int i1 = (int)((i / g.n0) % g.n1);
    int i2 = (int)(i / ((int64_t)g.n0 * g.n1));
    apply_bc<D>(g, i0, i1, i2, v);
    *gp = make_float4(q.x, v[0], v[1], D == 3 ? v[2] : 0.0f);
}

// ---------------------------------------------------------------------------
// G2P

template <int D>
__global__ void __launch_bounds__(256) g2p_kernel(GridK g, int64_t n, float *x, float *v,
                                                  float *C, float *F, const int32_t *subset,
                                                  int64_t ns, float dt, const float *grid,
                                                  int apic, int update_F, int trial,
                                                  float *x_trial, float *v_trial, int32_t *flag)
{
    int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= ns) return;
    int64_t p = subset ? (int64_t)subset[s] : s;
    float xp[D];
#pragma unroll
    for (int a = 0; a < D; ++a) xp[a] = x[a * n + p];
    Stencil<D> st;
    if (!make_stencil<D>(g, xp, st)) {
        raise_flag(flag, MR_FLAG_DOMAIN);
        return;
    }
    float vp[D], Bp[D * D], gv[D * D];
    const float4 *g4 = reinterpret_cast<const float4 *>(grid);
    g2p_separable<D>(g, st, [&](int o0, int o1, int o2) {
        return g4[node_lin(g, st.base[0] + o0, st.base[1] + o1, D == 3 ? st.base[2] + o2 : 0)];
    }, vp, Bp, gv);
    if (trial) {
#pragma unroll
        for (int a = 0; a < D; ++a) {
            v_trial[a * ns + s] = vp[a];
            x_trial[a * ns + s] = xp[a] + dt * vp[a];
        }
        return;
    }
#pragma unroll
    for (int a = 0; a < D; ++a) v[a * n + p] = vp[a];
    if (C) {
        float sc = apic ? 4.0f * g.inv_dx * g.inv_dx : 0.0f;
#pragma unroll
        for (int k = 0; k < D * D; ++k) C[k * n + p] = sc * Bp[k];
    }
    if (update_F) {
        float Fp[D * D], Fn[D * D];
#pragma unroll
        for (int k = 0; k < D * D; ++k) Fp[k] = F[k * n + p];
        mr::update_F<D>(gv, Fp, dt, Fn);
#pragma unroll
        for (int k = 0; k < D * D; ++k) F[k * n + p] = Fn[k];
    }
#pragma unroll
    for (int a = 0; a < D; ++a) x[a * n + p] = xp[a] + dt * vp[a];
}

// ---------------------------------------------------------------------------
// workspace layout of the cell sort / sorted P2G

struct SortWorkspace {
    int32_t *keys, *counts, *offsets, *fill, *cell_sorted, *perm, *block_sums, *total;
    float *copy;
    float4 *stage;   // deterministic P2G: every tile's region, [tile][region node]
    int64_t ncells;
};

template <int D>
int64_t sort_ws_bytes(const GridK &g, int64_t n, SortWorkspace *ws, char *basep)
{
    TileGeom tg = tile_geom<D>(g);
    int64_t ncells = tg.ntiles * Tiling<D>::CELLS + 1;  // + overflow bucket
    int64_t nb = ceil_div(ncells + 1, SCAN_BLOCK);
    int64_t off = 0;
    auto take = [&](int64_t bytes) {
        int64_t o = off;
        off += (bytes + 255) & ~(int64_t)255;
        return o;
    };
    int64_t o_keys = take(4 * n), o_counts = take(4 * (ncells + 1)),
            o_offsets = take(4 * (ncells + 1)), o_fill = take(4 * (ncells + 1)),
            o_cs = take(4 * n), o_perm = take(4 * n), o_bs = take(4 * nb), o_tot = take(4),
            o_copy = take(4 * n * (2 * D + 2 * D * D + 3)),
            o_stage = take(16 * tg.ntiles * (int64_t)Tiling<D>::RN);
    if (ws) {
        ws->keys = (int32_t *)(basep + o_keys);
        ws->counts = (int32_t *)(basep + o_counts);
        ws->offsets = (int32_t *)(basep + o_offsets);
        ws->fill = (int32_t *)(basep + o_fill);
        ws->cell_sorted = (int32_t *)(basep + o_cs);
        ws->perm = (int32_t *)(basep + o_perm);
        ws->block_sums = (int32_t *)(basep + o_bs);
        ws->total = (int32_t *)(basep + o_tot);
        ws->copy = (float *)(basep + o_copy);
        ws->stage = (float4 *)(basep + o_stage);
        ws->ncells = ncells;
    }
    return off;
}

template <int D>
int32_t cell_sort_impl(const GridK &g, mr_particles *parts, int32_t *perm_out, void *workspace,
                       int32_t *flag, hipStream_t st, int32_t *carry = nullptr,
                       const mr_particles *dst = nullptr, int32_t *carry_dst = nullptr,
                       bool canonical = false)
{
    const int64_t n = parts->n;
    SortWorkspace ws;
    sort_ws_bytes<D>(g, n, &ws, (char *)workspace);
    TileGeom tg = tile_geom<D>(g);
    const int64_t ncells = ws.ncells;
    zero_words(ws.counts, ncells + 1, st);
    zero_words(ws.fill, ncells + 1, st);
    if (n == 0) {
        zero_words(ws.offsets, ncells + 1, st);
        MR_LAUNCH_CHECK();
        return MR_OK;
    }
    const int TB = 256;
    unsigned gb = (unsigned)ceil_div(n, TB);
    cell_key_kernel<D><<<gb, TB, 0, st>>>(g, tg, parts->x, n, ws.keys, ws.counts, flag);
    int32_t rc = exclusive_scan(ws.counts, ncells + 1, ws.offsets, ws.block_sums, ws.total, st);
    if (rc != MR_OK) return rc;
    cell_scatter_kernel<<<gb, TB, 0, st>>>(ws.keys, n, ws.offsets, ws.fill, ws.cell_sorted);
    cell_segment_sort_kernel<D><<<(unsigned)ceil_div(ncells, TB), TB, 0, st>>>(
        ws.offsets, ws.counts, ncells, ws.cell_sorted, parts->x, n, canonical ? 1 : 0);
    tile_slot_kernel<D><<<(unsigned)tg.ntiles, Tiling<D>::CELLS, 0, st>>>(
        ws.offsets, ws.counts, ws.cell_sorted, ws.perm, tg.ntiles);
    tail_copy_kernel<<<gb, TB, 0, st>>>(ws.cell_sorted, ws.perm,
                                        ws.offsets + tg.ntiles * Tiling<D>::CELLS, n);
    MR_LAUNCH_CHECK();
    // gather every particle array through the permutation: in place (through
    // a copy) or, when a destination set is given, straight into it
    struct Arr {
        float *p, *q;
        int planes;
    } arrs[7] = {{parts->x, dst ? dst->x : nullptr, D},
                 {parts->v, dst ? dst->v : nullptr, D},
                 {parts->C, dst ? dst->C : nullptr, D * D},
                 {parts->F, dst ? dst->F : nullptr, D * D},
                 {const_cast<float *>(parts->m), dst ? const_cast<float *>(dst->m) : nullptr, 1},
                 {const_cast<float *>(parts->V0), dst ? const_cast<float *>(dst->V0) : nullptr, 1},
                 {reinterpret_cast<float *>(carry), reinterpret_cast<float *>(carry_dst), 1}};
    for (auto &a : arrs) {
        if (!a.p) continue;
        if (dst) {
            gather_plane_kernel<<<gb, TB, 0, st>>>(a.p, a.q, ws.perm, n, a.planes);
        } else {
            MR_CHECK_HIP(hipMemcpyAsync(ws.copy, a.p, 4 * n * a.planes, hipMemcpyDeviceToDevice, st));
            gather_plane_kernel<<<gb, TB, 0, st>>>(ws.copy, a.p, ws.perm, n, a.planes);
        }
    }
    MR_LAUNCH_CHECK();
    if (perm_out)
        MR_CHECK_HIP(hipMemcpyAsync(perm_out, ws.perm, 4 * n, hipMemcpyDeviceToDevice, st));
    return MR_OK;
}

template <int D>
PartPtrs<D> part_ptrs(const mr_particles *p)
{
    PartPtrs<D> pp;
    pp.x = p->x;
    pp.v = p->v;
    pp.C = p->C;
    pp.F = p->F;
    pp.m = p->m;
    pp.V0 = p->V0;
    pp.m_u = p->m_uniform;
    pp.V0_u = p->V0_uniform;
    pp.n = p->n;
    return pp;
}

template <int D>
int32_t p2g_impl(const GridK &g, const mr_material *mat, const mr_particles *parts,
                 const int32_t *subset, int64_t ns, float dt, float *grid, int32_t flags,
                 void *workspace, int32_t *flag, hipStream_t st)
{
    Lame lm = lame_of(mat->E, mat->nu);
    int apic = (flags & MR_NO_AFFINE) ? 0 : 1;
    PartPtrs<D> pp = part_ptrs<D>(parts);
    if (flags & MR_DETERMINISTIC) {
        // every node is written by the combine (added to with MR_ACCUMULATE)
        SortWorkspace ws;
        sort_ws_bytes<D>(g, parts->n, &ws, (char *)workspace);
        TileGeom tg = tile_geom<D>(g);
        if (tg.ntiles > 0)
            tile_scatter_kernel<D, false, true><<<tile_blocks<D>(tg), 64 * CellTile<D>::WPB, 0, st>>>(
                g, tg, parts->x, parts->v, parts->C, parts->F, parts->m, parts->V0, parts->m_uniform,
                parts->V0_uniform, parts->n, ws.offsets, ws.counts, apic, mat->model, lm.mu, lm.la, dt,
                nullptr, grid, nullptr, nullptr, flag, ws.stage);
        const int64_t nodes = grid_nodes(g);
        det_combine_kernel<D><<<(unsigned)ceil_div(nodes, 256), 256, 0, st>>>(
            g, tg, ws.offsets, ws.stage, grid, (flags & MR_ACCUMULATE) ? 1 : 0);
        MR_LAUNCH_CHECK();
        return MR_OK;
    }
    if (!(flags & MR_ACCUMULATE)) zero_words(grid, 4 * grid_nodes(g), st);
    if ((flags & MR_SORTED) && !subset) {
        SortWorkspace ws;
        sort_ws_bytes<D>(g, parts->n, &ws, (char *)workspace);
        TileGeom tg = tile_geom<D>(g);
        if (tg.ntiles > 0 && D == 3 && MR_TILE_WPB == 1) {
            // the per-cell kernel reads both per-particle arrays (masses and
            // volumes) or neither; with only one of them the general tile
            // kernel runs
            const bool per = parts->m || parts->V0;
            const float *Cl = apic && parts->C ? parts->C : parts->F;
            const unsigned nb = tile_blocks<D>(tg);
            // the sort's key array is dead until the next sort: the tiles'
            // overflowing deferred lists go there
            auto launch = [&](auto kern) {
                kern<<<nb, 64, 0, st>>>(g, tg, parts->x, parts->v, Cl, parts->F, parts->m,
                                        parts->V0, parts->m_uniform, parts->V0_uniform, parts->n,
                                        ws.offsets, ws.counts, apic, lm.mu, lm.la, dt, grid,
                                        ws.keys, flag);
            };
            if (per && !(parts->m && parts->V0)) {
                // one per-particle array only: the general kernel
                tile_scatter_kernel<D, false><<<nb, 64 * CellTile<D>::WPB, 0, st>>>(
                    g, tg, parts->x, parts->v, parts->C, parts->F, parts->m, parts->V0,
                    parts->m_uniform, parts->V0_uniform, parts->n, ws.offsets, ws.counts, apic,
                    mat->model, lm.mu, lm.la, dt, nullptr, grid, nullptr, nullptr, flag);
            } else if (mat->model == MR_NEO_HOOKEAN) {
                if (per)
                    launch(cell_sum_p2g_kernel<MR_NEO_HOOKEAN, true>);
                else
                    launch(cell_sum_p2g_kernel<MR_NEO_HOOKEAN, false>);
            } else {
                if (per)
                    launch(cell_sum_p2g_kernel<MR_FIXED_COROTATED, true>);
                else
                    launch(cell_sum_p2g_kernel<MR_FIXED_COROTATED, false>);
            }
        } else if (tg.ntiles > 0) {
            tile_scatter_kernel<D, false><<<tile_blocks<D>(tg), 64 * CellTile<D>::WPB, 0, st>>>(
                g, tg, parts->x, parts->v, parts->C, parts->F, parts->m, parts->V0, parts->m_uniform,
                parts->V0_uniform, parts->n, ws.offsets, ws.counts, apic, mat->model, lm.mu, lm.la, dt,
                nullptr, grid, nullptr, nullptr, flag);
        }
        // particles in the overflow bucket (outside the lattice at sort time)
        // were flagged by the sort; the tiled kernel only covers tiles
        MR_LAUNCH_CHECK();
        return MR_OK;
    }
    if (ns > 0)
        p2g_atomic_kernel<D><<<(unsigned)ceil_div(ns, 256), 256, 0, st>>>(
            g, pp, subset, ns, apic, mat->model, lm.mu, lm.la, dt, grid, flag);
    MR_LAUNCH_CHECK();
    return MR_OK;
}

}  // namespace mr

using namespace mr;

static bool check_parts(const mr_particles *p, int dim, bool need_vCF)
{
    if (!p || p->n < 0) return false;
    if (p->n == 0) return true;  // nothing is dereferenced
    if (!p->x) return false;
    if (need_vCF && (!p->v || !p->F)) return false;
    (void)dim;
    return true;
}

extern "C" int32_t mpm_p2g(const mr_grid *grid_desc, const mr_material *mat,
                           const mr_particles *parts, const int32_t *subset, int64_t n_subset,
                           float dt, float *grid, int32_t flags, void *workspace,
                           int32_t *status_flag, void *stream)
{
    GridK g;
    if (!grid_from_desc(grid_desc, g) || !mat || !grid || !check_parts(parts, grid_desc->dim, true))
        return MR_EINVAL;
    if (!(flags & MR_NO_AFFINE) && !parts->C && parts->n > 0) return MR_EINVAL;
    if (mat->model != MR_FIXED_COROTATED && mat->model != MR_NEO_HOOKEAN) return MR_EINVAL;
    if ((flags & MR_SORTED) && !workspace) return MR_EINVAL;
    if ((flags & MR_DETERMINISTIC) && (!(flags & MR_SORTED) || subset)) return MR_EINVAL;
    int64_t ns = subset ? n_subset : parts->n;
    if (ns < 0) return MR_EINVAL;
    hipStream_t st = as_stream(stream);
    if (grid_desc->dim == 2)
        return p2g_impl<2>(g, mat, parts, subset, ns, dt, grid, flags, workspace, status_flag, st);
    return p2g_impl<3>(g, mat, parts, subset, ns, dt, grid, flags, workspace, status_flag, st);
}

extern "C" int32_t mpm_grid_update(const mr_grid *grid_desc, float dt, float *grid,
                                   const int32_t *active, int64_t n_active, void *stream)
{
    GridK g;
    if (!grid_from_desc(grid_desc, g) || !grid) return MR_EINVAL;
    int64_t count = active ? n_active : grid_nodes(g);
    if (count < 0) return MR_EINVAL;
    if (count == 0) return MR_OK;
    hipStream_t st = as_stream(stream);
    unsigned gb = (unsigned)ceil_div(count, 256);
    if (grid_desc->dim == 2)
        grid_update_kernel<2><<<gb, 256, 0, st>>>(g, dt, grid, active, count);
    else
        grid_update_kernel<3><<<gb, 256, 0, st>>>(g, dt, grid, active, count);
    MR_LAUNCH_CHECK();
    return MR_OK;
}

extern "C" int32_t mpm_g2p(const mr_grid *grid_desc, mr_particles *parts, const int32_t *subset,
                           int64_t n_subset, float dt, const float *grid, int32_t flags,
                           float *x_trial, float *v_trial, int32_t *status_flag, void *stream)
{
    GridK g;
    if (!grid_from_desc(grid_desc, g) || !grid || !parts || parts->n < 0 ||
        (parts->n > 0 && !parts->x))
        return MR_EINVAL;
    bool trial = (flags & MR_TRIAL) != 0;
    if (trial && (!x_trial || !v_trial)) return MR_EINVAL;
    int update_F = (!trial && !(flags & MR_NO_F_UPDATE)) ? 1 : 0;
    if (!trial && parts->n > 0 && (!parts->v || (update_F && !parts->F))) return MR_EINVAL;
    int apic = (flags & MR_NO_AFFINE) ? 0 : 1;
    int64_t ns = subset ? n_subset : parts->n;
    if (ns < 0) return MR_EINVAL;
    if (ns == 0) return MR_OK;
    hipStream_t st = as_stream(stream);
    unsigned gb = (unsigned)ceil_div(ns, 256);
    if (grid_desc->dim == 2)
        g2p_kernel<2><<<gb, 256, 0, st>>>(g, parts->n, parts->x, parts->v, parts->C, parts->F,
                                          subset, ns, dt, grid, apic, update_F, trial ? 1 : 0,
                                          x_trial, v_trial, status_flag);
    else
        g2p_kernel<3><<<gb, 256, 0, st>>>(g, parts->n, parts->x, parts->v, parts->C, parts->F,
                                          subset, ns, dt, grid, apic, update_F, trial ? 1 : 0,
                                          x_trial, v_trial, status_flag);
    MR_LAUNCH_CHECK();
    return MR_OK;
}

extern "C" int64_t mpm_workspace_bytes(const mr_grid *grid_desc, int64_t n)
{
    GridK g;
    if (!grid_from_desc(grid_desc, g) || n < 0) return -1;
    return grid_desc->dim == 2 ? sort_ws_bytes<2>(g, n, nullptr, nullptr)
                               : sort_ws_bytes<3>(g, n, nullptr, nullptr);
}

extern "C" int32_t mpm_cell_sort_ex(const mr_grid *grid_desc, mr_particles *parts,
                                    int32_t *perm_out, void *workspace, int32_t flags,
                                    int32_t *status_flag, void *stream)
{
    GridK g;
    if (!grid_from_desc(grid_desc, g) || !workspace || !check_parts(parts, grid_desc->dim, false))
        return MR_EINVAL;
    if (parts->n > INT32_MAX || (flags & ~MR_DETERMINISTIC)) return MR_EINVAL;
    hipStream_t st = as_stream(stream);
    const bool canon = (flags & MR_DETERMINISTIC) != 0;
    return grid_desc->dim == 2
               ? cell_sort_impl<2>(g, parts, perm_out, workspace, status_flag, st, nullptr, nullptr,
                                   nullptr, canon)
               : cell_sort_impl<3>(g, parts, perm_out, workspace, status_flag, st, nullptr, nullptr,
                                   nullptr, canon);
}

extern "C" int32_t mpm_cell_sort(const mr_grid *grid_desc, mr_particles *parts, int32_t *perm_out,
                                 void *workspace, int32_t *status_flag, void *stream)
{
    return mpm_cell_sort_ex(grid_desc, parts, perm_out, workspace, 0, status_flag, stream);
}

extern "C" int32_t mpm_cell_keys(const mr_grid *grid_desc, const mr_particles *parts,
                                 int32_t *keys_out, void *stream)
{
    GridK g;
    if (!grid_from_desc(grid_desc, g) || !keys_out || !check_parts(parts, grid_desc->dim, false))
        return MR_EINVAL;
    if (parts->n == 0) return MR_OK;
    hipStream_t st = as_stream(stream);
    unsigned gb = (unsigned)ceil_div(parts->n, 256);
    if (grid_desc->dim == 2) {
        TileGeom tg = tile_geom<2>(g);
        cell_key_kernel<2><<<gb, 256, 0, st>>>(g, tg, parts->x, parts->n, keys_out, nullptr, nullptr);
    } else {
        TileGeom tg = tile_geom<3>(g);
        cell_key_kernel<3><<<gb, 256, 0, st>>>(g, tg, parts->x, parts->n, keys_out, nullptr, nullptr);
    }
    MR_LAUNCH_CHECK();
    return MR_OK;
}

extern "C" int32_t mr_sync_status(void *stream, const int32_t *device_flags, int32_t n,
                                  int32_t *host_flags)
{
    if (n < 0 || (n > 0 && (!device_flags || !host_flags))) return MR_EINVAL;
    hipStream_t st = as_stream(stream);
    if (n > 0)
        MR_CHECK_HIP(hipMemcpyAsync(host_flags, device_flags, sizeof(int32_t) * n,
                                    hipMemcpyDeviceToHost, st));
    MR_CHECK_HIP(hipStreamSynchronize(st));
    int32_t bits = 0;
    for (int32_t i = 0; i < n; ++i) bits |= host_flags[i];
    if (bits & MR_FLAG_DOMAIN) return MR_EDOMAIN;
    if (bits & MR_FLAG_SINGULAR) return MR_ESINGULAR;
    if (bits & (MR_FLAG_NOCONV | MR_FLAG_LINESEARCH)) return MR_ENOCONV;
    return MR_OK;
}

extern "C" const char *mr_version(void) { return "mpmrom 0.1 gfx950"; }

// ---------------------------------------------------------------------------
// fused grid-to-particle (step n) and particle-to-grid (step n + 1): the same
// tile kernel, with each lane first gathering its particle's G2P stencil from
// the incoming grid (HBM / L2), updating v, C, F and x in registers and then
// scattering the next step's contributions at the new state.  Per particle
// and step only x and F travel through HBM (48 bytes read, 48 written); v and
// C are stored only when v_out / C_out are given.

namespace mr {

template <int D>
int32_t g2p2g_impl(const GridK &g, const mr_material *mat, mr_particles *parts, float dt,
                   const float *grid_in, float *grid_out, int32_t flags, void *workspace,
                   float *v_out, float *C_out, int32_t *flag, hipStream_t st)
{
    Lame lm = lame_of(mat->E, mat->nu);
    int apic = (flags & MR_NO_AFFINE) ? 0 : 1;
    if (!(flags & MR_ACCUMULATE)) zero_words(grid_out, 4 * grid_nodes(g), st);
    SortWorkspace ws;
    sort_ws_bytes<D>(g, parts->n, &ws, (char *)workspace);
    TileGeom tg = tile_geom<D>(g);
    if (tg.ntiles > 0 && parts->n > 0)
        tile_scatter_kernel<D, true><<<tile_blocks<D>(tg), 64 * CellTile<D>::WPB, 0, st>>>(
            g, tg, parts->x, parts->v, parts->C, parts->F, parts->m, parts->V0, parts->m_uniform,
            parts->V0_uniform, parts->n, ws.offsets, ws.counts, apic, mat->model, lm.mu, lm.la, dt,
            grid_in, grid_out, v_out, C_out, flag);
    MR_LAUNCH_CHECK();
    return MR_OK;
}

}  // namespace mr

extern "C" int32_t mpm_g2p2g(const mr_grid *grid_desc, const mr_material *mat,
                             mr_particles *parts, float dt, const float *grid_in, float *grid_out,
                             int32_t flags, void *workspace, int32_t *status_flag, void *stream)
{
    GridK g;
    if (!grid_from_desc(grid_desc, g) || !mat || !grid_in || !grid_out || grid_in == grid_out ||
        !workspace || !check_parts(parts, grid_desc->dim, true))
        return MR_EINVAL;
    if (mat->model != MR_FIXED_COROTATED && mat->model != MR_NEO_HOOKEAN) return MR_EINVAL;
    hipStream_t st = as_stream(stream);
    float *vo = (flags & MR_NO_VC_OUT) ? nullptr : parts->v;
    float *co = ((flags & MR_NO_VC_OUT) || (flags & MR_NO_AFFINE)) ? nullptr : parts->C;
    if (!(flags & MR_NO_AFFINE) && !(flags & MR_NO_VC_OUT) && !parts->C && parts->n > 0)
        return MR_EINVAL;
    return grid_desc->dim == 2
               ? g2p2g_impl<2>(g, mat, parts, dt, grid_in, grid_out, flags, workspace, vo, co,
                               status_flag, st)
               : g2p2g_impl<3>(g, mat, parts, dt, grid_in, grid_out, flags, workspace, vo, co,
                               status_flag, st);
}

// ---------------------------------------------------------------------------
// launch timing (HIP events recorded around each launch on its stream)

struct mr_timing {
    int32_t cap, count;
    hipEvent_t *ev;  // 2 per record
    int32_t *cls;
    uint32_t mask;        // classes recorded
    int32_t every;        // record every `every`-th launch of a class
    int64_t seen[32];     // launches of each class since the last reset
};

extern "C" int32_t mr_timing_create(int32_t capacity, mr_timing **out)
{
    if (capacity < 1 || !out) return MR_EINVAL;
    mr_timing *t = (mr_timing *)calloc(1, sizeof(mr_timing));
    if (!t) return MR_ENOMEM;
    t->cap = capacity;
    t->mask = ~0u;
    t->every = 1;
    t->ev = (hipEvent_t *)calloc(2 * (size_t)capacity, sizeof(hipEvent_t));
    t->cls = (int32_t *)calloc((size_t)capacity, sizeof(int32_t));
    if (!t->ev || !t->cls) {
        free(t->ev);
        free(t->cls);
        free(t);
        return MR_ENOMEM;
    }
    for (int32_t i = 0; i < 2 * capacity; ++i)
        if (hipEventCreate(&t->ev[i]) != hipSuccess) {
            for (int32_t j = 0; j < i; ++j) (void)hipEventDestroy(t->ev[j]);
            free(t->ev);
            free(t->cls);
            free(t);
            return MR_EDEVICE;
        }
    *out = t;
    return MR_OK;
}

extern "C" void mr_timing_destroy(mr_timing *t)
{
    if (!t) return;
    for (int32_t i = 0; i < 2 * t->cap; ++i) (void)hipEventDestroy(t->ev[i]);
    free(t->ev);
    free(t->cls);
    free(t);
}

extern "C" int32_t mr_timing_reset(mr_timing *t)
{
    if (!t) return MR_EINVAL;
    t->count = 0;
    for (int64_t &c : t->seen) c = 0;
    return MR_OK;
}

extern "C" int32_t mr_timing_sample(mr_timing *t, uint32_t class_mask, int32_t every)
{
    if (!t || every < 1) return MR_EINVAL;
    t->mask = class_mask;
    t->every = every;
    for (int64_t &c : t->seen) c = 0;
    return MR_OK;
}

extern "C" int32_t mr_timing_read(mr_timing *t, int32_t n_classes, int64_t *launches,
                                  double *total_ms)
{
    if (!t || n_classes < 1 || !launches || !total_ms) return MR_EINVAL;
    for (int32_t c = 0; c < n_classes; ++c) {
        launches[c] = 0;
        total_ms[c] = 0.0;
    }
    for (int32_t i = 0; i < t->count; ++i) {
        MR_CHECK_HIP(hipEventSynchronize(t->ev[2 * i + 1]));
        float ms = 0.0f;
        MR_CHECK_HIP(hipEventElapsedTime(&ms, t->ev[2 * i], t->ev[2 * i + 1]));
        int32_t c = t->cls[i];
        if (c >= 0 && c < n_classes) {
            launches[c] += 1;
            total_ms[c] += ms;
        }
    }
    return MR_OK;
}

namespace mr {
struct TimedLaunch {
    mr_timing *t;
    int idx;
    hipStream_t st;
    TimedLaunch(mr_timing *tm, int cls, hipStream_t s) : t(tm), idx(-1), st(s)
    {
        if (t && cls >= 0 && cls < 32 && ((t->mask >> cls) & 1u) &&
            t->seen[cls]++ % t->every == 0 && t->count < t->cap) {
            idx = t->count++;
            t->cls[idx] = cls;
            (void)hipEventRecord(t->ev[2 * idx], st);
        }
    }
    ~TimedLaunch()
    {
        if (idx >= 0) (void)hipEventRecord(t->ev[2 * idx + 1], st);
    }
};
}  // namespace mr

// ---------------------------------------------------------------------------
// multi-step driver

extern "C" int64_t mpm_step_workspace_bytes(const mr_grid *grid_desc, int64_t n)
{
    GridK g;
    if (!grid_from_desc(grid_desc, g) || n < 0) return -1;
    int64_t sort_bytes = mpm_workspace_bytes(grid_desc, n);
    return sort_bytes + 16 * grid_nodes(g) + 256;  // + the second grid buffer
}

__global__ void iota_kernel(int32_t *a, int64_t n)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = (int32_t)i;
}

extern "C" int32_t mpm_step(const mr_grid *grid_desc, const mr_material *mat,
                            mr_particles *parts, float dt, int32_t n_steps, int32_t sort_every,
                            int32_t flags, float *grid, void *workspace, int32_t *perm_accum,
                            int32_t *status_flag, mr_timing *timing, void *stream)
{
    GridK g;
    if (!grid_from_desc(grid_desc, g) || !mat || !grid || !workspace || n_steps < 0 ||
        sort_every < 0 || !check_parts(parts, grid_desc->dim, true))
        return MR_EINVAL;
    if (!(flags & MR_NO_AFFINE) && !parts->C && parts->n > 0) return MR_EINVAL;
    if (sort_every > 0 && parts->n > INT32_MAX) return MR_EINVAL;
    if ((flags & MR_DETERMINISTIC) && sort_every < 1) return MR_EINVAL;
    const bool det = (flags & MR_DETERMINISTIC) != 0;
    const int dim = grid_desc->dim;
    int32_t rc = MR_OK;
    hipStream_t st = as_stream(stream);
    if (perm_accum && parts->n > 0) {
        iota_kernel<<<(unsigned)ceil_div(parts->n, 256), 256, 0, st>>>(perm_accum, parts->n);
        MR_LAUNCH_CHECK();
    }
    if (n_steps == 0) return MR_OK;
    const bool sorted = sort_every > 0;
    const int32_t naff = flags & MR_NO_AFFINE;
    float *gA = grid;
    float *gB = (float *)((char *)workspace + ((mpm_workspace_bytes(grid_desc, parts->n) + 255) &
                                               ~(int64_t)255));
    // The state alternates between the caller's arrays and a copy in the
    // sort workspace: each sort gathers from one set into the other, and the
    // last state is copied back at the end if it lives in the workspace.
    const int64_t n = parts->n;
    SortWorkspace sws;
    if (dim == 2)
        sort_ws_bytes<2>(g, n, &sws, (char *)workspace);
    else
        sort_ws_bytes<3>(g, n, &sws, (char *)workspace);
    mr_particles shadow = *parts;
    int32_t *shadow_carry = nullptr;
    {
        float *cp = sws.copy;
        auto carve = [&](const float *src, int planes) -> float * {
            if (!src) return nullptr;
            float *q = cp;
            cp += (int64_t)planes * n;
            return q;
        };
        shadow.x = carve(parts->x, dim);
        shadow.v = carve(parts->v, dim);
        shadow.C = carve(parts->C, dim * dim);
        shadow.F = carve(parts->F, dim * dim);
        shadow.m = carve(parts->m, 1);
        shadow.V0 = carve(parts->V0, 1);
        shadow_carry = perm_accum ? reinterpret_cast<int32_t *>(cp) : nullptr;
    }
    mr_particles *cur = parts, *other = &shadow;
    int32_t *carry_cur = perm_accum, *carry_other = shadow_carry;
    auto do_sort = [&]() -> int32_t {
        TimedLaunch tl(timing, MR_KC_SORT, st);
        int32_t r = dim == 2 ? cell_sort_impl<2>(g, cur, nullptr, workspace, status_flag, st,
                                                 carry_cur, other, carry_other, det)
                             : cell_sort_impl<3>(g, cur, nullptr, workspace, status_flag, st,
                                                 carry_cur, other, carry_other, det);
        mr_particles *tp = cur;
        cur = other;
        other = tp;
        int32_t *tc = carry_cur;
        carry_cur = carry_other;
        carry_other = tc;
        return r;
    };
    auto copy_back = [&]() -> int32_t {
        if (cur == parts) return MR_OK;
        struct {
            const float *src;
            float *dst;
            int planes;
        } planes[7] = {{shadow.x, parts->x, dim},
                       {shadow.v, parts->v, dim},
                       {shadow.C, parts->C, dim * dim},
                       {shadow.F, parts->F, dim * dim},
                       {shadow.m, const_cast<float *>(parts->m), 1},
                       {shadow.V0, const_cast<float *>(parts->V0), 1},
                       {reinterpret_cast<const float *>(shadow_carry),
                        reinterpret_cast<float *>(perm_accum), 1}};
        for (auto &c : planes)
            if (c.src && c.dst)
                MR_CHECK_HIP(hipMemcpyAsync(c.dst, c.src, 4 * n * c.planes, hipMemcpyDeviceToDevice,
                                            st));
        return MR_OK;
    };
    auto do_p2g = [&](float *target, bool cleared) -> int32_t {
        TimedLaunch tl(timing, MR_KC_P2G, st);
        return mpm_p2g(grid_desc, mat, cur, nullptr, 0, dt, target,
                       naff | (sorted ? MR_SORTED : 0) | (cleared ? MR_ACCUMULATE : 0) |
                           (det ? MR_DETERMINISTIC : 0), workspace,
                       status_flag, stream);
    };
    const int64_t nodes = grid_nodes(g);
    auto do_update = [&]() -> int32_t {
        // after every grid update the other buffer is free: it is cleared in
        // the same pass for the next scatter
        TimedLaunch tl(timing, MR_KC_GRID, st);
        const unsigned gbn = (unsigned)ceil_div(nodes, 256);
        if (dim == 2)
            grid_update_kernel<2><<<gbn, 256, 0, st>>>(g, dt, gA, nullptr, nodes, gB);
        else
            grid_update_kernel<3><<<gbn, 256, 0, st>>>(g, dt, gA, nullptr, nodes, gB);
        MR_LAUNCH_CHECK();
        return MR_OK;
    };
    auto do_g2p = [&]() -> int32_t {
        TimedLaunch tl(timing, MR_KC_G2P, st);
        return mpm_g2p(grid_desc, cur, nullptr, 0, dt, gA, naff, nullptr, nullptr, status_flag,
                       stream);
    };
    // Every step: G2P from the updated grid, the cell sort when due, the
    // sorted P2G into the other grid buffer (cleared by the previous grid
    // update), then the grid update of that buffer, which clears the first.
    // The separate gather and sorted scatter outrun the fused kernel
    // (mpm_g2p2g) on this part despite re-reading v and C: the gather runs at
    // high occupancy and the scatter alone fits three waves per SIMD.
    if (sorted && (rc = do_sort()) != MR_OK) return rc;
    if ((rc = do_p2g(gA, false)) != MR_OK) return rc;
    if ((rc = do_update()) != MR_OK) return rc;
    for (int32_t s = 1; s < n_steps; ++s) {
        if ((rc = do_g2p()) != MR_OK) return rc;
        if (sorted && s % sort_every == 0 && (rc = do_sort()) != MR_OK) return rc;
        if ((rc = do_p2g(gB, true)) != MR_OK) return rc;
        float *tmp = gA;
        gA = gB;
        gB = tmp;
        if ((rc = do_update()) != MR_OK) return rc;
    }
    if ((rc = do_g2p()) != MR_OK) return rc;
    return copy_back();
}
