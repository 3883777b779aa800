// sort.hip -- periodic counting sort of a species by cell, in tile-major cell
// order, so that the particles of one tile (the unit of work of the particle
// kernel) are contiguous, and rank-interleaved inside each tile: the particle
// of rank 0 of every cell of the tile (cells in the tile's cell order), then
// those of rank 1, and so on, so that the 64 lanes of a wave that take
// consecutive particles work in distinct cells.  Histogram with atomics (the
// returned slot is the particle's rank in its cell), exclusive scan of the
// counts, a per-tile pass computing every particle's final slot, and one
// scatter of the particle arrays into the spare copy, which becomes current.
// Not part of the paper's method; it only fixes the memory order.
#include "pic_internal.h"

namespace pic {
namespace {

constexpr int kSortThreads = 256;
constexpr int kScanItems = 4;
constexpr int kScanChunk = kSortThreads * kScanItems;

__device__ __forceinline__ void unpack(uint32_t c, int i[3])
{
    i[0] = (int)(c & 2047u);
    i[1] = (int)((c >> 11) & 2047u);
    i[2] = (int)(c >> 22);
}

// Order of the 64 cells of one z-plane of a 3D tile (T = 8).  The particle
// kernel's LDS current tile has a row stride of 14 doubles, so cell (lx, ly)
// of a plane sits in 8-byte bank pair r = (lx + 14 ly) mod 16.  Each r is
// taken by exactly four cells of the plane; ordering the plane as (q, r) --
// q the rank of the cell among those four -- makes any 16 consecutive cells
// hit 16 distinct bank pairs, so a wave of rank-interleaved particles issues
// its current atomics without bank conflicts.
__device__ __forceinline__ uint32_t plane_order(uint32_t lx, uint32_t ly)
{
    const uint32_t r = (lx + 14u * ly) & 15u;
    uint32_t q = 0;
    for (uint32_t y = 0; y < ly; ++y) q += ((r + 2u * y) & 15u) < 8u ? 1u : 0u;
    return q * 16u + r;
}

template <class R, int D, int T>
__device__ __forceinline__ uint32_t key_of(const GridK& g, const PartArrays& a, int64_t p)
{
    int i[3] = {0, 0, 0};
    if (sizeof(R) == 4) {
        unpack(a.cell[p], i);
    } else {
        for (int ax = 0; ax < D; ++ax) i[ax] = (int)floor(((const double*)a.pos[ax])[p]);
    }
    for (int ax = 0; ax < 3; ++ax)  // positions are in [0, N); clamp so keys stay in range
        i[ax] = i[ax] < 0 ? 0 : (i[ax] >= g.n[ax] ? g.n[ax] - 1 : i[ax]);
    const int tx = i[0] / T, ty = i[1] / T, tz = D == 3 ? i[2] / T : 0;
    const uint32_t tile = ((uint32_t)tz * g.nt[1] + ty) * g.nt[0] + tx;
    const uint32_t lx = i[0] - tx * T, ly = i[1] - ty * T, lz = D == 3 ? i[2] - tz * T : 0;
    const uint32_t local = D == 3 ? lz * T * T + plane_order(lx, ly) : ly * T + lx;
    return tile * (uint32_t)(D == 3 ? T * T * T : T * T) + local;
}

__global__ void k_zero_u32(uint32_t* p, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * kSortThreads + threadIdx.x;
    if (i < n) p[i] = 0;
}

template <class R, int D, int T>
__global__ __launch_bounds__(kSortThreads) void k_histogram(GridK g, PartArrays a, int64_t n,
                                                            uint32_t* __restrict__ key,
                                                            uint32_t* __restrict__ rank,
                                                            uint32_t* __restrict__ hist)
{
    const int64_t p = (int64_t)blockIdx.x * kSortThreads + threadIdx.x;
    if (p >= n) return;
    const uint32_t k = key_of<R, D, T>(g, a, p);
    key[p] = k;
    rank[p] = atomicAdd(&hist[k], 1u);
}

// Exclusive scan of a block's 1024 counts; returns the block total.
__device__ uint32_t block_scan(uint32_t (&v)[kScanItems], uint32_t* sh)
{
    uint32_t run = 0;
    for (int i = 0; i < kScanItems; ++i) {
        const uint32_t x = v[i];
        v[i] = run;
        run += x;
    }
    const int t = threadIdx.x;
    sh[t] = run;
    __syncthreads();
    for (int off = 1; off < kSortThreads; off <<= 1) {
        const uint32_t x = t >= off ? sh[t - off] : 0u;
        __syncthreads();
        sh[t] += x;
        __syncthreads();
    }
    const uint32_t total = sh[kSortThreads - 1];
    const uint32_t excl = sh[t] - run;
    __syncthreads();
    for (int i = 0; i < kScanItems; ++i) v[i] += excl;
    return total;
}

__global__ __launch_bounds__(kSortThreads) void k_scan_reduce(const uint32_t* __restrict__ in,
                                                              int64_t n, uint32_t* __restrict__ part)
{
    __shared__ uint32_t sh[kSortThreads];
    const int64_t base = (int64_t)blockIdx.x * kScanChunk + (int64_t)threadIdx.x * kScanItems;
    uint32_t s = 0;
    for (int i = 0; i < kScanItems; ++i)
        if (base + i < n) s += in[base + i];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int off = kSortThreads / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

// One workgroup: exclusive scan of the per-block partials, in place.
__global__ __launch_bounds__(kSortThreads) void k_scan_partials(uint32_t* __restrict__ part, int64_t nb)
{
    __shared__ uint32_t sh[kSortThreads];
    uint32_t carry = 0;
    for (int64_t c0 = 0; c0 < nb; c0 += kScanChunk) {
        uint32_t v[kScanItems];
        const int64_t base = c0 + (int64_t)threadIdx.x * kScanItems;
        for (int i = 0; i < kScanItems; ++i) v[i] = base + i < nb ? part[base + i] : 0u;
        const uint32_t total = block_scan(v, sh);
        for (int i = 0; i < kScanItems; ++i)
            if (base + i < nb) part[base + i] = v[i] + carry;
        carry += total;
        __syncthreads();
    }
}

__global__ __launch_bounds__(kSortThreads) void k_scan_apply(uint32_t* __restrict__ data, int64_t n,
                                                             const uint32_t* __restrict__ part)
{
    __shared__ uint32_t sh[kSortThreads];
    const int64_t base = (int64_t)blockIdx.x * kScanChunk + (int64_t)threadIdx.x * kScanItems;
    uint32_t v[kScanItems];
    for (int i = 0; i < kScanItems; ++i) v[i] = base + i < n ? data[base + i] : 0u;
    block_scan(v, sh);
    const uint32_t off = part[blockIdx.x];
    for (int i = 0; i < kScanItems; ++i)
        if (base + i < n) data[base + i] = v[i] + off;
}

// Final slot of every particle of one tile in the rank-interleaved order,
// written per cell-sorted position: dest[cb + r] for the particle of rank r of
// the cell starting at cb.  Rank level r holds the cells with more than r
// particles, in the tile's cell order, contiguously after level r - 1.  One workgroup per
// tile, one thread per cell; only 4-byte writes.
template <int TPD>
__global__ __launch_bounds__(TPD) void k_dest(const uint32_t* __restrict__ offs, int64_t nkeys,
                                              int64_t n, uint32_t* __restrict__ dest)
{
    constexpr int NW = TPD / 64;
    __shared__ uint32_t wsum[NW];
    __shared__ uint32_t wmax[NW];
    const int c = threadIdx.x;
    const int lane = c & 63, wv = c >> 6;
    const int64_t key = (int64_t)blockIdx.x * TPD + c;
    const int64_t cb = offs[key];
    const int64_t ce = key + 1 < nkeys ? (int64_t)offs[key + 1] : n;
    const uint32_t cnt = (uint32_t)(ce - cb);
    const int64_t base = offs[(int64_t)blockIdx.x * TPD];
    uint32_t m = cnt;
    for (int off = 32; off > 0; off >>= 1) m = max(m, (uint32_t)__shfl_xor((int)m, off, 64));
    if (lane == 0) wmax[wv] = m;
    __syncthreads();
    uint32_t maxcnt = 0;
    for (int w = 0; w < NW; ++w) maxcnt = max(maxcnt, wmax[w]);
    int64_t level_base = base;
    for (uint32_t r = 0; r < maxcnt; ++r) {
        const bool flag = cnt > r;
        const unsigned long long mask = __ballot(flag);
        const uint32_t below = (uint32_t)__popcll(mask & ((1ull << lane) - 1ull));
        if (lane == 0) wsum[wv] = (uint32_t)__popcll(mask);
        __syncthreads();
        uint32_t pre = 0, tot = 0;
        for (int w = 0; w < NW; ++w) {
            pre += w < wv ? wsum[w] : 0u;
            tot += wsum[w];
        }
        if (flag) dest[cb + r] = (uint32_t)(level_base + pre + below);
        level_base += tot;
        __syncthreads();
    }
}

// Move every particle straight to its final slot.  Consecutive particles are
// (nearly) tile-ordered from the previous sort, so each XCD takes a contiguous
// run of them: a tile's writes then gather in one XCD's L2.
template <class R>
__global__ __launch_bounds__(kSortThreads) void k_scatter_final(PartArrays src, PartArrays dst, int64_t n,
                                                                const uint32_t* __restrict__ key,
                                                                const uint32_t* __restrict__ rank,
                                                                const uint32_t* __restrict__ offs,
                                                                const uint32_t* __restrict__ dest)
{
    const int nb = gridDim.x;
    const int per = nb / kXcds, rem = nb % kXcds;
    const int x = blockIdx.x % kXcds, local = blockIdx.x / kXcds;
    const int blk = x < rem ? x * (per + 1) + local : rem * (per + 1) + (x - rem) * per + local;
    const int64_t p = (int64_t)blk * kSortThreads + threadIdx.x;
    if (p >= n) return;
    const int64_t q = dest[(int64_t)offs[key[p]] + rank[p]];
    for (int ax = 0; ax < 3; ++ax) {
        ((R*)dst.pos[ax])[q] = ((const R*)src.pos[ax])[p];
        ((R*)dst.mom[ax])[q] = ((const R*)src.mom[ax])[p];
    }
    ((R*)dst.weight)[q] = ((const R*)src.weight)[p];
    if (sizeof(R) == 4) dst.cell[q] = src.cell[p];
    dst.id[q] = src.id[p];
}

template <int TPD>
__global__ void k_tile_start(const uint32_t* __restrict__ offs, int ntiles, int64_t n,
                             int64_t* __restrict__ ts)
{
    const int t = blockIdx.x * kSortThreads + threadIdx.x;
    if (t < ntiles) ts[t] = offs[(int64_t)t * TPD];
    if (t == ntiles) ts[t] = n;
}

unsigned nblk(int64_t n) { return (unsigned)((n + kSortThreads - 1) / kSortThreads); }

template <class R, int D, int T>
hipError_t sort_impl(Ctx& c, Species& sp, hipStream_t s)
{
    const int64_t n = sp.n;
    const int64_t nk = c.nkeys;
    hipLaunchKernelGGL(k_zero_u32, dim3(nblk(nk)), dim3(kSortThreads), 0, s, c.hist, nk);
    if (n > 0)
        hipLaunchKernelGGL((k_histogram<R, D, T>), dim3(nblk(n)), dim3(kSortThreads), 0, s, c.k,
                           sp.cur, n, sp.key, sp.rank, c.hist);
    const int64_t nb = (nk + kScanChunk - 1) / kScanChunk;
    hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(kSortThreads), 0, s, c.hist, nk,
                       c.scan_part);
    hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(kSortThreads), 0, s, c.scan_part, nb);
    hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nb), dim3(kSortThreads), 0, s, c.hist, nk,
                       c.scan_part);
    constexpr int TPD = D == 3 ? T * T * T : T * T;
    if (n > 0) {
        // final slots, then one scatter into the spare copy, which becomes current
        hipLaunchKernelGGL((k_dest<TPD>), dim3(c.k.ntiles), dim3(TPD), 0, s, c.hist, nk, n, sp.dest);
        hipLaunchKernelGGL((k_scatter_final<R>), dim3(nblk(n)), dim3(kSortThreads), 0, s, sp.cur,
                           sp.alt, n, sp.key, sp.rank, c.hist, sp.dest);
        const PartArrays t = sp.cur;
        sp.cur = sp.alt;
        sp.alt = t;
        sp.swapped ^= 1;
    }
    hipLaunchKernelGGL((k_tile_start<TPD>), dim3(nblk(c.k.ntiles + 1)), dim3(kSortThreads), 0, s,
                       c.hist, c.k.ntiles, n, sp.tile_start);
    sp.sorted = true;
    return hipGetLastError();
}

}  // namespace

hipError_t launch_sort(Ctx& c, Species& sp, hipStream_t s)
{
    if (c.g.precision == PIC_FP64)
        return c.k.dims == 3 ? sort_impl<double, 3, kTile3>(c, sp, s) : sort_impl<double, 2, kTile2>(c, sp, s);
    return c.k.dims == 3 ? sort_impl<float, 3, kTile3>(c, sp, s) : sort_impl<float, 2, kTile2>(c, sp, s);
}

}  // namespace pic
