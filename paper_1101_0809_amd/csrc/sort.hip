// sort.hip -- periodic counting sort of a species by cell, in tile-major cell
// order, so that the particles of one tile (the unit of work of the particle
// kernel) are contiguous.  Inside a tile the order serves the particle
// kernel's LDS banks:
//   3D: the cells are grouped by lane class (see cell_class3) and slot s of
//       the tile's range holds a particle of class s mod C wherever the class
//       counts allow (round g of the tile = one particle of each class); the
//       particles left over by the fuller classes fill the empty places;
//   2D: rank-interleaved -- the particle of rank 0 of every cell, then those
//       of rank 1, and so on, so that consecutive lanes work in distinct cells.
// Histogram with atomics (the returned slot is the particle's rank in its
// cell), exclusive scan of the counts, a per-tile pass computing every
// particle's final slot, the inverse map (which particle fills each slot), and
// one gather of the particle arrays into the spare copy, which becomes
// current.  Not part of the paper's method; it only fixes
// the memory order.
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

// Tile-local key of a 3D cell (T = kTile3): class-major, class k owning keys
// k * T^3 / C .. (k + 1) * T^3 / C - 1.  Each row (ly, lz) of the tile holds at
// most one cell of a class (T < C consecutive x offsets), so the cell's index
// inside its class is the number of earlier rows, in (lz, ly) order, that
// hold a cell of that class.
template <class R>
__device__ __forceinline__ uint32_t class_major_local(int lx, int ly, int lz)
{
    constexpr int T = kTile3, C = lane_classes<R>();
    static_assert(T < C && (T * T * T) % C == 0, "one cell of a class per row, equal classes");
    const int cls = cell_class3<R>(lx, ly, lz);
    uint32_t idx = 0;
    for (int row = 0; row < ly + lz * T; ++row) {
        const int b = cell_class3<R>(0, row % T, row / T);
        idx += ((cls - b) & (C - 1)) < T ? 1u : 0u;
    }
    return (uint32_t)cls * (T * T * T / C) + idx;
}

// Sort key of particle p.  lut (3D, may be null) holds class_major_local of
// the T^3 tile-local cells, x fastest.
template <class R, int D, int T>
__device__ __forceinline__ uint32_t key_of(const GridK& g, const PartArrays& a, int64_t p,
                                           const uint32_t* lut = nullptr)
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
    uint32_t local = ly * T + lx;
    if (D == 3)
        local = lut ? lut[(lz * T + ly) * T + lx] : class_major_local<R>((int)lx, (int)ly, (int)lz);
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

// Histogram of a species that is still grouped by the tiles of its previous
// sort (particles move at most one cell per step): one workgroup per old tile
// range.  Each of its waves takes a contiguous block of the range and counts
// the particles still in that tile per cell in its own LDS counters (a
// wave's atomics rank its lanes in lane order, so the ranks follow the
// storage order), a prefix over the waves orders the blocks, and each cell's
// rank range in the global histogram is reserved with one atomic.  The ranks
// of a cell's particles therefore keep their old order: a particle that did
// not move keeps its place, and the final gather stays a near copy.  A
// particle now in another tile takes its rank from a global atomic directly.
// Ranks stay unique per cell.
constexpr uint32_t kLocalRank = 1u << 31;

template <class R, int D, int T>
__global__ __launch_bounds__(1024) void k_histogram_tiled(GridK g, PartArrays a, const int64_t* __restrict__ ts,
                                                          uint32_t* __restrict__ key, uint32_t* __restrict__ rank,
                                                          uint32_t* __restrict__ hist)
{
    constexpr int TPD = D == 3 ? T * T * T : T * T;
    constexpr int NTH = 1024, NW = NTH / 64, U = 4;  // threads, waves, slots of a lane in flight
    __shared__ uint32_t cnt[NW][TPD];                // per wave, then per wave's first rank
    __shared__ uint32_t lut[D == 3 ? TPD : 1];       // class-major local keys, computed once per tile
    const int t = blockIdx.x;
    const int wv = (int)threadIdx.x >> 6, lane = (int)threadIdx.x & 63;
    const int64_t b = ts[t], e = ts[t + 1];
    const uint32_t k0 = (uint32_t)t * TPD;
    for (int c = threadIdx.x; c < NW * TPD; c += NTH) (&cnt[0][0])[c] = 0;
    for (int c = threadIdx.x; c < TPD; c += NTH)
        if (D == 3) lut[c] = class_major_local<R>(c % T, (c / T) % T, c / (T * T));
    __syncthreads();
    // wave w: slots [b + w L, b + (w + 1) L)
    const int64_t L = (e - b + NW - 1) / NW;
    const int64_t wb = b + wv * L, we = min(e, wb + L);
    for (int64_t p0 = wb + lane; p0 < we; p0 += U * 64) {
        uint32_t k[U];
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (p0 + u * 64 < we) k[u] = key_of<R, D, T>(g, a, p0 + u * 64, D == 3 ? lut : nullptr);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t p = p0 + u * 64;
            if (p >= we) continue;
            key[p] = k[u];
            rank[p] = k[u] - k0 < (uint32_t)TPD ? (kLocalRank | atomicAdd(&cnt[wv][k[u] - k0], 1u))
                                                : atomicAdd(&hist[k[u]], 1u);
        }
    }
    __syncthreads();
    // per cell: the waves' first ranks, then the reservation of the whole range
    for (int c = threadIdx.x; c < TPD; c += NTH) {
        uint32_t run = 0;
        for (int w = 0; w < NW; ++w) {
            const uint32_t m = cnt[w][c];
            cnt[w][c] = run;
            run += m;
        }
        const uint32_t base = run ? atomicAdd(&hist[k0 + c], run) : 0u;
        for (int w = 0; w < NW; ++w) cnt[w][c] += base;
    }
    __syncthreads();
    for (int64_t p = wb + lane; p < we; p += 64) {
        const uint32_t r = rank[p];
        if (r & kLocalRank) rank[p] = cnt[wv][key[p] - k0] + (r & ~kLocalRank);
    }
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
                                              int64_t n, uint32_t* __restrict__ dest,
                                              int64_t* __restrict__ ts)
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
    if (c == 0) ts[blockIdx.x] = base;  // the tile table of the new order
    if (c == 0 && blockIdx.x == gridDim.x - 1) ts[gridDim.x] = n;
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

// 3D: final slot of every particle of one tile in the class-round order,
// written per cell-sorted position as in k_dest.  With n_t particles in the
// tile, slot s belongs to column s mod C, row s / C; column k has rows_k =
// ceil((n_t - k) / C) rows.  The particle of class k and index g within its
// class (cells of the class in key order, then rank) takes row g of column k
// if g < rows_k; the others (classes with more particles than rows), in
// (class, g) order, fill the empty rows of the poorer columns in (column,
// row) order.  The two counts agree: both classes and columns sum to n_t.
template <int C>
__global__ __launch_bounds__(kTile3 * kTile3 * kTile3) void k_dest3(const uint32_t* __restrict__ offs,
                                                                     int64_t nkeys, int64_t n,
                                                                     uint32_t* __restrict__ dest,
                                                                     int64_t* __restrict__ ts)
{
    constexpr int TPD = kTile3 * kTile3 * kTile3;
    constexpr int CPC = TPD / C;  // cells per class
    __shared__ uint32_t ccnt[C], cbase[C], rows[C], hpre[C + 1], lpre[C + 1];
    const int c = threadIdx.x;
    const int64_t k0 = (int64_t)blockIdx.x * TPD;
    const int64_t key = k0 + c;
    const int64_t cb = offs[key];
    const int64_t ce = key + 1 < nkeys ? (int64_t)offs[key + 1] : n;
    const int64_t tb = offs[k0];
    const int64_t te = k0 + TPD < nkeys ? (int64_t)offs[k0 + TPD] : n;
    const int64_t nt = te - tb;
    if (c == 0) ts[blockIdx.x] = tb;  // the tile table of the new order
    if (c == 0 && blockIdx.x == gridDim.x - 1) ts[gridDim.x] = n;
    if (c < C) {
        const int64_t kc = k0 + (int64_t)c * CPC;
        const int64_t b0 = offs[kc];
        const int64_t b1 = kc + CPC < nkeys ? (int64_t)offs[kc + CPC] : n;
        cbase[c] = (uint32_t)(b0 - tb);
        ccnt[c] = (uint32_t)(b1 - b0);
        rows[c] = nt > c ? (uint32_t)((nt - c + C - 1) / C) : 0u;
    }
    __syncthreads();
    if (c == 0) {
        hpre[0] = 0;
        lpre[0] = 0;
        for (int k = 0; k < C; ++k) {
            hpre[k + 1] = hpre[k] + (rows[k] > ccnt[k] ? rows[k] - ccnt[k] : 0u);
            lpre[k + 1] = lpre[k] + (ccnt[k] > rows[k] ? ccnt[k] - rows[k] : 0u);
        }
    }
    __syncthreads();
    const int cls = c / CPC;
    const uint32_t cnt = (uint32_t)(ce - cb);
    const uint32_t g0 = (uint32_t)(cb - tb) - cbase[cls];
    for (uint32_t r = 0; r < cnt; ++r) {
        const uint32_t gi = g0 + r;
        uint32_t slot;
        if (gi < rows[cls]) {
            slot = gi * C + cls;
        } else {
            const uint32_t k = lpre[cls] + (gi - rows[cls]);
            int lam = 0;
            while (lam < C - 1 && hpre[lam + 1] <= k) ++lam;
            slot = (ccnt[lam] + (k - hpre[lam])) * C + lam;
        }
        dest[cb + r] = (uint32_t)(tb + slot);
    }
}

// This workgroup's place in a run of consecutive blocks per XCD: workgroup
// ids are dealt round-robin to the 8 XCDs, so XCD x takes blocks
// [x * per, (x + 1) * per) (one more for the first nb % 8 XCDs), and the
// blocks an XCD runs at a time touch neighbouring memory.
__device__ __forceinline__ int xcd_block()
{
    const int nb = gridDim.x;
    const int per = nb / kXcds, rem = nb % kXcds;
    const int x = blockIdx.x % kXcds, local = blockIdx.x / kXcds;
    return x < rem ? x * (per + 1) + local : rem * (per + 1) + (x - rem) * per + local;
}

// Which particle fills each final slot: the inverse of the final-slot map, by
// one 4-byte scatter, so that the move writes every slot once, in order.
// Each XCD takes a contiguous run of particles: a tile's particles scatter
// into the same few tile ranges of src, whose lines are then written whole
// in one XCD's L2 rather than in pieces by all of them.
__global__ __launch_bounds__(kSortThreads) void k_final_src(int64_t n, const uint32_t* __restrict__ key,
                                                            const uint32_t* __restrict__ rank,
                                                            const uint32_t* __restrict__ offs,
                                                            const uint32_t* __restrict__ dest,
                                                            uint32_t* __restrict__ src)
{
    const int blk = xcd_block();
    const int64_t p = (int64_t)blk * kSortThreads + threadIdx.x;
    if (p >= n) return;
    src[dest[(int64_t)offs[key[p]] + rank[p]]] = (uint32_t)p;
}

// Move the particle arrays: slot q of the spare copy takes particle src[q].
// Writes are coalesced; reads are local, since a particle's new slot is
// mostly in or near the tile range it came from.  Each XCD takes a
// contiguous run of slots, so a tile's reads gather in one XCD's L2.  One
// launch moves one array (A = 0..2 positions, 3..5 momenta, 6 weight, 7 id,
// 8 the FP32 cell): the source lines that the tiles in flight on an XCD
// touch then fit its L2, where all arrays at once would not.  A thread moves
// kGatherU particles, all their loads in flight before the stores.
constexpr int kGatherU = 4;

template <class V, int A>
__device__ __forceinline__ V* gather_array(const PartArrays& P)
{
    return (V*)(A < 3 ? P.pos[A] : (A < 6 ? P.mom[A - 3] : (A == 6 ? P.weight : (A == 7 ? (void*)P.id : (void*)P.cell))));
}

template <class V, int A>
__global__ __launch_bounds__(kSortThreads) void k_gather_final(PartArrays from, PartArrays to, int64_t n,
                                                               const uint32_t* __restrict__ src)
{
    const int blk = xcd_block();
    const int64_t q0 = (int64_t)blk * kSortThreads * kGatherU + threadIdx.x;
    const V* __restrict__ in = gather_array<V, A>(from);
    V* __restrict__ out = gather_array<V, A>(to);
    int64_t p[kGatherU];
#pragma unroll
    for (int u = 0; u < kGatherU; ++u) {
        const int64_t q = q0 + u * kSortThreads;
        p[u] = q < n ? (int64_t)src[q] : -1;
    }
    V v[kGatherU];
#pragma unroll
    for (int u = 0; u < kGatherU; ++u)
        if (p[u] >= 0) v[u] = in[p[u]];
#pragma unroll
    for (int u = 0; u < kGatherU; ++u)
        if (p[u] >= 0) out[q0 + u * kSortThreads] = v[u];
}

template <class R>
void launch_gather_final(const PartArrays& from, const PartArrays& to, int64_t n, const uint32_t* src,
                         hipStream_t s, dim3 grid)
{
    hipLaunchKernelGGL((k_gather_final<R, 0>), grid, dim3(kSortThreads), 0, s, from, to, n, src);
    hipLaunchKernelGGL((k_gather_final<R, 1>), grid, dim3(kSortThreads), 0, s, from, to, n, src);
    hipLaunchKernelGGL((k_gather_final<R, 2>), grid, dim3(kSortThreads), 0, s, from, to, n, src);
    hipLaunchKernelGGL((k_gather_final<R, 3>), grid, dim3(kSortThreads), 0, s, from, to, n, src);
    hipLaunchKernelGGL((k_gather_final<R, 4>), grid, dim3(kSortThreads), 0, s, from, to, n, src);
    hipLaunchKernelGGL((k_gather_final<R, 5>), grid, dim3(kSortThreads), 0, s, from, to, n, src);
    hipLaunchKernelGGL((k_gather_final<R, 6>), grid, dim3(kSortThreads), 0, s, from, to, n, src);
    hipLaunchKernelGGL((k_gather_final<int64_t, 7>), grid, dim3(kSortThreads), 0, s, from, to, n, src);
    if (sizeof(R) == 4)
        hipLaunchKernelGGL((k_gather_final<uint32_t, 8>), grid, dim3(kSortThreads), 0, s, from, to, n, src);
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
    if (n > 0 && sp.sorted)  // still grouped by the tiles of the previous sort
        hipLaunchKernelGGL((k_histogram_tiled<R, D, T>), dim3(c.k.ntiles), dim3(1024), 0, s, c.k,
                           sp.cur, sp.tile_start, sp.key, sp.rank, c.hist);
    else if (n > 0)
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
        // final slots, their inverse, and one gather into the spare copy, which
        // becomes current
        if (D == 3)
            hipLaunchKernelGGL((k_dest3<lane_classes<R>()>), dim3(c.k.ntiles), dim3(TPD), 0, s, c.hist, nk, n,
                               sp.dest, sp.tile_start);
        else
            hipLaunchKernelGGL((k_dest<TPD>), dim3(c.k.ntiles), dim3(TPD), 0, s, c.hist, nk, n, sp.dest,
                               sp.tile_start);
        hipLaunchKernelGGL(k_final_src, dim3(nblk(n)), dim3(kSortThreads), 0, s, n, sp.key, sp.rank, c.hist,
                           sp.dest, sp.src);
        launch_gather_final<R>(sp.cur, sp.alt, n, sp.src, s, dim3(nblk((n + kGatherU - 1) / kGatherU)));
        const PartArrays t = sp.cur;
        sp.cur = sp.alt;
        sp.alt = t;
        sp.swapped ^= 1;
    } else {
        hipLaunchKernelGGL((k_tile_start<TPD>), dim3(nblk(c.k.ntiles + 1)), dim3(kSortThreads), 0, s,
                           c.hist, c.k.ntiles, n, sp.tile_start);
    }
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
