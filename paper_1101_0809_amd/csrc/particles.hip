// particles.hip -- the per-particle hot path of one time step (paper Appendix):
// alternating-order form factor at x^n (Section 4.5), gather of E with the
// alpha weights (Eq. alphax) and of B^n with the beta weights (Eq. betax),
// momentum advance (Eq. p2 and the three-stage split before it), position
// advance (Eq. coordscheme) and the charge-conserving current of Eq. current.
//
// Kernel organisation (one workgroup per cell tile; particles are cell-sorted
// so a tile's particles are contiguous):
//   1. stage E^n and B^n of the tile plus guard cells into LDS (R precision);
//   2. clear an LDS current tile covering the deposit reach plus guards;
//   3. each thread advances particles of the tile; a particle whose cell lies
//      within M cells of its tile (it may have drifted since the last sort)
//      gathers from LDS and deposits with LDS atomics, any other particle uses
//      the same arithmetic on global memory (wrapped indices, global atomics).
//      In 3D a particle that stays in its cell deposits its 54 non-zero
//      contributions at once; one that crosses a cell face is queued and
//      deposited with the full 144-entry window after the loop, by all lanes;
//   4. flush the LDS current tile into the global FP64 J with atomics.
// Precision R = double (FP64 mode: absolute FP64 positions) or float (FP32
// mode: packed int cell + FP32 offset, FP32 gather, push and current
// contributions); the LDS current tile is FP64 in both.
#include "pic_math.h"

namespace pic {
namespace {

// ---------------------------------------------------------------------------
// LDS current storage.  Both precisions accumulate in FP64.  In FP32 mode a
// contribution is the product of two FP32 factors, formed in FP64, where it
// is exact, so the tile sums carry only FP64 rounding (relative 2^-53 per
// add).  This is the compensated accumulation of the FP32
// mode: a hi/lo pair of FP32 arrays updated by two-sum from the atomic's
// returned old value moves the same LDS bytes per contribution but needs the
// round trip of a returning atomic, and measured about ten times slower.
// ---------------------------------------------------------------------------
template <class R, int NJ>
struct LdsJ {
    double v[NJ];
    __device__ __forceinline__ void zero(int i) { v[i] = 0.0; }
    __device__ __forceinline__ void add(int i, double x) { atomicAdd(&v[i], x); }
    __device__ __forceinline__ double get(int i) const { return v[i]; }
};

__device__ __forceinline__ void global_add(double* p, double v)
{
    unsafeAtomicAdd(p, v);
}

// ---------------------------------------------------------------------------
// The 2D3V particle-step kernel (tile kTile2^2, margin kMargin2); every
// particle deposits its window at once.
// ---------------------------------------------------------------------------
template <class R, int D, int T, int M, int NT>
__global__ __launch_bounds__(NT) void k_particle_step(GridK g, StepArgs a, const double* __restrict__ fields,
                                                     const double* __restrict__ bfield, double* __restrict__ Jg)
{
    static_assert(D == 2, "the 3D step is k_particle_step3");
    constexpr int LF = T + 2 + 2 * M;  // field region: cells T0-1-M .. T0+T+M
    constexpr int LJ = T + 4 + 2 * M;  // current region: T0-2-M .. T0+T+1+M
    constexpr int SFY = LF, SFZ = SFY * LF;
    constexpr int NF = D == 3 ? SFZ * LF : LF * LF;
    constexpr int NJ = D == 3 ? LJ * LJ * LJ : LJ * LJ;
    constexpr int SJY = LJ, SJZ = LJ * LJ;
    __shared__ R sf[6 * NF];
    __shared__ LdsJ<R, 3 * NJ> sj;
    __shared__ unsigned int n_fallback;

    const int tile = xcd_tile(blockIdx.x, g.ntiles);
    const int tx = tile % g.nt[0];
    const int ty = (tile / g.nt[0]) % g.nt[1];
    const int tz = D == 3 ? tile / (g.nt[0] * g.nt[1]) : 0;
    const int T0[3] = {tx * T, ty * T, tz * T};
    const int64_t N = g.ncell;
    const int nx = g.n[0], ny = g.n[1], nz = g.n[2];

    // every region index lies in [-n, 2n) unless an axis is shorter than the
    // current region; then the general modulo is used
    const bool small = nx < LJ || ny < LJ || (D == 3 && nz < LJ);
    auto wr = [&](int v, int n) { return small ? wrapi(v, n) : wrap1(v, n); };

    // 1. stage E^n, B^n (+ guard cells) into LDS; B^n is in bfield
    constexpr int NV = D == 3 ? LF * LF * LF : LF * LF;  // values per component
    for (int e = threadIdx.x; e < 6 * NV; e += NT) {
        const int comp = e / NV;
        const int r = e - comp * NV;
        const int lx = r % LF;
        const int ly = (r / LF) % LF;
        const int lz = D == 3 ? r / (LF * LF) : 0;
        const int gx = wr(T0[0] - 1 - M + lx, nx);
        const int gy = wr(T0[1] - 1 - M + ly, ny);
        const int gz = D == 3 ? wr(T0[2] - 1 - M + lz, nz) : 0;
        sf[comp * NF + lx + ly * SFY + lz * SFZ] =
            (R)(comp < 3 ? fields + comp * N : bfield + (comp - 3) * N)[((int64_t)gz * ny + gy) * nx + gx];
    }
    // 2. clear the LDS current tile
    for (int e = threadIdx.x; e < 3 * NJ; e += NT) sj.zero(e);
    if (threadIdx.x == 0) n_fallback = 0;
    __syncthreads();

    const R c = (R)g.c;
    const R c2 = c * c;
    const R qmdt2 = (R)(0.5 * a.qm * g.dt);
    const R cfl[3] = {(R)g.cfl[0], (R)g.cfl[1], (R)g.cfl[2]};
    const R bext[3] = {(R)g.bext[0], (R)g.bext[1], (R)g.bext[2]};
    const int64_t begin = a.tile_start[tile], end = a.tile_start[tile + 1];
    unsigned int my_fallback = 0;

    // 3. particles
    for (int64_t p = begin + threadIdx.x; p < end; p += NT) {
        int i0[3];
        R d0[3];
        PosIO<R, D>::load(a, p, i0, d0);
        R w[3];
        for (int ax = 0; ax < 3; ++ax) w[ax] = ((const R*)a.mom[ax])[p];
        const R qp = (R)a.q * ((const R*)a.weight)[p];

        Axis<R> ax0[3];
        for (int ax = 0; ax < D; ++ax) ax0[ax] = form_factor<R>(d0[ax]);
        if (D == 2) ax0[2] = form_factor<R>(R(0));

        // position relative to the tile, periodic-corrected
        int rel[3];
        bool inside = true;
        for (int ax = 0; ax < D; ++ax) {
            int r = i0[ax] - T0[ax];
            const int n = g.n[ax];
            if (r > n / 2) r -= n;
            if (r < -(n / 2)) r += n;
            rel[ax] = r;
            inside = inside && (r >= -M) && (r <= T - 1 + M);
        }
        if (D == 2) rel[2] = 0;

        R E[3], B[3];
        if (inside) {
            const int base = (rel[0] + 1 + M) + (rel[1] + 1 + M) * SFY +
                             (D == 3 ? (rel[2] + 1 + M) * SFZ : 0);
            auto F = [&](int comp, int da, int db, int dc) -> R {
                return sf[comp * NF + base + da + db * SFY + (D == 3 ? dc * SFZ : 0)];
            };
            if (D == 3) gather3<R>(ax0, F, E, B);
            else gather2<R>(ax0, F, E, B);
        } else {
            ++my_fallback;
            int xi[3], yj[3];
            int64_t zk[3];
            for (int o = 0; o < 3; ++o) {
                xi[o] = wrapi(i0[0] + o - 1, nx);
                yj[o] = wrapi(i0[1] + o - 1, ny) * nx;
                zk[o] = D == 3 ? (int64_t)wrapi(i0[2] + o - 1, nz) * nx * ny : 0;
            }
            auto F = [&](int comp, int da, int db, int dc) -> R {
                return (R)(comp < 3 ? fields + comp * N : bfield + (comp - 3) * N)[zk[dc + 1] + yj[db + 1] + xi[da + 1]];
            };
            if (D == 3) gather3<R>(ax0, F, E, B);
            else gather2<R>(ax0, F, E, B);
        }
        for (int ax = 0; ax < 3; ++ax) B[ax] += bext[ax];

        push<R>(qmdt2, c2, E, B, w);
        for (int ax = 0; ax < 3; ++ax) ((R*)a.mom[ax])[p] = w[ax];

        const R inv = over_sqrt<R>(R(1), w[0] * w[0] + w[1] * w[1] + w[2] * w[2] + c2);
        R disp[3];
        for (int ax = 0; ax < 3; ++ax) disp[ax] = w[ax] * inv * cfl[ax];
        R d1[3];
        int delta[3] = {0, 0, 0};
        PosIO<R, D>::move(a, p, g, i0, d0, disp, d1, delta, true);

        // deposit
        R jfac[3];
        for (int ax = 0; ax < 3; ++ax) jfac[ax] = (R)g.jscale[ax] * qp;
        R dm[3][4], dp[3][4];
        for (int ax = 0; ax < D; ++ax) {
            R s1[3];
            cell_weights<R>(d1[ax], s1);
            window<R>(ax0[ax].s, s1, delta[ax], dm[ax], dp[ax]);
        }
        const R jz2 = D == 2 ? qp * (R)(0.25 * g.inv_vol) * c * w[2] * inv : R(0);
        int s[3];
        for (int ax = 0; ax < 3; ++ax) s[ax] = (ax < D) ? rel[ax] + (delta[ax] < 0 ? -1 : 0) - 1 : 0;

        if (inside) {
            const int jb = (s[0] + 2 + M) + (s[1] + 2 + M) * SJY + (D == 3 ? (s[2] + 2 + M) * SJZ : 0);
            auto S = [&](int comp, int ix, int iy, int iz, double v) {
                sj.add(comp * NJ + jb + ix + iy * SJY + (D == 3 ? iz * SJZ : 0), v);
            };
            if (D == 3) deposit3<R>(dm, dp, jfac, S);
            else deposit2<R>(dm, dp, jfac, jz2, S);
        } else {
            int xi[4], yj[4];
            int64_t zk[4];
            for (int o = 0; o < 4; ++o) {
                xi[o] = wrapi(T0[0] + s[0] + o, nx);
                yj[o] = wrapi(T0[1] + s[1] + o, ny) * nx;
                zk[o] = D == 3 ? (int64_t)wrapi(T0[2] + s[2] + o, nz) * nx * ny : 0;
            }
            auto S = [&](int comp, int ix, int iy, int iz, double v) {
                global_add(&Jg[comp * N + zk[iz] + yj[iy] + xi[ix]], v);
            };
            if (D == 3) deposit3<R>(dm, dp, jfac, S);
            else deposit2<R>(dm, dp, jfac, jz2, S);
        }
    }
    if (my_fallback) atomicAdd(&n_fallback, my_fallback);
    __syncthreads();

    // 4. flush the LDS current tile
    for (int e = threadIdx.x; e < 3 * NJ; e += NT) {
        const double v = sj.get(e);
        if (v == 0.0) continue;
        const int comp = e / NJ;
        const int r = e - comp * NJ;
        const int lx = r % LJ;
        const int ly = (r / LJ) % LJ;
        const int lz = D == 3 ? r / (LJ * LJ) : 0;
        const int gx = wr(T0[0] - 2 - M + lx, nx);
        const int gy = wr(T0[1] - 2 - M + ly, ny);
        const int gz = D == 3 ? wr(T0[2] - 2 - M + lz, nz) : 0;
        global_add(&Jg[comp * N + ((int64_t)gz * ny + gy) * nx + gx], v);
    }
    if (threadIdx.x == 0 && a.counters) {
        atomicAdd(&a.counters[1], (unsigned long long)n_fallback);
        atomicAdd(&a.counters[2], (unsigned long long)(end - begin));
    }
}

// ---------------------------------------------------------------------------
// The 3D particle-step kernel (tile kTile3^3; layout Tile3<R>).
//
// LDS: the field tile holds E^n and B^n on the tile plus its margin and the
// stencil: cells T0-1-MX .. T0+T+MX along x and T0-1-M .. T0+T+M along y and
// z, in rows of FROW values and planes of FPLANE; the components that are
// node-centred in z (E^z, B^x, B^y) never read the first plane and store
// planes 1..11 only.  The FP64 current tile covers T0-2-MX .. T0+T+1+MX along
// x and T0-2-M .. T0+T+1+M along y and z, rows of JROW, planes of JPLANE.  A
// cell's field and current base indices share their residue modulo 32, and
// that residue modulo C (16 in FP64, 32 in FP32) is the cell's lane class.
// Lanes of one LDS pass that hold cells of distinct classes read and add in
// distinct banks.
//
// Each wave takes chunks of 64 KC consecutive storage slots (chunks w, w + NW,
// ... of the tile), so every load and store of a chunk stays within a few
// cache lines per array however far the particles have drifted since the last
// sort, and orders its own chunk without a workgroup barrier:
//   (a) every slot's cell is classified (its load was issued during the
//       previous chunk).  A particle inside the tile region takes a rank among
//       the chunk's particles of its class (LDS counter per wave and class);
//       any other particle has left the region: it joins the tile's migrant
//       list with its rank among the migrants to its neighbour tile (one
//       further away takes a bucket slot at once);
//   (b) one ballot per rank r < 16 gives row r, the classes with more than r
//       particles in the chunk, so a row holds distinct classes;
//   (c) each particle's place is its row's start plus the number of smaller
//       classes in the row (ranks from 16 on follow the rows), written into
//       the wave's permutation of the chunk;
//   (d) lane t advances the particle at place t, t + 64, ...: gather (LDS),
//       push, move (state stored), and, if it stays in its cell, its 54
//       non-zero current contributions; a particle that crosses a cell face
//       is appended to the crossing queue, with its place in a class map
//       (column = class of its window's first cell).
// After the chunks, the migrants go into the buckets of their new tiles (one
// global reservation per neighbour tile), those whose bucket was full are
// advanced with global memory (gather from the grid, global atomics), and the
// crossing pass deposits the queued windows in class-map order, in sections by
// crossing axis (74 contributions for one axis, 144 for several); the entries
// a full map column could not take follow in arrival order.  Last, the
// non-zero current entries are flushed with global FP64 atomics.  The spare
// particle copy holds the crossing queue and the migrant lists (idle between
// sorts); the sort scratch holds the buckets.
// ---------------------------------------------------------------------------
__host__ __device__ constexpr int fplane0(int comp)  // first stored plane of a field component
{
    return comp < 2 ? 12 * comp : (comp < 5 ? 24 + 11 * (comp - 2) : 57);
}
__host__ __device__ constexpr int fnodez(int comp) { return comp >= 2 && comp <= 4 ? 1 : 0; }
// Lowest offset of the gather stencil of a component along an axis: 0 where
// the component takes node factors along it (two points), -1 where it takes
// cell factors (three points).
__host__ __device__ constexpr int lo_offset(int comp, int ax)
{
    // bit ax set: node factors along ax (E^x, E^y, E^z, B^x, B^y, B^z)
    const int node = comp == 0 ? 1 : comp == 1 ? 2 : comp == 2 ? 4 : comp == 3 ? 6 : comp == 4 ? 5 : 3;
    return (node >> ax) & 1 ? 0 : -1;
}
constexpr int kFieldPlanes3 = 69;  // 12 + 12 + 11 + 11 + 11 + 12
constexpr int64_t kUnmapped = (int64_t)1 << 62;  // crossing entry not in the class map
// A migrant bucket this full is advanced with LDS tiles.  Staging the tile and
// flushing its current cost about as much as 8 particles on the global path
// (144 global atomics each).
constexpr unsigned kMigLds = 8;

// Stage E^n and B^n of the 3D tile region into LDS.  The region is a set of
// rows of at most 16 x values (69 stored planes x LFY rows): 16 lanes take a
// row, each lane one x column, so a lane wraps its x coordinate once and
// each row is decoded once.  SK rows' loads of a thread are in flight before
// their stores (one load at a time would wait out the memory latency once per
// value).
template <class R, int NT>
__device__ __forceinline__ void stage_fields3(const GridK& g, const int T0[3], const double* __restrict__ fields,
                                              const double* __restrict__ bfield, R* sf, bool small)
{
    using TL = Tile3Dims<R>;
    constexpr int MX = TL::MX, M = TL::M, LFX = TL::LFX, LFY = TL::LFY;
    constexpr int SFY = TL::FROW, SFZ = TL::FPLANE;
    constexpr int RPP = NT / 16;                 // rows per pass of the workgroup
    constexpr int NROWS = kFieldPlanes3 * LFY;  // (stored plane, row) pairs
    constexpr int SK = 7;
    static_assert(LFX <= 16 && NT % 64 == 0, "a field-tile row fits 16 lanes");
    const int64_t N = g.ncell;
    const int nx = g.n[0], ny = g.n[1], nz = g.n[2];
    auto wr = [&](int v, int n) { return small ? wrapi(v, n) : wrap1(v, n); };
    const int lx = (int)threadIdx.x & 15;
    const int gx = wr(T0[0] - 1 - MX + (lx < LFX ? lx : 0), nx);
    for (int r0 = lx < LFX ? (int)threadIdx.x >> 4 : NROWS; r0 < NROWS; r0 += SK * RPP) {
        double v[SK];
        int li[SK];
#pragma unroll
        for (int u = 0; u < SK; ++u) {
            const int r = r0 + u * RPP;
            li[u] = -1;
            if (r < NROWS) {
                const int pl = r / LFY;
                const int ly = r - pl * LFY;
                const int comp = pl < 12 ? 0 : (pl < 24 ? 1 : (pl < 35 ? 2 : (pl < 46 ? 3 : (pl < 57 ? 4 : 5))));
                const int lz = pl - fplane0(comp) + fnodez(comp);
                const int gy = wr(T0[1] - 1 - M + ly, ny);
                const int gz = wr(T0[2] - 1 - M + lz, nz);
                v[u] = (comp < 3 ? fields + comp * N : bfield + (comp - 3) * N)[((int64_t)gz * ny + gy) * nx + gx];
                li[u] = pl * SFZ + ly * SFY + lx;
            }
        }
#pragma unroll
        for (int u = 0; u < SK; ++u)
            if (li[u] >= 0) sf[li[u]] = (R)v[u];
    }
}

// Flush the LDS current tile of a 3D tile into the grid's J: 16 lanes per
// row of the tile, one x column each (the padding is never written); the
// columns of a row beyond 16 (FP32 mode's wider margin) follow, one (row,
// column) pair per thread.  Only the non-zero entries take a global atomic.
template <class R, int NT, class LJT>
__device__ __forceinline__ void flush_current3(const GridK& g, const int T0[3], const LJT& sj,
                                               double* __restrict__ Jg, bool small)
{
    using TL = Tile3Dims<R>;
    constexpr int MX = TL::MX, M = TL::M, LJX = TL::LJX, LJY = TL::LJY;
    constexpr int SJY = TL::JROW, SJZ = TL::JPLANE;
    constexpr int NJ = TL::NJ;
    constexpr int RPP = NT / 16;
    constexpr int NROWS = 3 * LJY * LJY;  // (component, plane, row)
    constexpr int XT = LJX > 16 ? LJX - 16 : 0;  // columns beyond the 16-lane rows
    static_assert(LJX <= 32 && NT % 64 == 0, "a current-tile row fits 16 lanes plus a tail");
    const int64_t N = g.ncell;
    const int nx = g.n[0], ny = g.n[1], nz = g.n[2];
    auto wr = [&](int v, int n) { return small ? wrapi(v, n) : wrap1(v, n); };
    auto one = [&](int r, int lx, int gx) {
        const int comp = r / (LJY * LJY);
        const int rr = r - comp * (LJY * LJY);
        const int lz = rr / LJY;
        const int ly = rr - lz * LJY;
        const double v = sj.get(comp * NJ + lz * SJZ + ly * SJY + lx);
        if (v == 0.0) return;
        const int gy = wr(T0[1] - 2 - M + ly, ny);
        const int gz = wr(T0[2] - 2 - M + lz, nz);
        global_add(&Jg[comp * N + ((int64_t)gz * ny + gy) * nx + gx], v);
    };
    const int lx = (int)threadIdx.x & 15;
    const int gx = wr(T0[0] - 2 - MX + (lx < LJX ? lx : 0), nx);
    for (int r = lx < LJX ? (int)threadIdx.x >> 4 : NROWS; r < NROWS; r += RPP) one(r, lx, gx);
    if (XT > 0)
        for (int e = threadIdx.x; e < NROWS * XT; e += NT) {
            const int r = e / (XT > 0 ? XT : 1);
            const int cx = 16 + (e - r * XT);
            one(r, cx, wr(T0[0] - 2 - MX + cx, nx));
        }
}

// Position of cell i0 relative to the tile at T0, periodic-corrected; true if
// within the tile's margins (MX along x, M along y and z: inside its LDS
// regions).
template <class R>
__device__ __forceinline__ bool relative3(const GridK& g, const int T0[3], const int i0[3], int rel[3])
{
    constexpr int T = kTile3;
    bool in = true;
    for (int ax = 0; ax < 3; ++ax) {
        const int m = ax == 0 ? Tile3<R>::MX : Tile3<R>::M;
        int r = i0[ax] - T0[ax];
        const int n = g.n[ax];
        if (r > n / 2) r -= n;
        if (r < -(n / 2)) r += n;
        rel[ax] = r;
        in = in && (r >= -m) && (r <= T - 1 + m);
    }
    return in;
}

// Tile that holds cell i (clamped into the grid, so that any input names a tile).
__device__ __forceinline__ int tile_of3(const GridK& g, const int i[3])
{
    int t[3];
    for (int ax = 0; ax < 3; ++ax) {
        const int c = i[ax] < 0 ? 0 : (i[ax] >= g.n[ax] ? g.n[ax] - 1 : i[ax]);
        t[ax] = c / kTile3;
    }
    return (t[2] * g.nt[1] + t[1]) * g.nt[0] + t[0];
}

// Code (ox+1) + 3(oy+1) + 9(oz+1) of the tile that holds cell i, at tile offset
// (ox, oy, oz) in {-1, 0, 1}^3 from tile (tx, ty, tz) with periodic wrap, or -1
// if it is further away.
__device__ __forceinline__ int neighbour_code3(const GridK& g, int tx, int ty, int tz, const int i[3])
{
    int c[3];
    for (int ax = 0; ax < 3; ++ax) c[ax] = i[ax] < 0 ? 0 : (i[ax] >= g.n[ax] ? g.n[ax] - 1 : i[ax]);
    const int t[3] = {tx, ty, tz};
    int code = 0, mul = 1;
    for (int ax = 0; ax < 3; ++ax) {
        const int nt = g.nt[ax];
        int o = c[ax] / kTile3 - t[ax];
        if (o > nt / 2) o -= nt;
        if (o < -(nt / 2)) o += nt;
        if (o < -1 || o > 1) return -1;
        code += (o + 1) * mul;
        mul *= 3;
    }
    return code;
}

// The tile at neighbour code `code` of tile (tx, ty, tz).
__device__ __forceinline__ int neighbour_tile3(const GridK& g, int tx, int ty, int tz, int code)
{
    const int t[3] = {tx, ty, tz};
    int d[3];
    for (int ax = 0; ax < 3; ++ax) {
        const int nt = g.nt[ax];
        int v = t[ax] + code % 3 - 1;
        code /= 3;
        d[ax] = v < 0 ? v + nt : (v >= nt ? v - nt : v);
    }
    return (d[2] * g.nt[1] + d[1]) * g.nt[0] + d[0];
}

// Gather from the LDS field tile, push and move one particle whose cell is at
// rel (inside the tile region); stores w and the new position.  Returns the
// start form factors, the end offsets, the cell shift and the macro charge.
template <class R>
__device__ __forceinline__ void advance_lds3(const GridK& g, const StepArgs& a, const R* sf, int64_t p,
                                             const int i0[3], const R d0[3], const int rel[3], Axis<R> (&ax0)[3],
                                             R d1[3], int delta[3], R& qp)
{
    using TL = Tile3<R>;
    constexpr int MX = TL::MX, M = TL::M;
    constexpr int SFY = TL::FROW, SFZ = TL::FPLANE;
    R w[3];
    for (int ax = 0; ax < 3; ++ax) w[ax] = ((const R*)a.mom[ax])[p];
    qp = (R)a.q * ((const R*)a.weight)[p];
    for (int ax = 0; ax < 3; ++ax) ax0[ax] = form_factor<R>(d0[ax]);
    R E[3], B[3];
    const int base = (rel[0] + 1 + MX) + (rel[1] + 1 + M) * SFY + (rel[2] + 1 + M) * SFZ;
    // One base register per component at the lowest point of its stencil,
    // and a second two planes up where the stencil spans three z planes:
    // every point is then a small immediate offset of a base (a paired LDS
    // read reaches 255 elements), where the compiler would otherwise derive
    // a new base for most rows.
    using LP = __attribute__((address_space(3))) const R*;
    LP lo[6], hi[6];
#pragma unroll
    for (int comp = 0; comp < 6; ++comp) {
        const int c0 = (fplane0(comp) - fnodez(comp)) * SFZ + base + lo_offset(comp, 0) +
                       lo_offset(comp, 1) * SFY + lo_offset(comp, 2) * SFZ;
        lo[comp] = (LP)(sf + c0);
        asm("" : "+v"(lo[comp]));
        if (!fnodez(comp)) {
            hi[comp] = (LP)(sf + c0 + 2 * SFZ);
            asm("" : "+v"(hi[comp]));
        }
    }
    static_assert(2 + 2 * SFY + SFZ <= 255, "a stencil's two lower z planes in reach of one base");
    auto F = [&](int comp, int da, int db, int dc) -> R {
        const int a = da - lo_offset(comp, 0), b = db - lo_offset(comp, 1), c = dc - lo_offset(comp, 2);
        return c == 2 ? hi[comp][a + b * SFY] : lo[comp][a + b * SFY + c * SFZ];
    };
    gather3<R>(ax0, F, E, B);
    for (int ax = 0; ax < 3; ++ax) B[ax] += (R)g.bext[ax];
    const R c2 = (R)g.c * (R)g.c;
    push<R>((R)(0.5 * a.qm * g.dt), c2, E, B, w);
    for (int ax = 0; ax < 3; ++ax) ((R*)a.mom[ax])[p] = w[ax];
    const R inv = over_sqrt<R>(R(1), w[0] * w[0] + w[1] * w[1] + w[2] * w[2] + c2);
    R disp[3];
    for (int ax = 0; ax < 3; ++ax) disp[ax] = w[ax] * inv * (R)g.cfl[ax];
    for (int ax = 0; ax < 3; ++ax) delta[ax] = 0;
    PosIO<R, 3>::move(a, p, g, i0, d0, disp, d1, delta, true);
}

// The whole step of one particle on global memory: gather from the grid
// (wrapped indices), push, move, and the full current window with global
// atomics.  Correct for any position; used only where the LDS tiles do not
// cover the particle.
template <class R>
__device__ __forceinline__ void advance_global3(const GridK& g, const StepArgs& a, int64_t p,
                                                const double* __restrict__ fields,
                                                const double* __restrict__ bfield, double* __restrict__ Jg)
{
    const int64_t N = g.ncell;
    const int nx = g.n[0], ny = g.n[1], nz = g.n[2];
    int i0[3];
    R d0[3];
    PosIO<R, 3>::load(a, p, i0, d0);
    R w[3];
    for (int ax = 0; ax < 3; ++ax) w[ax] = ((const R*)a.mom[ax])[p];
    const R qp = (R)a.q * ((const R*)a.weight)[p];
    Axis<R> ax0[3];
    for (int ax = 0; ax < 3; ++ax) ax0[ax] = form_factor<R>(d0[ax]);
    R E[3], B[3];
    {
        int xi[3], yj[3];
        int64_t zk[3];
        for (int o = 0; o < 3; ++o) {
            xi[o] = wrapi(i0[0] + o - 1, nx);
            yj[o] = wrapi(i0[1] + o - 1, ny) * nx;
            zk[o] = (int64_t)wrapi(i0[2] + o - 1, nz) * nx * ny;
        }
        auto F = [&](int comp, int da, int db, int dc) -> R {
            return (R)(comp < 3 ? fields + comp * N : bfield + (comp - 3) * N)[zk[dc + 1] + yj[db + 1] + xi[da + 1]];
        };
        gather3<R>(ax0, F, E, B);
    }
    for (int ax = 0; ax < 3; ++ax) B[ax] += (R)g.bext[ax];
    const R c2 = (R)g.c * (R)g.c;
    push<R>((R)(0.5 * a.qm * g.dt), c2, E, B, w);
    for (int ax = 0; ax < 3; ++ax) ((R*)a.mom[ax])[p] = w[ax];
    const R inv = over_sqrt<R>(R(1), w[0] * w[0] + w[1] * w[1] + w[2] * w[2] + c2);
    R disp[3];
    for (int ax = 0; ax < 3; ++ax) disp[ax] = w[ax] * inv * (R)g.cfl[ax];
    R d1[3];
    int delta[3] = {0, 0, 0};
    PosIO<R, 3>::move(a, p, g, i0, d0, disp, d1, delta, true);
    R jfac[3];
    for (int ax = 0; ax < 3; ++ax) jfac[ax] = (R)g.jscale[ax] * qp;
    R dm[3][4], dp[3][4];
    for (int ax = 0; ax < 3; ++ax) {
        R s1[3];
        cell_weights<R>(d1[ax], s1);
        window<R>(ax0[ax].s, s1, delta[ax], dm[ax], dp[ax]);
    }
    int xi[4], yj[4];
    int64_t zk[4];
    for (int o = 0; o < 4; ++o) {
        xi[o] = wrapi(i0[0] + (delta[0] < 0 ? -1 : 0) - 1 + o, nx);
        yj[o] = wrapi(i0[1] + (delta[1] < 0 ? -1 : 0) - 1 + o, ny) * nx;
        zk[o] = (int64_t)wrapi(i0[2] + (delta[2] < 0 ? -1 : 0) - 1 + o, nz) * nx * ny;
    }
    auto S = [&](int comp, int ix, int iy, int iz, double v) {
        global_add(&Jg[comp * N + zk[iz] + yj[iy] + xi[ix]], v);
    };
    deposit3<R>(dm, dp, jfac, S);
}

template <class R, int NT, int KC>
__global__ __launch_bounds__(NT) void k_particle_step3(GridK g, StepArgs a, const double* __restrict__ fields,
                                                      const double* __restrict__ bfield, double* __restrict__ Jg)
{
    constexpr int NW = NT / 64;  // waves
    constexpr int WCH = 64 * KC;  // slots per wave chunk
    // class rows ordered per wave chunk; higher ranks follow in arrival order.
    // A chunk averages 4 (FP64) or 6 (FP32) particles per class; a class
    // fills more than 10, or 12, rows in under 1% of chunks.
    constexpr int RW = 64 * KC / lane_classes<R>() >= 6 ? 12 : 10;
    using TL = Tile3Dims<R>;
    constexpr int T = kTile3, MX = TL::MX, M = TL::M;  // margins along x; along y and z
    constexpr int LJX = TL::LJX, LJY = TL::LJY;  // current region: T0-2-M .. T0+T+1+M per axis
    constexpr int SJY = TL::JROW, SJZ = TL::JPLANE;
    constexpr int NJ = TL::NJ;  // per current component
    constexpr int C = lane_classes<R>();
    constexpr int CJ = 16;  // classes of the FP64 current tile
    constexpr unsigned kRankBits = 27;  // migrant list entry: rank | neighbour code << 27
    constexpr uint32_t kPlaced = 0xffffffffu;  // migrant list entry already in its bucket (code 31)
    static_assert(NT % 256 == 0 && WCH <= 256 && C <= 32, "wave chunk layout");
    static_assert(TL::LFY == 12 && fplane0(5) + 12 == kFieldPlanes3, "z planes of the 3D field tile");
    __shared__ R sf[kFieldPlanes3 * TL::FPLANE];
    __shared__ LdsJ<R, 3 * NJ> sj;
    __shared__ unsigned int wcnt[NW][C];   // per wave: particles of each class in its chunk
    __shared__ uint8_t wperm[NW][WCH];     // per wave: chunk position -> slot offset in the chunk
    __shared__ unsigned int wtail[NW];     // per wave: ranks beyond the ordered rows
    __shared__ unsigned int mg_n[27];      // migrants of the tile per neighbour tile
    __shared__ unsigned int mg_base[27];   // their first bucket slot
    __shared__ unsigned int ml_n;          // migrant list length
    __shared__ unsigned int qc_n[4 * CJ];  // crossing map: 4 sections (axis 0, 1, 2, several) x CJ classes
    __shared__ unsigned int qc_total, qc_unmapped;
    __shared__ unsigned int qo_n;  // migrants whose bucket was full
    __shared__ unsigned int n_migrant;

    const int tile = xcd_tile(blockIdx.x, g.ntiles);
    const int tx = tile % g.nt[0];
    const int ty = (tile / g.nt[0]) % g.nt[1];
    const int tz = tile / (g.nt[0] * g.nt[1]);
    const int T0[3] = {tx * T, ty * T, tz * T};
    const bool small = g.n[0] < LJX || g.n[1] < LJY || g.n[2] < LJY;
    const int wv = (int)threadIdx.x >> 6, lane = (int)threadIdx.x & 63;
    const int64_t begin = a.tile_start[tile], end = a.tile_start[tile + 1];
    if (begin == end) return;  // no particle: nothing to stage, deposit or count (the whole workgroup)

    // 1. stage E^n and B^n (B^n from bfield) into LDS
    stage_fields3<R, NT>(g, T0, fields, bfield, sf, small);
    // 2. clear the LDS current tile, the class counts and the queue counters
    for (int e = threadIdx.x; e < 3 * NJ; e += NT) sj.zero(e);
    if (lane < C) wcnt[wv][lane] = 0;
    if (threadIdx.x < 27) mg_n[threadIdx.x] = 0;
    if (threadIdx.x < 4 * CJ) qc_n[threadIdx.x] = 0;
    if (threadIdx.x == 0) {
        qc_total = 0;
        qc_unmapped = 0;
        qo_n = 0;
        n_migrant = 0;
        ml_n = 0;
    }
    __syncthreads();

    const int nt = (int)(end - begin);
    const unsigned capc = (unsigned)(nt / (4 * CJ));
    uint32_t* qmap = (uint32_t*)a.qmap + begin;
    uint32_t* qother = (uint32_t*)a.qother + begin;
    uint32_t* mslot = (uint32_t*)a.mlist + begin;   // migrant list: slot offsets
    uint32_t* mword = (uint32_t*)a.mlist2 + begin;  // migrant list: rank | code << 27
    unsigned my_migrant = 0;

    // Classify slot sl (cell ci): true if its cell lies in the tile region,
    // with its lane class; otherwise the particle joins the tile's migrant
    // list, whose entries are placed after the particle loop (a wave with one
    // migrant would otherwise run the whole placement with its other lanes
    // idle).
    auto classify = [&](int sl, const int ci[3], int& cls) -> bool {
        int rel[3];
        if (relative3<R>(g, T0, ci, rel)) {
            cls = cell_class3<R>(rel[0], rel[1], rel[2]);
            return true;
        }
        mslot[atomicAdd(&ml_n, 1u)] = (uint32_t)sl;
        return false;
    };

    // Advance particle p, whose cell lies in the tile region: gather (LDS),
    // push, move (state stored); a particle that stays in its cell deposits
    // its 54 non-zero contributions, one that crosses a cell face is queued:
    // its entry densely, in arrival order, and its place in the class map.
    // Every lane of the wave that calls it must call it (the queue uses the
    // wave's ballot); `active` false makes a lane a no-op.
    auto advance = [&](int64_t p, bool active) {
        bool still = true;
        int rel[3] = {0, 0, 0}, delta[3] = {0, 0, 0};
        R d0[3] = {0, 0, 0};
        if (active) {
            int i0[3];
            PosIO<R, 3>::load(a, p, i0, d0);
            relative3<R>(g, T0, i0, rel);
            Axis<R> ax0[3];
            R d1[3], qp;
            advance_lds3<R>(g, a, sf, p, i0, d0, rel, ax0, d1, delta, qp);
            still = (delta[0] | delta[1] | delta[2]) == 0;
            if (still) {
                R jfac[3];
                for (int ax = 0; ax < 3; ++ax) jfac[ax] = (R)g.jscale[ax] * qp;
                R s1[3][3], s0[3][3];
                for (int ax = 0; ax < 3; ++ax) {
                    cell_weights<R>(d1[ax], s1[ax]);
                    for (int k = 0; k < 3; ++k) s0[ax][k] = ax0[ax].s[k];
                }
                const int jb = (rel[0] + 1 + MX) + (rel[1] + 1 + M) * SJY + (rel[2] + 1 + M) * SJZ;
                auto S = [&](int comp, int ix, int iy, int iz, double v) {
                    sj.add(comp * NJ + jb + ix + iy * SJY + iz * SJZ, v);
                };
                deposit3_still<R>(s0, s1, jfac, S);
            }
        }
        const unsigned long long mask = __ballot(!still);
        if (!mask) return;
        const int leader = __ffsll((long long)mask) - 1;
        unsigned int qbase = 0;
        if (lane == leader) qbase = atomicAdd(&qc_total, (unsigned int)__popcll(mask));
        qbase = __shfl(qbase, leader, 64);
        if (still) return;
        const unsigned e = qbase + (unsigned)__popcll(mask & ((1ull << lane) - 1ull));
        for (int ax = 0; ax < 3; ++ax) ((R*)a.qd0[ax])[begin + e] = d0[ax];
        int64_t word = p - begin;
        for (int ax = 0; ax < 3; ++ax) {
            word |= (int64_t)(rel[ax] + (ax == 0 ? MX : M)) << (32 + 4 * ax);
            word |= (int64_t)(delta[ax] + 1) << (44 + 2 * ax);
        }
        // map section: the crossing axis if there is one, 3 if several
        const int nax = (delta[0] != 0) + (delta[1] != 0) + (delta[2] != 0);
        const int sec = nax == 1 ? (delta[0] != 0 ? 0 : (delta[1] != 0 ? 1 : 2)) : 3;
        int sw[3];
        for (int ax = 0; ax < 3; ++ax) sw[ax] = rel[ax] + (delta[ax] < 0 ? -1 : 0) - 1;
        const int jw = (sw[0] + 2 + MX) + (sw[1] + 2 + M) * SJY + (sw[2] + 2 + M) * SJZ;
        const int col = sec * CJ + (jw & (CJ - 1));
        const unsigned r = atomicAdd(&qc_n[col], 1u);
        if (r < capc) {
            qmap[col + 4 * CJ * r] = e;
        } else {
            word |= kUnmapped;
            atomicAdd(&qc_unmapped, 1u);
        }
        a.qword[begin + e] = word;
    };

    // 3. wave chunks: wave w takes chunks w, w + NW, ... of WCH slots;
    //    lane l the slots l + 64 u.  No workgroup barrier inside the loop:
    //    the class order of a chunk is the wave's own, in its own rows.
    int ci[KC][3];
#pragma unroll
    for (int u = 0; u < KC; ++u)
        if (wv * WCH + lane + 64 * u < nt) PosIO<R, 3>::cell(a, begin + wv * WCH + lane + 64 * u, ci[u]);
    for (int cb = wv * WCH; cb < nt; cb += NW * WCH) {
        // (a) classify
        int cls[KC];
        unsigned rk[KC];
        bool in[KC];
#pragma unroll
        for (int u = 0; u < KC; ++u) {
            const int sl = cb + lane + 64 * u;
            cls[u] = 0;
            rk[u] = 0;
            in[u] = sl < nt && classify(sl, ci[u], cls[u]);
            if (in[u]) rk[u] = atomicAdd(&wcnt[wv][cls[u]], 1u);
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        __builtin_amdgcn_wave_barrier();
        // (b) class rows: row r holds the rank-r particle of each class
        //     that has one; lane r keeps row r's class mask and first position
        const unsigned mycnt = lane < C ? wcnt[wv][lane] : 0u;
        uint32_t rmask = 0;
        unsigned rstart = 0, rows = 0;
#pragma unroll
        for (int r = 0; r < RW; ++r) {
            const uint32_t m = (uint32_t)__ballot(mycnt > (unsigned)r);
            rmask = lane == r ? m : rmask;
            rstart = lane == r ? rows : rstart;
            rows += (unsigned)__popc(m);
        }
        if (lane < C) wcnt[wv][lane] = 0;
        if (lane == 0) wtail[wv] = 0;
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        __builtin_amdgcn_wave_barrier();
        // (c) chunk order
#pragma unroll
        for (int u = 0; u < KC; ++u) {
            const int rsel = in[u] && rk[u] < (unsigned)RW ? (int)rk[u] : 0;
            const uint32_t m = (uint32_t)__shfl((int)rmask, rsel, 64);
            const unsigned st = (unsigned)__shfl((int)rstart, rsel, 64);
            if (in[u]) {
                const unsigned pos = rk[u] < (unsigned)RW ? st + (unsigned)__popc(m & ((1u << cls[u]) - 1u))
                                                          : rows + atomicAdd(&wtail[wv], 1u);
                wperm[wv][pos] = (uint8_t)(lane + 64 * u);
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        __builtin_amdgcn_wave_barrier();
        const int ninside = (int)(rows + wtail[wv]);
        // the next chunk's cells load while this chunk is advanced
#pragma unroll
        for (int u = 0; u < KC; ++u) {
            const int nsl = cb + NW * WCH + lane + 64 * u;
            if (nsl < nt) PosIO<R, 3>::cell(a, begin + nsl, ci[u]);
        }
        // (d) advance: lane t takes chunk positions t, t + 64, ...
        for (int q0 = 0; q0 < ninside; q0 += 64) {
            const int q = q0 + lane;
            advance(begin + cb + (q < ninside ? wperm[wv][q] : 0), q < ninside);
        }
    }
    __syncthreads();
    // The tile's migrants into the buckets of their new tiles.  First each
    // migrant's rank among those to its neighbour tile (a tile further away
    // takes its bucket slot at once); then one reservation per neighbour
    // tile; then the bucket entries.
    for (int e = threadIdx.x; e < (int)ml_n; e += NT) {
        const uint32_t sl = mslot[e];
        int ci[3];
        PosIO<R, 3>::cell(a, begin + sl, ci);
        const int code = neighbour_code3(g, tx, ty, tz, ci);
        const unsigned r = code >= 0 ? atomicAdd(&mg_n[code], 1u) : 0u;
        if (code >= 0 && r < (1u << kRankBits)) {
            mword[e] = r | ((uint32_t)code << kRankBits);
            continue;
        }
        mword[e] = kPlaced;
        const int dt = tile_of3(g, ci);
        const unsigned rr = atomicAdd(&a.mig_n[dt], 1u);
        if (rr < a.mig_cap) {
            a.mig[(int64_t)dt * a.mig_cap + rr] = (uint32_t)(begin + sl);
            ++my_migrant;
        } else {
            qother[atomicAdd(&qo_n, 1u)] = sl;
        }
    }
    __syncthreads();
    if (threadIdx.x < 27 && mg_n[threadIdx.x])
        mg_base[threadIdx.x] = atomicAdd(&a.mig_n[neighbour_tile3(g, tx, ty, tz, threadIdx.x)], mg_n[threadIdx.x]);
    __syncthreads();
    for (int e = threadIdx.x; e < (int)ml_n; e += NT) {
        const uint32_t word = mword[e];
        if (word == kPlaced) continue;
        const int code = (int)(word >> kRankBits);
        const unsigned r = mg_base[code] + (word & ((1u << kRankBits) - 1u));
        if (r < a.mig_cap) {
            a.mig[(int64_t)neighbour_tile3(g, tx, ty, tz, code) * a.mig_cap + r] = (uint32_t)(begin + mslot[e]);
            ++my_migrant;
        } else {
            qother[atomicAdd(&qo_n, 1u)] = mslot[e];
        }
    }
    if (my_migrant) atomicAdd(&n_migrant, my_migrant);
    __syncthreads();

    // 4. migrants whose bucket was full: global memory
    for (int q = threadIdx.x; q < (int)qo_n; q += NT)
        advance_global3<R>(g, a, begin + qother[q], fields, bfield, Jg);

    // 5. pass 3: the crossing queue -- the class map's four sections, then,
    //    only if a map column was full, the unmapped entries in arrival order
    {
        auto cross = [&](int64_t e, int sec) {
            const int64_t word = a.qword[e];
            const int64_t p = begin + (word & 0xffffffffll);
            int rel[3], delta[3];
            R d0[3], d1[3];
            for (int ax = 0; ax < 3; ++ax) {
                rel[ax] = (int)((word >> (32 + 4 * ax)) & 15) - (ax == 0 ? MX : M);
                delta[ax] = (int)((word >> (44 + 2 * ax)) & 3) - 1;
                d0[ax] = ((const R*)a.qd0[ax])[e];
                if (sizeof(R) == 8) {  // the stored end position, as in PosIO::move
                    const double x = ((const double*)a.pos[ax])[p];
                    d1[ax] = (R)(x - floor(x));
                } else {
                    d1[ax] = ((const R*)a.pos[ax])[p];
                }
            }
            const R qp = (R)a.q * ((const R*)a.weight)[p];
            R jfac[3];
            for (int ax = 0; ax < 3; ++ax) jfac[ax] = (R)g.jscale[ax] * qp;
            R dm[3][4], dp[3][4];
            for (int ax = 0; ax < 3; ++ax) {
                R s0[3], s1[3];
                cell_weights<R>(d0[ax], s0);
                cell_weights<R>(d1[ax], s1);
                window<R>(s0, s1, delta[ax], dm[ax], dp[ax]);
            }
            int sw[3];
            for (int ax = 0; ax < 3; ++ax) sw[ax] = rel[ax] + (delta[ax] < 0 ? -1 : 0) - 1;
            const int jb = (sw[0] + 2 + MX) + (sw[1] + 2 + M) * SJY + (sw[2] + 2 + M) * SJZ;
            auto S = [&](int comp, int ix, int iy, int iz, double v) {
                sj.add(comp * NJ + jb + ix + iy * SJY + iz * SJZ, v);
            };
            if (sec == 0) deposit3_axis<0, R>(dm, dp, jfac, S);
            else if (sec == 1) deposit3_axis<1, R>(dm, dp, jfac, S);
            else if (sec == 2) deposit3_axis<2, R>(dm, dp, jfac, S);
            else deposit3<R>(dm, dp, jfac, S);
        };
        // the sections run side by side, one group of waves each, so that every
        // wave runs a single deposit variant
        {
            constexpr int NG = NT / 64 / 4;  // waves per group
            const int wv = threadIdx.x >> 6;
            const int sec = wv & 3;
            const int gt = (wv >> 2) * 64 + (threadIdx.x & 63);
            unsigned rows = 0;
            for (int k = 0; k < CJ; ++k) rows = max(rows, min(qc_n[sec * CJ + k], capc));
            const int nmap = (int)rows * CJ;
            for (int sl = gt; sl < nmap; sl += NG * 64) {
                const int col = sec * CJ + (sl & (CJ - 1));
                const unsigned row = (unsigned)(sl / CJ);
                if (row >= min(qc_n[col], capc)) continue;
                cross(begin + qmap[col + 4 * CJ * row], sec);
            }
        }
        if (qc_unmapped) {
            for (int q = threadIdx.x; q < (int)qc_total; q += NT) {
                const int64_t e = begin + q;
                if (a.qword[e] & kUnmapped) cross(e, 3);
            }
        }
        __syncthreads();
    }

    // 6. flush the LDS current tile
    flush_current3<R, NT>(g, T0, sj, Jg, small);
    if (threadIdx.x == 0 && a.counters) {
        atomicAdd(&a.counters[1], (unsigned long long)qo_n);
        atomicAdd(&a.counters[2], (unsigned long long)(end - begin));
        atomicAdd(&a.counters[3], (unsigned long long)n_migrant);
    }
}

// ---------------------------------------------------------------------------
// Migrants: the particles that the step kernel found outside their sorted
// tile's region, advanced by the workgroup of the tile that now holds their
// cell.  A bucket of at least kMigLds particles stages the tile's fields and
// current in LDS as the step kernel does (every migrant lies inside its new
// tile, so it always fits); a smaller one takes the global-memory path.  The
// bucket counter is cleared for the next launch.
// ---------------------------------------------------------------------------
template <class R, int NT>
__global__ __launch_bounds__(NT) void k_migrants3(GridK g, StepArgs a, const double* __restrict__ fields,
                                                 const double* __restrict__ bfield, double* __restrict__ Jg)
{
    using TL = Tile3Dims<R>;
    constexpr int T = kTile3, MX = TL::MX, M = TL::M;
    constexpr int SJY = TL::JROW, SJZ = TL::JPLANE;
    constexpr int NJ = TL::NJ;
    __shared__ R sf[kFieldPlanes3 * TL::FPLANE];
    __shared__ LdsJ<R, 3 * NJ> sj;
    __shared__ unsigned int n_global;

    const int tile = xcd_tile(blockIdx.x, g.ntiles);
    const unsigned cnt = min(a.mig_n[tile], a.mig_cap);
    if (cnt == 0) return;
    const uint32_t* bucket = a.mig + (int64_t)tile * a.mig_cap;
    if (cnt < kMigLds) {
        for (unsigned q = threadIdx.x; q < cnt; q += NT) advance_global3<R>(g, a, bucket[q], fields, bfield, Jg);
        __syncthreads();
        if (threadIdx.x == 0) {
            a.mig_n[tile] = 0;
            if (a.counters) atomicAdd(&a.counters[1], (unsigned long long)cnt);
        }
        return;
    }
    const int tx = tile % g.nt[0];
    const int ty = (tile / g.nt[0]) % g.nt[1];
    const int tz = tile / (g.nt[0] * g.nt[1]);
    const int T0[3] = {tx * T, ty * T, tz * T};
    const bool small = g.n[0] < TL::LJX || g.n[1] < TL::LJY || g.n[2] < TL::LJY;
    stage_fields3<R, NT>(g, T0, fields, bfield, sf, small);
    for (int e = threadIdx.x; e < 3 * NJ; e += NT) sj.zero(e);
    if (threadIdx.x == 0) n_global = 0;
    __syncthreads();
    unsigned my_global = 0;
    for (unsigned q = threadIdx.x; q < cnt; q += NT) {
        const int64_t p = bucket[q];
        int i0[3];
        R d0[3];
        PosIO<R, 3>::load(a, p, i0, d0);
        int rel[3];
        if (!relative3<R>(g, T0, i0, rel)) {  // not a cell of this tile (non-finite input): global memory
            advance_global3<R>(g, a, p, fields, bfield, Jg);
            ++my_global;
            continue;
        }
        Axis<R> ax0[3];
        R d1[3], qp;
        int delta[3];
        advance_lds3<R>(g, a, sf, p, i0, d0, rel, ax0, d1, delta, qp);
        R jfac[3];
        for (int ax = 0; ax < 3; ++ax) jfac[ax] = (R)g.jscale[ax] * qp;
        R dm[3][4], dp[3][4];
        for (int ax = 0; ax < 3; ++ax) {
            R s1[3];
            cell_weights<R>(d1[ax], s1);
            window<R>(ax0[ax].s, s1, delta[ax], dm[ax], dp[ax]);
        }
        int s[3];
        for (int ax = 0; ax < 3; ++ax) s[ax] = rel[ax] + (delta[ax] < 0 ? -1 : 0) - 1;
        const int jb = (s[0] + 2 + MX) + (s[1] + 2 + M) * SJY + (s[2] + 2 + M) * SJZ;
        auto S = [&](int comp, int ix, int iy, int iz, double v) {
            sj.add(comp * NJ + jb + ix + iy * SJY + iz * SJZ, v);
        };
        deposit3<R>(dm, dp, jfac, S);
    }
    if (my_global) atomicAdd(&n_global, my_global);
    __syncthreads();
    flush_current3<R, NT>(g, T0, sj, Jg, small);
    if (threadIdx.x == 0) {
        a.mig_n[tile] = 0;
        if (a.counters && n_global) atomicAdd(&a.counters[1], (unsigned long long)n_global);
    }
}

// ---------------------------------------------------------------------------
// Standalone current of position pairs (pic_deposit_J): same arithmetic,
// global atomics.
// ---------------------------------------------------------------------------
template <class R, int D>
__global__ __launch_bounds__(256) void k_deposit_pairs(GridK g, const double* __restrict__ x0,
                                                       const double* __restrict__ x1,
                                                       const double* __restrict__ charge, int64_t n,
                                                       double* __restrict__ Jg)
{
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= n) return;
    const int64_t N = g.ncell;
    const int nx = g.n[0], ny = g.n[1], nz = g.n[2];
    int i0[3] = {0, 0, 0};
    R d0[3] = {0, 0, 0}, disp[3] = {0, 0, 0}, d1[3] = {0, 0, 0};
    int delta[3] = {0, 0, 0};
    for (int ax = 0; ax < D; ++ax) {
        const double a0 = x0[ax * n + p], a1 = x1[ax * n + p];
        double fl = floor(a0);
        R o = (R)(a0 - fl);
        if (o >= R(1)) {  // FP32 rounding of an offset just below 1
            o = R(0);
            fl += 1.0;
        }
        i0[ax] = wrapi((int)fl, g.n[ax]);
        d0[ax] = o;
        disp[ax] = (R)(a1 - a0);
    }
    StepArgs dummy{};
    PosIO<R, D>::move(dummy, p, g, i0, d0, disp, d1, delta, false);
    const R qp = (R)charge[p];
    R dm[3][4], dp[3][4];
    for (int ax = 0; ax < D; ++ax) {
        R s0[3], s1[3];
        cell_weights<R>(d0[ax], s0);
        cell_weights<R>(d1[ax], s1);
        window<R>(s0, s1, delta[ax], dm[ax], dp[ax]);
    }
    R jfac[3];
    for (int ax = 0; ax < 3; ++ax) jfac[ax] = (R)g.jscale[ax] * qp;
    // 2D: J^z from the z displacement, u_z = (z1 - z0) dz / dt
    const R jz2 = D == 2 ? qp * (R)(0.25 * g.inv_vol * (x1[2 * n + p] - x0[2 * n + p]) /
                                    g.inv_h[2] / g.dt)
                         : R(0);
    int xi[4], yj[4];
    int64_t zk[4];
    int s[3];
    for (int ax = 0; ax < 3; ++ax) s[ax] = (ax < D) ? i0[ax] + (delta[ax] < 0 ? -1 : 0) - 1 : 0;
    for (int o = 0; o < 4; ++o) {
        xi[o] = wrapi(s[0] + o, nx);
        yj[o] = wrapi(s[1] + o, ny) * nx;
        zk[o] = D == 3 ? (int64_t)wrapi(s[2] + o, nz) * nx * ny : 0;
    }
    auto S = [&](int comp, int ix, int iy, int iz, double v) {
        global_add(&Jg[comp * N + zk[iz] + yj[iy] + xi[ix]], v);
    };
    if (D == 3) deposit3<R>(dm, dp, jfac, S);
    else deposit2<R>(dm, dp, jfac, jz2, S);
}

// ---------------------------------------------------------------------------
// Load (FP64 input -> species layout) and readback.
// ---------------------------------------------------------------------------
template <class R, int D>
__global__ __launch_bounds__(256) void k_load(GridK g, PartArrays dst, int64_t offset,
                                              const double* __restrict__ x,
                                              const double* __restrict__ w,
                                              const double* __restrict__ weight, int64_t n,
                                              unsigned long long* bad)
{
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= n) return;
    const int64_t q = offset + p;
    bool ok = true;
    int ic[3] = {0, 0, 0};
    for (int ax = 0; ax < 3; ++ax) {
        const double v = x[ax * n + p];
        if (ax < D) ok = ok && (v >= 0.0) && (v < (double)g.n[ax]);
        if (sizeof(R) == 8) {
            ((double*)dst.pos[ax])[q] = v;
        } else if (ax < D) {
            double fl = floor(v);
            float o = (float)(v - fl);
            if (o >= 1.0f) {
                o = 0.0f;
                fl += 1.0;
            }
            int ci = (int)fl;
            if (ci >= g.n[ax]) ci -= g.n[ax];
            ic[ax] = ci;
            ((float*)dst.pos[ax])[q] = o;
        }
        const double wv = w[ax * n + p];
        ok = ok && isfinite(wv);
        ((R*)dst.mom[ax])[q] = (R)wv;
    }
    const double wt = weight[p];
    ok = ok && (wt > 0.0) && isfinite(wt);
    ((R*)dst.weight)[q] = (R)wt;
    if (sizeof(R) == 4) dst.cell[q] = pack_cell(ic[0], ic[1], ic[2]);
    dst.id[q] = q;
    if (!ok) atomicAdd(bad, 1ull);
}

template <class R, int D>
__global__ __launch_bounds__(256) void k_get(PartArrays src, int64_t n, double* __restrict__ x,
                                             double* __restrict__ w, double* __restrict__ weight,
                                             int64_t* __restrict__ id)
{
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= n) return;
    int ic[3] = {0, 0, 0};
    if (sizeof(R) == 4) unpack_cell(src.cell[p], ic);
    for (int ax = 0; ax < 3; ++ax) {
        if (x) {
            double v;
            if (sizeof(R) == 8) v = ((const double*)src.pos[ax])[p];
            else v = ax < D ? (double)ic[ax] + (double)((const float*)src.pos[ax])[p] : 0.5;
            x[ax * n + p] = v;
        }
        if (w) w[ax * n + p] = (double)((const R*)src.mom[ax])[p];
    }
    if (weight) weight[p] = (double)((const R*)src.weight)[p];
    if (id) id[p] = src.id[p];
}

// Charge density of particles (Eq. rho), FP64, global atomics.
template <class R, int D>
__global__ __launch_bounds__(256) void k_rho(GridK g, PartArrays src, int64_t n, double q,
                                             double* __restrict__ rho)
{
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= n) return;
    int i[3] = {0, 0, 0};
    double d[3] = {0, 0, 0};
    if (sizeof(R) == 4) {
        unpack_cell(src.cell[p], i);
        for (int ax = 0; ax < D; ++ax) d[ax] = (double)((const float*)src.pos[ax])[p];
    } else {
        for (int ax = 0; ax < D; ++ax) {
            const double x = ((const double*)src.pos[ax])[p];
            const double fl = floor(x);
            i[ax] = (int)fl;
            d[ax] = x - fl;
        }
    }
    double s[3][3];
    for (int ax = 0; ax < 3; ++ax) cell_weights<double>(ax < D ? d[ax] : 0.0, s[ax]);
    const double qv = q * (double)((const R*)src.weight)[p] * g.inv_vol;
    const int nx = g.n[0], ny = g.n[1], nz = g.n[2];
    for (int c = (D == 3 ? -1 : 0); c <= (D == 3 ? 1 : 0); ++c) {
        const double wz = D == 3 ? s[2][c + 1] : 1.0;
        const int64_t kz = (int64_t)wrapi(i[2] + c, nz) * ny * nx;
        for (int b = -1; b <= 1; ++b) {
            const int64_t jy = (int64_t)wrapi(i[1] + b, ny) * nx;
            for (int a2 = -1; a2 <= 1; ++a2)
                global_add(&rho[kz + jy + wrapi(i[0] + a2, nx)], qv * wz * s[1][b + 1] * s[0][a2 + 1]);
        }
    }
}

// Charge density of a cell-sorted species (Eq. rho), one workgroup per tile:
// particles within M cells of their tile accumulate into an LDS density tile
// (cells T0-1-M .. T0+T+M), the rest go straight to global memory; the tile
// is then added to the global density with atomics.
template <class R, int D, int T, int M, int NT>
__global__ __launch_bounds__(NT) void k_rho_tiled(GridK g, PartArrays src, const int64_t* __restrict__ ts,
                                                  double q, double* __restrict__ rho)
{
    constexpr int L = T + 2 + 2 * M;
    constexpr int NL = D == 3 ? L * L * L : L * L;
    __shared__ double sr[NL];
    const int tile = xcd_tile(blockIdx.x, g.ntiles);
    const int T0[3] = {(tile % g.nt[0]) * T, ((tile / g.nt[0]) % g.nt[1]) * T,
                       D == 3 ? (tile / (g.nt[0] * g.nt[1])) * T : 0};
    const int nx = g.n[0], ny = g.n[1], nz = g.n[2];
    for (int e = threadIdx.x; e < NL; e += NT) sr[e] = 0.0;
    __syncthreads();
    const int64_t begin = ts[tile], end = ts[tile + 1];
    for (int64_t p = begin + threadIdx.x; p < end; p += NT) {
        int i[3] = {0, 0, 0};
        double d[3] = {0, 0, 0};
        if (sizeof(R) == 4) {
            unpack_cell(src.cell[p], i);
            for (int ax = 0; ax < D; ++ax) d[ax] = (double)((const float*)src.pos[ax])[p];
        } else {
            for (int ax = 0; ax < D; ++ax) {
                const double x = ((const double*)src.pos[ax])[p];
                const double fl = floor(x);
                i[ax] = (int)fl;
                d[ax] = x - fl;
            }
        }
        double w3[3][3];
        for (int ax = 0; ax < 3; ++ax) cell_weights<double>(ax < D ? d[ax] : 0.0, w3[ax]);
        const double qv = q * (double)((const R*)src.weight)[p] * g.inv_vol;
        int rel[3] = {0, 0, 0};
        bool inside = true;
        for (int ax = 0; ax < D; ++ax) {
            int r = i[ax] - T0[ax];
            const int n = g.n[ax];
            if (r > n / 2) r -= n;
            if (r < -(n / 2)) r += n;
            rel[ax] = r;
            inside = inside && r >= -M && r <= T - 1 + M;
        }
        for (int c = (D == 3 ? -1 : 0); c <= (D == 3 ? 1 : 0); ++c) {
            const double wz = D == 3 ? w3[2][c + 1] : 1.0;
            for (int b = -1; b <= 1; ++b)
                for (int a2 = -1; a2 <= 1; ++a2) {
                    const double v = qv * wz * w3[1][b + 1] * w3[0][a2 + 1];
                    if (inside) {
                        const int li = rel[0] + 1 + M + a2, lj = rel[1] + 1 + M + b;
                        const int lk = D == 3 ? rel[2] + 1 + M + c : 0;
                        atomicAdd(&sr[(lk * L + lj) * L + li], v);
                    } else {
                        const int64_t kz = D == 3 ? (int64_t)wrapi(i[2] + c, nz) * ny * nx : 0;
                        global_add(&rho[kz + (int64_t)wrapi(i[1] + b, ny) * nx + wrapi(i[0] + a2, nx)], v);
                    }
                }
        }
    }
    __syncthreads();
    for (int e = threadIdx.x; e < NL; e += NT) {
        const double v = sr[e];
        if (v == 0.0) continue;
        const int lx = e % L, ly = (e / L) % L, lz = D == 3 ? e / (L * L) : 0;
        const int gx = wrapi(T0[0] - 1 - M + lx, nx), gy = wrapi(T0[1] - 1 - M + ly, ny);
        const int gz = D == 3 ? wrapi(T0[2] - 1 - M + lz, nz) : 0;
        global_add(&rho[((int64_t)gz * ny + gy) * nx + gx], v);
    }
}

// Charge density of FP64 position arrays [3][n] (immobile species at load).
template <int D>
__global__ __launch_bounds__(256) void k_rho_raw(GridK g, const double* __restrict__ x,
                                                 const double* __restrict__ weight, double q,
                                                 int64_t n, double* __restrict__ rho, bool w32)
{
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= n) return;
    int i[3] = {0, 0, 0};
    double s[3][3];
    for (int ax = 0; ax < 3; ++ax) {
        double d = 0.0;
        if (ax < D) {
            const double v = x[ax * n + p];
            const double fl = floor(v);
            i[ax] = (int)fl;
            d = v - fl;
        }
        cell_weights<double>(d, s[ax]);
    }
    // FP32 mode stores every weight in FP32; the background uses the same
    // rounded weight so that a co-located neutral start has zero total charge
    const double wt = w32 ? (double)(float)weight[p] : weight[p];
    const double qv = q * wt * g.inv_vol;
    const int nx = g.n[0], ny = g.n[1], nz = g.n[2];
    for (int c = (D == 3 ? -1 : 0); c <= (D == 3 ? 1 : 0); ++c) {
        const double wz = D == 3 ? s[2][c + 1] : 1.0;
        const int64_t kz = (int64_t)wrapi(i[2] + c, nz) * ny * nx;
        for (int b = -1; b <= 1; ++b) {
            const int64_t jy = (int64_t)wrapi(i[1] + b, ny) * nx;
            for (int a2 = -1; a2 <= 1; ++a2)
                global_add(&rho[kz + jy + wrapi(i[0] + a2, nx)], qv * wz * s[1][b + 1] * s[0][a2 + 1]);
        }
    }
}

template <class R>
StepArgs step_args(const Ctx& c, const Species& sp, unsigned long long* counters)
{
    StepArgs a{};
    for (int ax = 0; ax < 3; ++ax) {
        a.pos[ax] = sp.cur.pos[ax];
        a.mom[ax] = sp.cur.mom[ax];
    }
    a.weight = sp.cur.weight;
    a.cell = sp.cur.cell;
    a.tile_start = sp.tile_start;
    a.q = sp.d.q;
    a.qm = sp.d.q / sp.d.m;
    a.counters = counters;
    // migrant buckets: the species' sort scratch (key .. src, idle between
    // sorts), an equal share per tile; counters in the workspace
    a.mig = sp.key;
    a.mig_cap = (uint32_t)(((size_t)((char*)sp.tile_start - (char*)sp.key) / 4) / (size_t)c.k.ntiles);
    a.mig_n = c.mig_n;
    for (int ax = 0; ax < 3; ++ax) a.qd0[ax] = sp.alt.pos[ax];
    a.qword = sp.alt.id;
    a.qmap = (void*)sp.alt.weight;
    a.qother = sp.alt.mom[2];
    a.mlist = sp.alt.mom[0];
    a.mlist2 = sp.alt.mom[1];
    return a;
}

// Threads per workgroup of each instantiation.
constexpr int kThreads3 = 768;    // FP64: 3 waves per SIMD, <= 170 VGPRs
constexpr int kThreads3f = 1024;  // FP32: 4 waves per SIMD
constexpr int kChunk3 = 1;        // FP64: slots per lane and wave chunk
constexpr int kChunk3f = 3;       // FP32: slots per lane and wave chunk
constexpr int kThreadsMig = 768;   // migrant pass, FP64 (as many waves as the step kernel)
constexpr int kThreadsMigf = 1024; // migrant pass, FP32
constexpr int kThreads2 = 256;
constexpr int kMargin2 = 2;

unsigned blocks_for(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

hipError_t launch_particle_step(Ctx& c, Species& sp, hipStream_t s)
{
    if (sp.n == 0) return hipSuccess;
    if (c.g.order == 2) return launch_particle_step_o2(c, sp, s);
    if (c.g.interp == 1) return launch_particle_step_conv(c, sp, s);
    double* J = c.fields + 6 * c.k.ncell;
    const dim3 grid(c.k.ntiles);
    if (c.g.precision == PIC_FP64) {
        StepArgs a = step_args<double>(c, sp, c.counters);
        if (c.k.dims == 3) {
            hipLaunchKernelGGL((k_particle_step3<double, kThreads3, kChunk3>), grid, dim3(kThreads3), 0, s, c.k, a,
                               c.fields, c.bn, J);
            hipLaunchKernelGGL((k_migrants3<double, kThreadsMig>), grid, dim3(kThreadsMig), 0, s, c.k, a,
                               c.fields, c.bn, J);
        }
        else
            hipLaunchKernelGGL((k_particle_step<double, 2, kTile2, kMargin2, kThreads2>), grid,
                               dim3(kThreads2), 0, s, c.k, a, c.fields, c.bn, J);
    } else {
        StepArgs a = step_args<float>(c, sp, c.counters);
        if (c.k.dims == 3) {
            hipLaunchKernelGGL((k_particle_step3<float, kThreads3f, kChunk3f>), grid, dim3(kThreads3f), 0, s, c.k, a,
                               c.fields, c.bn, J);
            hipLaunchKernelGGL((k_migrants3<float, kThreadsMigf>), grid, dim3(kThreadsMigf), 0, s, c.k, a,
                               c.fields, c.bn, J);
        }
        else
            hipLaunchKernelGGL((k_particle_step<float, 2, kTile2, kMargin2, kThreads2>), grid,
                               dim3(kThreads2), 0, s, c.k, a, c.fields, c.bn, J);
    }
    return hipGetLastError();
}

hipError_t launch_deposit_only(const Ctx& c, const double* x0, const double* x1,
                               const double* charge, int64_t n, double* J, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    if (c.g.order == 2) return launch_deposit_only_o2(c, x0, x1, charge, n, J, s);
    const dim3 grid(blocks_for(n));
    if (c.g.precision == PIC_FP64) {
        if (c.k.dims == 3)
            hipLaunchKernelGGL((k_deposit_pairs<double, 3>), grid, dim3(256), 0, s, c.k, x0, x1, charge, n, J);
        else
            hipLaunchKernelGGL((k_deposit_pairs<double, 2>), grid, dim3(256), 0, s, c.k, x0, x1, charge, n, J);
    } else {
        if (c.k.dims == 3)
            hipLaunchKernelGGL((k_deposit_pairs<float, 3>), grid, dim3(256), 0, s, c.k, x0, x1, charge, n, J);
        else
            hipLaunchKernelGGL((k_deposit_pairs<float, 2>), grid, dim3(256), 0, s, c.k, x0, x1, charge, n, J);
    }
    return hipGetLastError();
}

hipError_t launch_load(Ctx& c, Species& sp, int64_t n, const double* x, const double* w,
                       const double* weight, hipStream_t s)
{
    const dim3 grid(blocks_for(n));
    unsigned long long* bad = c.counters;
    if (c.g.precision == PIC_FP64) {
        if (c.k.dims == 3)
            hipLaunchKernelGGL((k_load<double, 3>), grid, dim3(256), 0, s, c.k, sp.cur, sp.n, x, w, weight, n, bad);
        else
            hipLaunchKernelGGL((k_load<double, 2>), grid, dim3(256), 0, s, c.k, sp.cur, sp.n, x, w, weight, n, bad);
    } else {
        if (c.k.dims == 3)
            hipLaunchKernelGGL((k_load<float, 3>), grid, dim3(256), 0, s, c.k, sp.cur, sp.n, x, w, weight, n, bad);
        else
            hipLaunchKernelGGL((k_load<float, 2>), grid, dim3(256), 0, s, c.k, sp.cur, sp.n, x, w, weight, n, bad);
    }
    return hipGetLastError();
}

hipError_t launch_get(const Ctx& c, const Species& sp, double* x, double* w, double* weight,
                      int64_t* id, hipStream_t s)
{
    if (sp.n == 0) return hipSuccess;
    const dim3 grid(blocks_for(sp.n));
    if (c.g.precision == PIC_FP64) {
        if (c.k.dims == 3)
            hipLaunchKernelGGL((k_get<double, 3>), grid, dim3(256), 0, s, sp.cur, sp.n, x, w, weight, id);
        else
            hipLaunchKernelGGL((k_get<double, 2>), grid, dim3(256), 0, s, sp.cur, sp.n, x, w, weight, id);
    } else {
        if (c.k.dims == 3)
            hipLaunchKernelGGL((k_get<float, 3>), grid, dim3(256), 0, s, sp.cur, sp.n, x, w, weight, id);
        else
            hipLaunchKernelGGL((k_get<float, 2>), grid, dim3(256), 0, s, sp.cur, sp.n, x, w, weight, id);
    }
    return hipGetLastError();
}

hipError_t launch_rho(const Ctx& c, const Species& sp, double* rho, hipStream_t s)
{
    if (sp.n == 0) return hipSuccess;
    if (c.g.order == 2) {
        const double* x[3] = {(const double*)sp.cur.pos[0], (const double*)sp.cur.pos[1],
                              (const double*)sp.cur.pos[2]};
        return launch_rho_o2(c, x, (const double*)sp.cur.weight, sp.n, sp.d.q, rho, s);
    }
    if (sp.sorted) {  // tiles are valid: LDS accumulation per tile
        const dim3 tg(c.k.ntiles);
        const bool f64 = c.g.precision == PIC_FP64;
        if (c.k.dims == 3) {
            if (f64)
                hipLaunchKernelGGL((k_rho_tiled<double, 3, kTile3, 2, 256>), tg, dim3(256), 0, s, c.k, sp.cur, sp.tile_start, sp.d.q, rho);
            else
                hipLaunchKernelGGL((k_rho_tiled<float, 3, kTile3, 2, 256>), tg, dim3(256), 0, s, c.k, sp.cur, sp.tile_start, sp.d.q, rho);
        } else {
            if (f64)
                hipLaunchKernelGGL((k_rho_tiled<double, 2, kTile2, 2, 256>), tg, dim3(256), 0, s, c.k, sp.cur, sp.tile_start, sp.d.q, rho);
            else
                hipLaunchKernelGGL((k_rho_tiled<float, 2, kTile2, 2, 256>), tg, dim3(256), 0, s, c.k, sp.cur, sp.tile_start, sp.d.q, rho);
        }
        return hipGetLastError();
    }
    const dim3 grid(blocks_for(sp.n));
    if (c.g.precision == PIC_FP64) {
        if (c.k.dims == 3)
            hipLaunchKernelGGL((k_rho<double, 3>), grid, dim3(256), 0, s, c.k, sp.cur, sp.n, sp.d.q, rho);
        else
            hipLaunchKernelGGL((k_rho<double, 2>), grid, dim3(256), 0, s, c.k, sp.cur, sp.n, sp.d.q, rho);
    } else {
        if (c.k.dims == 3)
            hipLaunchKernelGGL((k_rho<float, 3>), grid, dim3(256), 0, s, c.k, sp.cur, sp.n, sp.d.q, rho);
        else
            hipLaunchKernelGGL((k_rho<float, 2>), grid, dim3(256), 0, s, c.k, sp.cur, sp.n, sp.d.q, rho);
    }
    return hipGetLastError();
}

hipError_t launch_rho_raw(const Ctx& c, const double* x, const double* weight, double charge,
                          int64_t n, double* rho, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    if (c.g.order == 2) {
        const double* xr[3] = {x, x + n, x + 2 * n};
        return launch_rho_o2(c, xr, weight, n, charge, rho, s);
    }
    const dim3 grid(blocks_for(n));
    const bool w32 = c.g.precision == PIC_FP32C;
    if (c.k.dims == 3)
        hipLaunchKernelGGL((k_rho_raw<3>), grid, dim3(256), 0, s, c.k, x, weight, charge, n, rho, w32);
    else
        hipLaunchKernelGGL((k_rho_raw<2>), grid, dim3(256), 0, s, c.k, x, weight, charge, n, rho, w32);
    return hipGetLastError();
}

}  // namespace pic
