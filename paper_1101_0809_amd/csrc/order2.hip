// order2.hip -- the particle step with the alternating form factor of order
// 2 1/2 (Section 4.5): gather of E with alpha (Eq. alphax) and of B^n with
// beta (Eq. betax) at quadratic node and cubic cell factors, the push
// (Appendix, Eq. p2), the position advance (Eq. coordscheme) and the
// charge-conserving current (Eq. current, one-quarter form) on a 5-cell
// window per axis; plus the order-2 1/2 charge density (Eq. rho) and the
// current of given moves.  FP64.
//
// One workgroup per cell tile (the tiles of the cell sort).  It stages E^n and
// B^n over the cells the tile's particles can read (offsets -2 .. +2 around
// each particle cell, plus a margin M for drift since the sort) and
// accumulates the current over the cells their windows can reach (-3 .. +3,
// plus M) in LDS, added to the grid once at the end; in 3D the two regions
// are handled by two passes.  A particle further than M cells from its tile
// reads and adds in global memory instead.
#include "pic_math.h"

namespace pic {
namespace {

__device__ __forceinline__ void add_global(double* p, double v) { unsafeAtomicAdd(p, v); }

// window5 with both weight sets in registers first: a select between two
// entries of one array (the window shifted one cell or not) would otherwise
// become one load at a run-time index, which keeps the array in scratch
// memory.
__device__ __forceinline__ void window5_reg(const double (&s0)[4], const double (&s1)[4], int shift, double dm[5],
                                            double dp[5])
{
    double a[4], b[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        a[k] = s0[k];
        b[k] = s1[k];
        asm("" : "+v"(a[k]));
        asm("" : "+v"(b[k]));
    }
    window5<double>(a, b, shift, dm, dp);
}

// The single pass, used in 2D3V (its two regions fit in LDS with margin 2).
constexpr int kO2M2 = 2, kO2NT2 = 256;

template <int D>
__global__ __launch_bounds__(kO2NT2) void k_step_o2(GridK g, StepArgs a, const double* __restrict__ fields,
                                                    const double* __restrict__ bfield, double* __restrict__ Jg)
{
    static_assert(D == 2, "the 3D order-2 1/2 step runs in two passes");
    constexpr int T = kTile2, M = kO2M2, NT = kO2NT2;
    constexpr int LF = T + 4 + 2 * M;  // field region: cells T0-2-M .. T0+T+1+M
    constexpr int LJ = T + 6 + 2 * M;  // current region: cells T0-3-M .. T0+T+2+M
    constexpr int NF = D == 3 ? LF * LF * LF : LF * LF;
    constexpr int NJ = D == 3 ? LJ * LJ * LJ : LJ * LJ;
    __shared__ double sf[6 * NF];
    __shared__ double sj[3 * NJ];
    __shared__ unsigned int n_fallback;

    const int tile = xcd_tile(blockIdx.x, g.ntiles);
    const int T0[3] = {(tile % g.nt[0]) * T, ((tile / g.nt[0]) % g.nt[1]) * T,
                       D == 3 ? (tile / (g.nt[0] * g.nt[1])) * T : 0};
    const int64_t N = g.ncell;
    const int nx = g.n[0], ny = g.n[1], nz = g.n[2];

    for (int e = threadIdx.x; e < 6 * NF; e += NT) {
        const int comp = e / NF, r = e - comp * NF;
        const int gx = wrapi(T0[0] - 2 - M + r % LF, nx);
        const int gy = wrapi(T0[1] - 2 - M + (r / LF) % LF, ny);
        const int gz = D == 3 ? wrapi(T0[2] - 2 - M + r / (LF * LF), nz) : 0;
        const int64_t cell = ((int64_t)gz * ny + gy) * nx + gx;
        sf[e] = comp < 3 ? fields[comp * N + cell] : bfield[(comp - 3) * N + cell];
    }
    for (int e = threadIdx.x; e < 3 * NJ; e += NT) sj[e] = 0.0;
    if (threadIdx.x == 0) n_fallback = 0;
    __syncthreads();

    const double c = g.c, c2 = c * c;
    const double qmdt2 = 0.5 * a.qm * g.dt;
    const int64_t begin = a.tile_start[tile], end = a.tile_start[tile + 1];
    unsigned int my_fallback = 0;
    for (int64_t p = begin + threadIdx.x; p < end; p += NT) {
        int i0[3];
        double d0[3];
        PosIO<double, D>::load(a, p, i0, d0);
        double w[3];
        for (int ax = 0; ax < 3; ++ax) w[ax] = ((const double*)a.mom[ax])[p];
        const double qp = a.q * ((const double*)a.weight)[p];
        Axis2<double> ax0[3];
        for (int ax = 0; ax < 3; ++ax) ax0[ax] = form_factor2<double>(ax < D ? d0[ax] : 0.0);

        int rel[3] = {0, 0, 0};
        bool inside = true;
        for (int ax = 0; ax < D; ++ax) {
            int r = i0[ax] - T0[ax];
            const int n = g.n[ax];
            if (r > n / 2) r -= n;
            if (r < -(n / 2)) r += n;
            rel[ax] = r;
            inside = inside && r >= -M && r <= T - 1 + M;
        }
        my_fallback += inside ? 0 : 1;

        double E[3], B[3];
        if (inside) {
            const int fb = (rel[0] + 2 + M) + (rel[1] + 2 + M) * LF + (D == 3 ? (rel[2] + 2 + M) * LF * LF : 0);
            auto F = [&](int comp, int oa, int ob, int oc) -> double {
                return sf[comp * NF + fb + oa + ob * LF + (D == 3 ? oc * LF * LF : 0)];
            };
            if (D == 3) gather3_o2<double>(ax0, F, E, B);
            else gather2_o2<double>(ax0, F, E, B);
        } else {
            auto F = [&](int comp, int oa, int ob, int oc) -> double {
                const int64_t cell = ((int64_t)(D == 3 ? wrapi(i0[2] + oc, nz) : 0) * ny + wrapi(i0[1] + ob, ny)) * nx +
                                     wrapi(i0[0] + oa, nx);
                return comp < 3 ? fields[comp * N + cell] : bfield[(comp - 3) * N + cell];
            };
            if (D == 3) gather3_o2<double>(ax0, F, E, B);
            else gather2_o2<double>(ax0, F, E, B);
        }
        for (int ax = 0; ax < 3; ++ax) B[ax] += g.bext[ax];

        push<double>(qmdt2, c2, E, B, w);
        for (int ax = 0; ax < 3; ++ax) ((double*)a.mom[ax])[p] = w[ax];
        const double inv = 1.0 / ::sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2] + c2);
        double disp[3];
        for (int ax = 0; ax < 3; ++ax) disp[ax] = w[ax] * inv * g.cfl[ax];
        double d1[3];
        int delta[3] = {0, 0, 0};
        PosIO<double, D>::move(a, p, g, i0, d0, disp, d1, delta, true);

        // window per axis: start i0 + h0, end (i0 + delta) + h1
        double dm[3][5], dp[3][5];
        int s[3] = {0, 0, 0};
        for (int ax = 0; ax < D; ++ax) {
            const Axis2<double> e1 = form_factor2<double>(d1[ax]);
            const int shift = delta[ax] + e1.h - ax0[ax].h;
            window5_reg(ax0[ax].s, e1.s, shift, dm[ax], dp[ax]);
            s[ax] = ax0[ax].h + (shift < 0 ? shift : 0) - 2;  // window start, from the particle cell
        }
        double jfac[3];
        for (int ax = 0; ax < 3; ++ax) jfac[ax] = g.jscale[ax] * qp;
        const double jz = D == 2 ? qp * (0.25 * g.inv_vol) * c * w[2] * inv : 0.0;
        if (inside) {
            const int jb = (rel[0] + s[0] + 3 + M) + (rel[1] + s[1] + 3 + M) * LJ +
                           (D == 3 ? (rel[2] + s[2] + 3 + M) * LJ * LJ : 0);
            auto S = [&](int comp, int ix, int iy, int iz, double v) {
                atomicAdd(&sj[comp * NJ + jb + ix + iy * LJ + (D == 3 ? iz * LJ * LJ : 0)], v);
            };
            if (D == 3) deposit3_o2<double>(dm, dp, jfac, S);
            else deposit2_o2<double>(dm, dp, jfac, jz, S);
        } else {
            auto S = [&](int comp, int ix, int iy, int iz, double v) {
                const int64_t cell =
                    ((int64_t)(D == 3 ? wrapi(i0[2] + s[2] + iz, nz) : 0) * ny + wrapi(i0[1] + s[1] + iy, ny)) * nx +
                    wrapi(i0[0] + s[0] + ix, nx);
                add_global(&Jg[comp * N + cell], v);
            };
            if (D == 3) deposit3_o2<double>(dm, dp, jfac, S);
            else deposit2_o2<double>(dm, dp, jfac, jz, S);
        }
    }
    if (my_fallback) atomicAdd(&n_fallback, my_fallback);
    __syncthreads();
    for (int e = threadIdx.x; e < 3 * NJ; e += NT) {
        const double v = sj[e];
        if (v == 0.0) continue;
        const int comp = e / NJ, r = e - comp * NJ;
        const int gx = wrapi(T0[0] - 3 - M + r % LJ, nx);
        const int gy = wrapi(T0[1] - 3 - M + (r / LJ) % LJ, ny);
        const int gz = D == 3 ? wrapi(T0[2] - 3 - M + r / (LJ * LJ), nz) : 0;
        add_global(&Jg[comp * N + ((int64_t)gz * ny + gy) * nx + gx], v);
    }
    if (threadIdx.x == 0 && a.counters) {
        atomicAdd(&a.counters[1], (unsigned long long)n_fallback);
        atomicAdd(&a.counters[2], (unsigned long long)(end - begin));
    }
}

// 3D in two passes, each staging one region with a wider drift margin than
// the single pass could afford (its two regions at margin 0 fill the LDS).
// Pass 1: gather, push and move with E^n, B^n over cells T0-3 .. T0+T+2 (132
// KB); the start position goes to the spare particle copy (idle between
// sorts) and the per-axis cell shifts to its id array.  Pass 2: the current
// over cells T0-5 .. T0+T+4 (140 KB).
constexpr int kO2M3a = 1, kO2M3b = 2, kO2NT3 = 512;

__global__ __launch_bounds__(kO2NT3) void k_push_o2_3d(GridK g, StepArgs a, PartArrays spare,
                                                       const double* __restrict__ fields,
                                                       const double* __restrict__ bfield)
{
    constexpr int T = kTile3, M = kO2M3a, NT = kO2NT3;
    constexpr int LF = T + 4 + 2 * M, NF = LF * LF * LF;
    __shared__ double sf[6 * NF];
    __shared__ unsigned int n_fallback;
    const int tile = xcd_tile(blockIdx.x, g.ntiles);
    const int T0[3] = {(tile % g.nt[0]) * T, ((tile / g.nt[0]) % g.nt[1]) * T, (tile / (g.nt[0] * g.nt[1])) * T};
    const int64_t N = g.ncell;
    const int nx = g.n[0], ny = g.n[1], nz = g.n[2];
    for (int e = threadIdx.x; e < 6 * NF; e += NT) {
        const int comp = e / NF, r = e - comp * NF;
        const int gx = wrapi(T0[0] - 2 - M + r % LF, nx);
        const int gy = wrapi(T0[1] - 2 - M + (r / LF) % LF, ny);
        const int gz = wrapi(T0[2] - 2 - M + r / (LF * LF), nz);
        const int64_t cell = ((int64_t)gz * ny + gy) * nx + gx;
        sf[e] = comp < 3 ? fields[comp * N + cell] : bfield[(comp - 3) * N + cell];
    }
    if (threadIdx.x == 0) n_fallback = 0;
    __syncthreads();
    const double c2 = g.c * g.c;
    const double qmdt2 = 0.5 * a.qm * g.dt;
    const int64_t begin = a.tile_start[tile], end = a.tile_start[tile + 1];
    unsigned int my_fallback = 0;
    for (int64_t p = begin + threadIdx.x; p < end; p += NT) {
        int i0[3];
        double d0[3];
        PosIO<double, 3>::load(a, p, i0, d0);
        double w[3];
        for (int ax = 0; ax < 3; ++ax) w[ax] = ((const double*)a.mom[ax])[p];
        Axis2<double> ax0[3];
        for (int ax = 0; ax < 3; ++ax) ax0[ax] = form_factor2<double>(d0[ax]);
        int rel[3];
        bool inside = true;
        for (int ax = 0; ax < 3; ++ax) {
            int r = i0[ax] - T0[ax];
            const int n = g.n[ax];
            if (r > n / 2) r -= n;
            if (r < -(n / 2)) r += n;
            rel[ax] = r;
            inside = inside && r >= -M && r <= T - 1 + M;
        }
        my_fallback += inside ? 0 : 1;
        double E[3], B[3];
        if (inside) {
            const int fb = (rel[0] + 2 + M) + (rel[1] + 2 + M) * LF + (rel[2] + 2 + M) * LF * LF;
            auto F = [&](int comp, int oa, int ob, int oc) -> double {
                return sf[comp * NF + fb + oa + ob * LF + oc * LF * LF];
            };
            gather3_o2<double>(ax0, F, E, B);
        } else {
            auto F = [&](int comp, int oa, int ob, int oc) -> double {
                const int64_t cell =
                    ((int64_t)wrapi(i0[2] + oc, nz) * ny + wrapi(i0[1] + ob, ny)) * nx + wrapi(i0[0] + oa, nx);
                return comp < 3 ? fields[comp * N + cell] : bfield[(comp - 3) * N + cell];
            };
            gather3_o2<double>(ax0, F, E, B);
        }
        for (int ax = 0; ax < 3; ++ax) B[ax] += g.bext[ax];
        push<double>(qmdt2, c2, E, B, w);
        for (int ax = 0; ax < 3; ++ax) ((double*)a.mom[ax])[p] = w[ax];
        const double inv = 1.0 / ::sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2] + c2);
        double disp[3], d1[3];
        for (int ax = 0; ax < 3; ++ax) disp[ax] = w[ax] * inv * g.cfl[ax];
        int delta[3] = {0, 0, 0};
        PosIO<double, 3>::move(a, p, g, i0, d0, disp, d1, delta, true);
        for (int ax = 0; ax < 3; ++ax) ((double*)spare.pos[ax])[p] = (double)i0[ax] + d0[ax];
        spare.id[p] = (int64_t)((delta[0] + 1) | ((delta[1] + 1) << 2) | ((delta[2] + 1) << 4));
    }
    if (my_fallback) atomicAdd(&n_fallback, my_fallback);
    __syncthreads();
    if (threadIdx.x == 0 && a.counters) {
        atomicAdd(&a.counters[1], (unsigned long long)n_fallback);
        atomicAdd(&a.counters[2], (unsigned long long)(end - begin));
    }
}

// One particle's windows for the current pass: start position from the spare
// copy, end position and cell shifts from pass 1.  Returns whether the
// particle is within the current region's margin of the tile.
struct O2Move {
    int i0[3], rel[3], s[3];
    bool still;
};

__device__ __forceinline__ bool o2_windows(const GridK& g, const StepArgs& a, const PartArrays& spare, int64_t p,
                                           const int T0[3], int M, double (&dm)[3][5], double (&dp)[3][5],
                                           O2Move& mv)
{
    const int64_t code = spare.id[p];
    bool inside = true;
    mv.still = true;
    for (int ax = 0; ax < 3; ++ax) {
        const double x0 = ((const double*)spare.pos[ax])[p];
        const double x1 = ((const double*)a.pos[ax])[p];
        const double f0 = floor(x0), f1 = floor(x1);
        mv.i0[ax] = (int)f0;
        const int delta = (int)((code >> (2 * ax)) & 3) - 1;
        const Axis2<double> e0 = form_factor2<double>(x0 - f0);
        const Axis2<double> e1 = form_factor2<double>(x1 - f1);
        const int shift = delta + e1.h - e0.h;
        mv.still = mv.still && shift == 0;
        window5_reg(e0.s, e1.s, shift, dm[ax], dp[ax]);
        mv.s[ax] = e0.h + (shift < 0 ? shift : 0) - 2;
        int r = mv.i0[ax] - T0[ax];
        const int n = g.n[ax];
        if (r > n / 2) r -= n;
        if (r < -(n / 2)) r += n;
        mv.rel[ax] = r;
        inside = inside && r >= -M && r <= kTile3 - 1 + M;
    }
    return inside;
}

// Pass 2.  Particles whose int(x + 1/2) stays put on every axis (most of
// them at thermal speeds) deposit their 144 contributions at once; the
// others are queued (their indices in the spare copy's weight array, at the
// tile's own index range) and deposit their 300 afterwards, so that a wave
// does not run both forms for a few lanes.
__global__ __launch_bounds__(kO2NT3) void k_deposit_o2_3d(GridK g, StepArgs a, PartArrays spare,
                                                          double* __restrict__ Jg)
{
    constexpr int T = kTile3, M = kO2M3b, NT = kO2NT3;
    constexpr int LJ = T + 6 + 2 * M, NJ = LJ * LJ * LJ;
    __shared__ double sj[3 * NJ];
    __shared__ unsigned int qn;
    const int tile = xcd_tile(blockIdx.x, g.ntiles);
    const int T0[3] = {(tile % g.nt[0]) * T, ((tile / g.nt[0]) % g.nt[1]) * T, (tile / (g.nt[0] * g.nt[1])) * T};
    const int64_t N = g.ncell;
    const int nx = g.n[0], ny = g.n[1], nz = g.n[2];
    for (int e = threadIdx.x; e < 3 * NJ; e += NT) sj[e] = 0.0;
    if (threadIdx.x == 0) qn = 0;
    __syncthreads();
    const int64_t begin = a.tile_start[tile], end = a.tile_start[tile + 1];
    int64_t* queue = (int64_t*)spare.weight + begin;  // end - begin entries
    auto deposit = [&](int64_t p, bool allow_still) {
        double dm[3][5], dp[3][5];
        O2Move mv;
        const bool inside = o2_windows(g, a, spare, p, T0, M, dm, dp, mv);
        if (allow_still && !(mv.still && inside)) {
            queue[atomicAdd(&qn, 1u)] = p;
            return;
        }
        const double qp = a.q * ((const double*)a.weight)[p];
        double jfac[3];
        for (int ax = 0; ax < 3; ++ax) jfac[ax] = g.jscale[ax] * qp;
        if (inside) {
            const int jb = (mv.rel[0] + mv.s[0] + 3 + M) + (mv.rel[1] + mv.s[1] + 3 + M) * LJ +
                           (mv.rel[2] + mv.s[2] + 3 + M) * LJ * LJ;
            auto S = [&](int comp, int ix, int iy, int iz, double v) {
                atomicAdd(&sj[comp * NJ + jb + ix + iy * LJ + iz * LJ * LJ], v);
            };
            if (allow_still) deposit3_o2_still<double>(dm, dp, jfac, S);
            else deposit3_o2<double>(dm, dp, jfac, S);
        } else {
            auto S = [&](int comp, int ix, int iy, int iz, double v) {
                const int64_t cell =
                    ((int64_t)wrapi(mv.i0[2] + mv.s[2] + iz, nz) * ny + wrapi(mv.i0[1] + mv.s[1] + iy, ny)) * nx +
                    wrapi(mv.i0[0] + mv.s[0] + ix, nx);
                add_global(&Jg[comp * N + cell], v);
            };
            deposit3_o2<double>(dm, dp, jfac, S);
        }
    };
    for (int64_t p = begin + threadIdx.x; p < end; p += NT) deposit(p, true);
    __syncthreads();
    const int64_t nq = qn;
    for (int64_t k = threadIdx.x; k < nq; k += NT) deposit(queue[k], false);
    __syncthreads();
    for (int e = threadIdx.x; e < 3 * NJ; e += NT) {
        const double v = sj[e];
        if (v == 0.0) continue;
        const int comp = e / NJ, r = e - comp * NJ;
        const int gx = wrapi(T0[0] - 3 - M + r % LJ, nx);
        const int gy = wrapi(T0[1] - 3 - M + (r / LJ) % LJ, ny);
        const int gz = wrapi(T0[2] - 3 - M + r / (LJ * LJ), nz);
        add_global(&Jg[comp * N + ((int64_t)gz * ny + gy) * nx + gx], v);
    }
}

// Current of given moves x0 -> x1 (positions in cell units, x1 not wrapped),
// one thread per move, global atomics.
template <int D>
__global__ __launch_bounds__(256) void k_deposit_pairs_o2(GridK g, const double* __restrict__ x0,
                                                          const double* __restrict__ x1,
                                                          const double* __restrict__ charge, int64_t n,
                                                          double* __restrict__ J)
{
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= n) return;
    int i0[3] = {0, 0, 0}, s[3] = {0, 0, 0};
    double dm[3][5], dp[3][5];
    for (int ax = 0; ax < D; ++ax) {
        const double a0 = x0[ax * n + p], a1 = x1[ax * n + p];
        const double f0 = floor(a0), f1 = floor(a1);
        const Axis2<double> e0 = form_factor2<double>(a0 - f0);
        const Axis2<double> e1 = form_factor2<double>(a1 - f1);
        i0[ax] = (int)f0;
        const int shift = ((int)f1 + e1.h) - ((int)f0 + e0.h);
        window5_reg(e0.s, e1.s, shift, dm[ax], dp[ax]);
        s[ax] = e0.h + (shift < 0 ? shift : 0) - 2;
    }
    const double q = charge[p];
    double jfac[3];
    for (int ax = 0; ax < 3; ++ax) jfac[ax] = g.jscale[ax] * q;
    // 2D3V: J^z from the z displacement, (q/V) (z1 - z0) dz/dt / 4
    const double jz = D == 2 ? q * 0.25 * g.inv_vol * (x1[2 * n + p] - x0[2 * n + p]) / g.inv_h[2] / g.dt : 0.0;
    const int64_t N = g.ncell;
    const int nx = g.n[0], ny = g.n[1], nz = g.n[2];
    auto S = [&](int comp, int ix, int iy, int iz, double v) {
        const int64_t cell = ((int64_t)(D == 3 ? wrapi(i0[2] + s[2] + iz, nz) : 0) * ny + wrapi(i0[1] + s[1] + iy, ny)) *
                                 nx +
                             wrapi(i0[0] + s[0] + ix, nx);
        add_global(&J[comp * N + cell], v);
    };
    if (D == 3) deposit3_o2<double>(dm, dp, jfac, S);
    else deposit2_o2<double>(dm, dp, jfac, jz, S);
}

// Charge density (Eq. rho) at order 2 1/2: cubic cell factors on 4 cells per
// axis, added into rho (charge per unit volume).  Positions x[ax][p], weights
// weight[p].
struct Rows3 {
    const double* x[3];
};

template <int D>
__global__ __launch_bounds__(256) void k_rho_o2(GridK g, Rows3 pos, const double* __restrict__ weight, int64_t n,
                                                double q, double* __restrict__ rho)
{
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= n) return;
    int i0[3] = {0, 0, 0};
    Axis2<double> w[3];
    for (int ax = 0; ax < 3; ++ax) {
        double d = 0.0;
        if (ax < D) {
            const double x = pos.x[ax][p];
            const double f = floor(x);
            i0[ax] = (int)f;
            d = x - f;
        }
        w[ax] = form_factor2<double>(d);
    }
    const double qv = q * weight[p] * g.inv_vol;
    const int nx = g.n[0], ny = g.n[1], nz = g.n[2];
    for (int c = 0; c < (D == 3 ? 4 : 1); ++c) {
        const double wz = D == 3 ? w[2].s[c] : 1.0;
        const int64_t kz = D == 3 ? (int64_t)wrapi(i0[2] + w[2].h - 2 + c, nz) * ny : 0;
        for (int b = 0; b < 4; ++b) {
            const int64_t jy = (kz + wrapi(i0[1] + w[1].h - 2 + b, ny)) * nx;
            for (int a = 0; a < 4; ++a)
                add_global(&rho[jy + wrapi(i0[0] + w[0].h - 2 + a, nx)], qv * wz * w[1].s[b] * w[0].s[a]);
        }
    }
}

unsigned blocks256(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

hipError_t launch_particle_step_o2(Ctx& c, Species& sp, hipStream_t s)
{
    if (sp.n == 0) return hipSuccess;
    StepArgs a{};
    for (int ax = 0; ax < 3; ++ax) {
        a.pos[ax] = sp.cur.pos[ax];
        a.mom[ax] = sp.cur.mom[ax];
    }
    a.weight = sp.cur.weight;
    a.tile_start = sp.tile_start;
    a.q = sp.d.q;
    a.qm = sp.d.q / sp.d.m;
    a.counters = c.counters;
    double* J = c.fields + 6 * c.k.ncell;
    if (c.k.dims == 3) {
        hipLaunchKernelGGL(k_push_o2_3d, dim3(c.k.ntiles), dim3(kO2NT3), 0, s, c.k, a, sp.alt, c.fields, c.bn);
        hipLaunchKernelGGL(k_deposit_o2_3d, dim3(c.k.ntiles), dim3(kO2NT3), 0, s, c.k, a, sp.alt, J);
    } else
        hipLaunchKernelGGL(k_step_o2<2>, dim3(c.k.ntiles), dim3(kO2NT2), 0, s, c.k, a, c.fields, c.bn, J);
    return hipGetLastError();
}

hipError_t launch_deposit_only_o2(const Ctx& c, const double* x0, const double* x1, const double* charge,
                                  int64_t n, double* J, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    if (c.k.dims == 3)
        hipLaunchKernelGGL(k_deposit_pairs_o2<3>, dim3(blocks256(n)), dim3(256), 0, s, c.k, x0, x1, charge, n, J);
    else
        hipLaunchKernelGGL(k_deposit_pairs_o2<2>, dim3(blocks256(n)), dim3(256), 0, s, c.k, x0, x1, charge, n, J);
    return hipGetLastError();
}

hipError_t launch_rho_o2(const Ctx& c, const double* const x[3], const double* weight, int64_t n, double q,
                         double* rho, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    Rows3 pos{{x[0], x[1], x[2]}};
    if (c.k.dims == 3)
        hipLaunchKernelGGL(k_rho_o2<3>, dim3(blocks256(n)), dim3(256), 0, s, c.k, pos, weight, n, q, rho);
    else
        hipLaunchKernelGGL(k_rho_o2<2>, dim3(blocks256(n)), dim3(256), 0, s, c.k, pos, weight, n, q, rho);
    return hipGetLastError();
}

}  // namespace pic
