// conventional.hip -- the particle step with the "conventional" uniform-order
// field interpolation of Eq. wrong1, the comparison of Section 5 (Fig. 2):
// gather with the mean of adjacent order-1 1/2 cell factors on a component's
// node axes, then the push (Appendix, Eq. p2), the position advance (Eq.
// coordscheme) and the order-1 1/2 charge-conserving current (Eq. current).
// FP64; the charge density and the current of given moves are those of the
// order-1 1/2 scheme.
//
// 2D3V: one workgroup per tile stages E^n, B^n (cells T0-1-M .. T0+T+1+M)
// and accumulates the current (T0-2-M .. T0+T+1+M) in LDS.  3D: the two
// regions do not fit in LDS together with a drift margin, so a first pass
// gathers, pushes and moves with the fields staged (margin 1, 105 KB), keeping
// the start position in the species' spare particle copy and the cell shifts
// in its id array, and a second pass deposits the current (margin 2, 98 KB):
// particles that stay in their cell first (54 contributions), the others
// queued (144).
#include "pic_math.h"

namespace pic {
namespace {

__device__ __forceinline__ void add_global(double* p, double v) { unsafeAtomicAdd(p, v); }

__device__ __forceinline__ int rel_of(int i, int t0, int n)
{
    int r = i - t0;
    if (r > n / 2) r -= n;
    if (r < -(n / 2)) r += n;
    return r;
}

constexpr int kCvT2 = kTile2, kCvM2 = 2, kCvNT2 = 256;

__global__ __launch_bounds__(kCvNT2) void k_step_conv2(GridK g, StepArgs a, const double* __restrict__ fields,
                                                     const double* __restrict__ bfield, double* __restrict__ Jg)
{
    constexpr int T = kCvT2, M = kCvM2, NT = kCvNT2;
    constexpr int LF = T + 3 + 2 * M, NF = LF * LF;  // cells T0-1-M .. T0+T+1+M
    constexpr int LJ = T + 4 + 2 * M, NJ = LJ * LJ;  // cells T0-2-M .. T0+T+1+M
    __shared__ double sf[6 * NF];
    __shared__ double sj[3 * NJ];
    const int tile = xcd_tile(blockIdx.x, g.ntiles);
    const int T0[2] = {(tile % g.nt[0]) * T, (tile / g.nt[0]) * T};
    const int64_t N = g.ncell;
    const int nx = g.n[0], ny = g.n[1];
    for (int e = threadIdx.x; e < 6 * NF; e += NT) {
        const int comp = e / NF, r = e - comp * NF;
        const int64_t cell = (int64_t)wrapi(T0[1] - 1 - M + r / LF, ny) * nx + wrapi(T0[0] - 1 - M + r % LF, nx);
        sf[e] = comp < 3 ? fields[comp * N + cell] : bfield[(comp - 3) * N + cell];
    }
    for (int e = threadIdx.x; e < 3 * NJ; e += NT) sj[e] = 0.0;
    __syncthreads();
    const double c = g.c, c2 = c * c;
    const double qmdt2 = 0.5 * a.qm * g.dt;
    const int64_t begin = a.tile_start[tile], end = a.tile_start[tile + 1];
    for (int64_t p = begin + threadIdx.x; p < end; p += NT) {
        int i0[3];
        double d0[3];
        PosIO<double, 2>::load(a, p, i0, d0);
        double w[3];
        for (int ax = 0; ax < 3; ++ax) w[ax] = ((const double*)a.mom[ax])[p];
        const double qp = a.q * ((const double*)a.weight)[p];
        AxisC<double> ax0[3];
        for (int ax = 0; ax < 3; ++ax) ax0[ax] = form_factor_conv<double>(d0[ax]);
        const int rel[2] = {rel_of(i0[0], T0[0], nx), rel_of(i0[1], T0[1], ny)};
        const bool inside = rel[0] >= -M && rel[0] <= T - 1 + M && rel[1] >= -M && rel[1] <= T - 1 + M;
        double E[3], B[3];
        if (inside) {
            const int fb = (rel[0] + 1 + M) + (rel[1] + 1 + M) * LF;
            auto F = [&](int comp, int oa, int ob, int) -> double { return sf[comp * NF + fb + oa + ob * LF]; };
            gather2_conv<double>(ax0, F, E, B);
        } else {
            auto F = [&](int comp, int oa, int ob, int) -> double {
                const int64_t cell = (int64_t)wrapi(i0[1] + ob, ny) * nx + wrapi(i0[0] + oa, nx);
                return comp < 3 ? fields[comp * N + cell] : bfield[(comp - 3) * N + cell];
            };
            gather2_conv<double>(ax0, F, E, B);
        }
        for (int ax = 0; ax < 3; ++ax) B[ax] += g.bext[ax];
        push<double>(qmdt2, c2, E, B, w);
        for (int ax = 0; ax < 3; ++ax) ((double*)a.mom[ax])[p] = w[ax];
        const double inv = 1.0 / ::sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2] + c2);
        double disp[3], d1[3];
        for (int ax = 0; ax < 3; ++ax) disp[ax] = w[ax] * inv * g.cfl[ax];
        int delta[3] = {0, 0, 0};
        PosIO<double, 2>::move(a, p, g, i0, d0, disp, d1, delta, true);
        double dm[3][4], dp[3][4], jfac[3];
        int s[2];
        for (int ax = 0; ax < 2; ++ax) {
            double s1[3];
            cell_weights<double>(d1[ax], s1);
            window<double>(ax0[ax].s, s1, delta[ax], dm[ax], dp[ax]);
            s[ax] = (delta[ax] < 0 ? -1 : 0) - 1;
        }
        for (int ax = 0; ax < 3; ++ax) jfac[ax] = g.jscale[ax] * qp;
        const double jz = qp * (0.25 * g.inv_vol) * c * w[2] * inv;
        if (inside) {
            const int jb = (rel[0] + s[0] + 2 + M) + (rel[1] + s[1] + 2 + M) * LJ;
            auto S = [&](int comp, int ix, int iy, int, double v) { atomicAdd(&sj[comp * NJ + jb + ix + iy * LJ], v); };
            deposit2<double>(dm, dp, jfac, jz, S);
        } else {
            auto S = [&](int comp, int ix, int iy, int, double v) {
                const int64_t cell = (int64_t)wrapi(i0[1] + s[1] + iy, ny) * nx + wrapi(i0[0] + s[0] + ix, nx);
                add_global(&Jg[comp * N + cell], v);
            };
            deposit2<double>(dm, dp, jfac, jz, S);
        }
    }
    __syncthreads();
    for (int e = threadIdx.x; e < 3 * NJ; e += NT) {
        const double v = sj[e];
        if (v == 0.0) continue;
        const int comp = e / NJ, r = e - comp * NJ;
        const int64_t cell = (int64_t)wrapi(T0[1] - 2 - M + r / LJ, ny) * nx + wrapi(T0[0] - 2 - M + r % LJ, nx);
        add_global(&Jg[comp * N + cell], v);
    }
}

constexpr int kCvM3a = 1, kCvM3b = 2, kCvNT3 = 512;

__global__ __launch_bounds__(kCvNT3) void k_push_conv3(GridK g, StepArgs a, PartArrays spare,
                                                     const double* __restrict__ fields,
                                                     const double* __restrict__ bfield)
{
    constexpr int T = kTile3, M = kCvM3a, NT = kCvNT3;
    constexpr int LF = T + 3 + 2 * M, NF = LF * LF * LF;  // cells T0-1-M .. T0+T+1+M
    __shared__ double sf[6 * NF];
    __shared__ unsigned int n_fallback;
    const int tile = xcd_tile(blockIdx.x, g.ntiles);
    const int T0[3] = {(tile % g.nt[0]) * T, ((tile / g.nt[0]) % g.nt[1]) * T, (tile / (g.nt[0] * g.nt[1])) * T};
    const int64_t N = g.ncell;
    const int nx = g.n[0], ny = g.n[1], nz = g.n[2];
    for (int e = threadIdx.x; e < 6 * NF; e += NT) {
        const int comp = e / NF, r = e - comp * NF;
        const int gx = wrapi(T0[0] - 1 - M + r % LF, nx);
        const int gy = wrapi(T0[1] - 1 - M + (r / LF) % LF, ny);
        const int gz = wrapi(T0[2] - 1 - M + r / (LF * LF), nz);
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
        AxisC<double> ax0[3];
        for (int ax = 0; ax < 3; ++ax) ax0[ax] = form_factor_conv<double>(d0[ax]);
        int rel[3];
        bool inside = true;
        for (int ax = 0; ax < 3; ++ax) {
            rel[ax] = rel_of(i0[ax], T0[ax], g.n[ax]);
            inside = inside && rel[ax] >= -M && rel[ax] <= T - 1 + M;
        }
        my_fallback += inside ? 0 : 1;
        double E[3], B[3];
        if (inside) {
            const int fb = (rel[0] + 1 + M) + (rel[1] + 1 + M) * LF + (rel[2] + 1 + M) * LF * LF;
            auto F = [&](int comp, int oa, int ob, int oc) -> double {
                return sf[comp * NF + fb + oa + ob * LF + oc * LF * LF];
            };
            gather3_conv<double>(ax0, F, E, B);
        } else {
            auto F = [&](int comp, int oa, int ob, int oc) -> double {
                const int64_t cell =
                    ((int64_t)wrapi(i0[2] + oc, nz) * ny + wrapi(i0[1] + ob, ny)) * nx + wrapi(i0[0] + oa, nx);
                return comp < 3 ? fields[comp * N + cell] : bfield[(comp - 3) * N + cell];
            };
            gather3_conv<double>(ax0, F, E, B);
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

__global__ __launch_bounds__(kCvNT3) void k_deposit_conv3(GridK g, StepArgs a, PartArrays spare,
                                                        double* __restrict__ Jg)
{
    constexpr int T = kTile3, M = kCvM3b, NT = kCvNT3;
    constexpr int LJ = T + 4 + 2 * M, NJ = LJ * LJ * LJ;  // cells T0-2-M .. T0+T+1+M
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
    auto deposit = [&](int64_t p, bool first) {
        const int64_t code = spare.id[p];
        int i0[3], rel[3], s[3];
        bool inside = true, still = true;
        double dm[3][4], dp[3][4], s0[3][3], s1[3][3];
        for (int ax = 0; ax < 3; ++ax) {
            const double x0 = ((const double*)spare.pos[ax])[p];
            const double x1 = ((const double*)a.pos[ax])[p];
            const double f0 = floor(x0);
            i0[ax] = (int)f0;
            const int delta = (int)((code >> (2 * ax)) & 3) - 1;
            still = still && delta == 0;
            cell_weights<double>(x0 - f0, s0[ax]);
            cell_weights<double>(x1 - floor(x1), s1[ax]);
            window<double>(s0[ax], s1[ax], delta, dm[ax], dp[ax]);
            s[ax] = (delta < 0 ? -1 : 0) - 1;
            rel[ax] = rel_of(i0[ax], T0[ax], g.n[ax]);
            inside = inside && rel[ax] >= -M && rel[ax] <= T - 1 + M;
        }
        if (first && !(still && inside)) {
            queue[atomicAdd(&qn, 1u)] = p;
            return;
        }
        const double qp = a.q * ((const double*)a.weight)[p];
        double jfac[3];
        for (int ax = 0; ax < 3; ++ax) jfac[ax] = g.jscale[ax] * qp;
        if (inside) {
            const int jb = (rel[0] + s[0] + 2 + M) + (rel[1] + s[1] + 2 + M) * LJ + (rel[2] + s[2] + 2 + M) * LJ * LJ;
            auto S = [&](int comp, int ix, int iy, int iz, double v) {
                atomicAdd(&sj[comp * NJ + jb + ix + iy * LJ + iz * LJ * LJ], v);
            };
            if (first) {
                deposit3_still<double>(s0, s1, jfac, S);
            } else {
                deposit3<double>(dm, dp, jfac, S);
            }
        } else {
            auto S = [&](int comp, int ix, int iy, int iz, double v) {
                const int64_t cell = ((int64_t)wrapi(i0[2] + s[2] + iz, nz) * ny + wrapi(i0[1] + s[1] + iy, ny)) * nx +
                                     wrapi(i0[0] + s[0] + ix, nx);
                add_global(&Jg[comp * N + cell], v);
            };
            deposit3<double>(dm, dp, jfac, S);
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
        const int gx = wrapi(T0[0] - 2 - M + r % LJ, nx);
        const int gy = wrapi(T0[1] - 2 - M + (r / LJ) % LJ, ny);
        const int gz = wrapi(T0[2] - 2 - M + r / (LJ * LJ), nz);
        add_global(&Jg[comp * N + ((int64_t)gz * ny + gy) * nx + gx], v);
    }
}

}  // namespace

hipError_t launch_particle_step_conv(Ctx& c, Species& sp, hipStream_t s)
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
        hipLaunchKernelGGL(k_push_conv3, dim3(c.k.ntiles), dim3(kCvNT3), 0, s, c.k, a, sp.alt, c.fields, c.bn);
        hipLaunchKernelGGL(k_deposit_conv3, dim3(c.k.ntiles), dim3(kCvNT3), 0, s, c.k, a, sp.alt, J);
    } else {
        hipLaunchKernelGGL(k_step_conv2, dim3(c.k.ntiles), dim3(kCvNT2), 0, s, c.k, a, c.fields, c.bn, J);
    }
    return hipGetLastError();
}

}  // namespace pic
