// diag.hip -- FP64 diagnostics on the GPU: charge density of the mobile
// particles (Eq. rho), discrete Gauss residual R = div_h E - 4 pi rho at cell
// centres and its drift from the reference R^0 (the charge-conservation
// invariant of Section 2), div_h B at nodes, field and kinetic energies
// (Section 4.1), including the half-step term sum (q dt / 2) u^{n-1/2} .
// E(x^n) with E gathered by the run's own interpolation.  Reductions run over
// a fixed grid of workgroups followed by one reducing workgroup, so the
// result does not depend on scheduling.
#include <mutex>

#include "pic_math.h"

namespace pic {
namespace {

constexpr int kRedThreads = 256;
constexpr int kRedBlocks = 1024;
constexpr int kSlots = 9;
// slots: 0 max|R-R0|  1 max|4 pi rho_m|  2 sum E^2  3 sum (B^n)^2  4 max|divB|
//        5 sum rho    6 nonfinite      7 kinetic   8 half-step term
constexpr bool kIsMax[kSlots] = {true, true, false, false, true, false, false, false, false};

__device__ __forceinline__ double combine(int slot, double a, double b)
{
    return kIsMax[slot] ? fmax(a, b) : a + b;
}

__device__ void block_reduce_store(double (&v)[kSlots], double* out)
{
    __shared__ double sh[kSlots][kRedThreads];
    for (int s = 0; s < kSlots; ++s) sh[s][threadIdx.x] = v[s];
    __syncthreads();
    for (int off = kRedThreads / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off)
            for (int s = 0; s < kSlots; ++s)
                sh[s][threadIdx.x] = combine(s, sh[s][threadIdx.x], sh[s][threadIdx.x + off]);
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int s = 0; s < kSlots; ++s) out[s] = sh[s][0];
}

__device__ __forceinline__ double gauss_at(const GridK& g, const double* f, const double* rho_m,
                                           const double* rho_bg, int64_t p, int i, int j, int k)
{
    const int64_t N = g.ncell;
    const int64_t sy = g.n[0], sz = (int64_t)g.n[0] * g.n[1];
    const int64_t ip = i == g.n[0] - 1 ? p - (g.n[0] - 1) : p + 1;
    const int64_t jp = j == g.n[1] - 1 ? p - (int64_t)(g.n[1] - 1) * sy : p + sy;
    const int64_t kp = k == g.n[2] - 1 ? p - (int64_t)(g.n[2] - 1) * sz : p + sz;
    const double div = (f[ip] - f[p]) * g.inv_h[0] + (f[N + jp] - f[N + p]) * g.inv_h[1] +
                       (f[2 * N + kp] - f[2 * N + p]) * g.inv_h[2];
    return div - 4.0 * kPi * (rho_m[p] + rho_bg[p]);
}

__device__ __forceinline__ void decode(const GridK& g, int64_t p, int& i, int& j, int& k)
{
    const int64_t row = p / g.n[0];
    i = (int)(p - row * g.n[0]);
    k = (int)(row / g.n[1]);
    j = (int)(row - (int64_t)k * g.n[1]);
}

__global__ __launch_bounds__(kRedThreads) void k_capture_r0(GridK g, const double* __restrict__ f,
                                                            const double* __restrict__ rho_m,
                                                            const double* __restrict__ rho_bg,
                                                            double* __restrict__ r0)
{
    for (int64_t p = (int64_t)blockIdx.x * kRedThreads + threadIdx.x; p < g.ncell;
         p += (int64_t)gridDim.x * kRedThreads) {
        int i, j, k;
        decode(g, p, i, j, k);
        r0[p] = gauss_at(g, f, rho_m, rho_bg, p, i, j, k);
    }
}

// The Gauss drift covers x cells gx0 .. gx1 and div B x nodes bx0 .. bx1 (all
// of them, unless the open x boundary excludes the walls' surroundings).
__global__ __launch_bounds__(kRedThreads) void k_diag_cells(GridK g, const double* __restrict__ f,
                                                            const double* __restrict__ rho_m,
                                                            const double* __restrict__ rho_bg,
                                                            const double* __restrict__ r0,
                                                            double* __restrict__ part, int gx0, int gx1,
                                                            int bx0, int bx1)
{
    double v[kSlots] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    const int64_t N = g.ncell;
    const int64_t sy = g.n[0], sz = (int64_t)g.n[0] * g.n[1];
    for (int64_t p = (int64_t)blockIdx.x * kRedThreads + threadIdx.x; p < N;
         p += (int64_t)gridDim.x * kRedThreads) {
        int i, j, k;
        decode(g, p, i, j, k);
        const double R = gauss_at(g, f, rho_m, rho_bg, p, i, j, k);
        if (i >= gx0 && i <= gx1) v[0] = fmax(v[0], fabs(R - r0[p]));
        v[1] = fmax(v[1], fabs(4.0 * kPi * rho_m[p]));
        const double ex = f[p], ey = f[N + p], ez = f[2 * N + p];
        v[2] += ex * ex + ey * ey + ez * ez;
        // B^n = B^{n-1/2} - (1/2) curl_h E^n
        const int64_t im = i == 0 ? p + (g.n[0] - 1) : p - 1;
        const int64_t jm = j == 0 ? p + (int64_t)(g.n[1] - 1) * sy : p - sy;
        const int64_t km = k == 0 ? p + (int64_t)(g.n[2] - 1) * sz : p - sz;
        const double* Ex = f;
        const double* Ey = f + N;
        const double* Ez = f + 2 * N;
        const double* Bx = f + 3 * N;
        const double* By = f + 4 * N;
        const double* Bz = f + 5 * N;
        const double bx = Bx[p] - g.half_cfl[1] * (ez - Ez[jm]) + g.half_cfl[2] * (ey - Ey[km]);
        const double by = By[p] - g.half_cfl[2] * (ex - Ex[km]) + g.half_cfl[0] * (ez - Ez[im]);
        const double bz = Bz[p] - g.half_cfl[0] * (ey - Ey[im]) + g.half_cfl[1] * (ex - Ex[jm]);
        v[3] += bx * bx + by * by + bz * bz;
        const double db = (Bx[p] - Bx[im]) * g.inv_h[0] + (By[p] - By[jm]) * g.inv_h[1] +
                          (Bz[p] - Bz[km]) * g.inv_h[2];
        if (i >= bx0 && i <= bx1) v[4] = fmax(v[4], fabs(db));
        v[5] += rho_m[p] + rho_bg[p];
        for (int c = 0; c < 6; ++c)
            if (!isfinite(f[c * N + p])) v[6] += 1.0;
    }
    block_reduce_store(v, part + (int64_t)blockIdx.x * kSlots);
}

// E^n at a particle with the run's interpolation (0: alternating order 1 1/2,
// 1: alternating order 2 1/2, 2: the conventional uniform order of Eq.
// wrong1), read from the grid.
template <int D>
__device__ __forceinline__ void gather_e(const GridK& g, int scheme, const double* f, const int i0[3],
                                        const double d0[3], double E[3])
{
    const int64_t N = g.ncell;
    auto F = [&](int comp, int oa, int ob, int oc) -> double {
        const int64_t cell = ((int64_t)(D == 3 ? wrapi(i0[2] + oc, g.n[2]) : 0) * g.n[1] + wrapi(i0[1] + ob, g.n[1])) *
                                 g.n[0] +
                             wrapi(i0[0] + oa, g.n[0]);
        return f[comp * N + cell];
    };
    double B[3];
    if (scheme == 1) {
        Axis2<double> w[3];
        for (int a = 0; a < 3; ++a) w[a] = form_factor2<double>(a < D ? d0[a] : 0.0);
        if (D == 3) gather3_o2<double>(w, F, E, B);
        else gather2_o2<double>(w, F, E, B);
    } else if (scheme == 2) {
        AxisC<double> w[3];
        for (int a = 0; a < 3; ++a) w[a] = form_factor_conv<double>(a < D ? d0[a] : 0.0);
        if (D == 3) gather3_conv<double>(w, F, E, B);
        else gather2_conv<double>(w, F, E, B);
    } else {
        Axis<double> w[3];
        for (int a = 0; a < 3; ++a) w[a] = form_factor<double>(a < D ? d0[a] : 0.0);
        if (D == 3) gather3<double>(w, F, E, B);
        else gather2<double>(w, F, E, B);
    }
}

template <class R, int D>
__global__ __launch_bounds__(kRedThreads) void k_diag_particles(GridK g, int scheme, PartArrays a, int64_t n,
                                                                double q, double m, double dt,
                                                                const double* __restrict__ fields,
                                                                double* __restrict__ part)
{
    const double inv_c2 = 1.0 / (g.c * g.c);
    StepArgs sa{};
    for (int ax = 0; ax < 3; ++ax) sa.pos[ax] = a.pos[ax];
    sa.cell = a.cell;
    double v[kSlots] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int64_t p = (int64_t)blockIdx.x * kRedThreads + threadIdx.x; p < n;
         p += (int64_t)gridDim.x * kRedThreads) {
        const double w0 = (double)((const R*)a.mom[0])[p];
        const double w1 = (double)((const R*)a.mom[1])[p];
        const double w2 = (double)((const R*)a.mom[2])[p];
        const double w2s = w0 * w0 + w1 * w1 + w2 * w2;
        if (!isfinite(w2s)) {
            v[6] += 1.0;
            continue;
        }
        const double gam = sqrt(1.0 + w2s * inv_c2);
        const double wt = (double)((const R*)a.weight)[p];
        v[7] += m * wt * w2s / (gam + 1.0);
        int i0[3];
        R dr[3];
        PosIO<R, D>::load(sa, p, i0, dr);
        double d0[3] = {0.0, 0.0, 0.0};
        for (int ax = 0; ax < D; ++ax) d0[ax] = (double)dr[ax];
        double E[3];
        gather_e<D>(g, scheme, fields, i0, d0, E);
        v[8] += 0.5 * q * wt * dt * (E[0] * w0 + E[1] * w1 + E[2] * w2) / gam;
    }
    block_reduce_store(v, part + (int64_t)blockIdx.x * kSlots);
}

__global__ __launch_bounds__(kRedThreads) void k_reduce_final(const double* __restrict__ part, int nb,
                                                              double* __restrict__ out)
{
    double v[kSlots] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int b = threadIdx.x; b < nb; b += kRedThreads)
        for (int s = 0; s < kSlots; ++s) v[s] = combine(s, v[s], part[(int64_t)b * kSlots + s]);
    block_reduce_store(v, out);
}

__global__ void k_zero_f64(double* p, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * kRedThreads + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kRedThreads)
        p[i] = 0.0;
}

// rho of the mobile species into rho_m (N doubles, cleared first by a kernel).
hipError_t mobile_rho(Ctx& c, double* rho_m, hipStream_t s)
{
    hipLaunchKernelGGL(k_zero_f64, dim3(kRedBlocks), dim3(kRedThreads), 0, s, rho_m, c.k.ncell);
    for (int i = 0; i < c.nsp; ++i)
        if (c.sp[i].d.mobile) {
            hipError_t e = launch_rho(c, c.sp[i], rho_m, s);
            if (e != hipSuccess) return e;
        }
    return hipGetLastError();
}

__global__ __launch_bounds__(kRedThreads) void k_sum2(const double* __restrict__ a, const double* __restrict__ b,
                                                      double* __restrict__ out, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * kRedThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kRedThreads)
        out[i] = a[i] + b[i];
}

}  // namespace

hipError_t launch_total_rho(Ctx& c, double* out, hipStream_t s)
{
    hipError_t e = mobile_rho(c, c.rho_m, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_sum2, dim3(kRedBlocks), dim3(kRedThreads), 0, s, c.rho_m, c.rho_bg, out, c.k.ncell);
    return hipGetLastError();
}

hipError_t launch_capture_r0(Ctx& c, hipStream_t s, double* rho_m)
{
    if (!rho_m) rho_m = c.rho_m;
    hipError_t e = mobile_rho(c, rho_m, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_capture_r0, dim3(kRedBlocks), dim3(kRedThreads), 0, s, c.k, c.fields,
                       rho_m, c.rho_bg, c.r0);
    return hipGetLastError();
}

hipError_t launch_diag(Ctx& c, pic_diag* out, hipStream_t s, double* rho_m, double* part)
{
    if (!rho_m) rho_m = c.rho_m;
    if (!part) part = c.red;
    hipError_t e = mobile_rho(c, rho_m, s);
    if (e != hipSuccess) return e;
    // partial layout: cells kRedBlocks x kSlots, then one block per species
    // open x boundary: the Gauss drift away from the absorbed charge, div B
    // where every B follows the curl of E (see pic_grid_desc.xbc)
    const int nx = c.k.n[0];
    const bool open = c.g.xbc == 1;
    hipLaunchKernelGGL(k_diag_cells, dim3(kRedBlocks), dim3(kRedThreads), 0, s, c.k, c.fields,
                       rho_m, c.rho_bg, c.r0, part, open ? PIC_ABSORB + 1 : 0,
                       open ? nx - 3 - PIC_ABSORB : nx - 1, open ? 1 : 0, open ? nx - 2 : nx - 1);
    int nb = kRedBlocks;
    int64_t nmob = 0;
    for (int i = 0; i < c.nsp; ++i) {
        const Species& sp = c.sp[i];
        if (!sp.d.mobile) continue;
        nmob += sp.n;
        double* pp = part + (int64_t)nb * kSlots;
        const int scheme = c.g.order == 2 ? 1 : (c.g.interp == 1 ? 2 : 0);
        const bool f64 = c.g.precision == PIC_FP64;
        if (c.k.dims == 3) {
            if (f64)
                hipLaunchKernelGGL((k_diag_particles<double, 3>), dim3(kRedBlocks), dim3(kRedThreads), 0, s, c.k,
                                   scheme, sp.cur, sp.n, sp.d.q, sp.d.m, c.g.dt, c.fields, pp);
            else
                hipLaunchKernelGGL((k_diag_particles<float, 3>), dim3(kRedBlocks), dim3(kRedThreads), 0, s, c.k,
                                   scheme, sp.cur, sp.n, sp.d.q, sp.d.m, c.g.dt, c.fields, pp);
        } else {
            if (f64)
                hipLaunchKernelGGL((k_diag_particles<double, 2>), dim3(kRedBlocks), dim3(kRedThreads), 0, s, c.k,
                                   scheme, sp.cur, sp.n, sp.d.q, sp.d.m, c.g.dt, c.fields, pp);
            else
                hipLaunchKernelGGL((k_diag_particles<float, 2>), dim3(kRedBlocks), dim3(kRedThreads), 0, s, c.k,
                                   scheme, sp.cur, sp.n, sp.d.q, sp.d.m, c.g.dt, c.fields, pp);
        }
        nb += kRedBlocks;
    }
    double* fin = part + (int64_t)nb * kSlots;
    hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(kRedThreads), 0, s, part, nb, fin);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    double h[kSlots];
    e = hipMemcpyAsync(h, fin, sizeof(h), hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return e;
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return e;
    const double V = c.g.dx * c.g.dy * c.g.dz;
    out->step = c.step;
    out->n_particles = nmob;
    out->kinetic = h[7];
    out->kinetic_half_step = h[8];
    out->field_e = V / (8.0 * kPi) * h[2];
    out->field_b = V / (8.0 * kPi) * h[3];
    out->charge = V * h[5];
    out->gauss_abs = h[0];
    out->rho_mobile_max = h[1];
    out->gauss_rel = h[1] > 0.0 ? h[0] / h[1] : h[0];
    out->divb_max = h[4];
    out->nonfinite = (int64_t)h[6];
    return hipSuccess;
}

size_t diag_partials_doubles(int nsp) { return (size_t)(kRedBlocks * (1 + nsp) + 1) * kSlots; }

}  // namespace pic

// ---------------------------------------------------------------------------
// Diagnostics without a workspace (pic_diagnostics_static): the mobile charge
// density and the reduction partials live in this file-scope device array,
// one per GPU, held until the process ends.  In host code the array's name
// stands for a host-side shadow, not the device memory: the device address
// comes from hipGetSymbolAddress, once per device, and only that address is
// handed to kernels.  Calls on one GPU share the array; calls that overlap on
// one GPU race.
// ---------------------------------------------------------------------------
static __device__ __align__(256) double scratch[pic::kStaticScratchBytes / sizeof(double)];

namespace pic {
namespace {

constexpr int kMaxDevices = 64;
double* g_scratch[kMaxDevices] = {};
std::mutex g_scratch_mutex;

}  // namespace

size_t static_scratch_doubles(const Ctx& c)
{
    return align_up((size_t)c.k.ncell, 32) + diag_partials_doubles(c.nsp);
}

hipError_t static_scratch_address(double** out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch[dev] = (double*)p;
    }
    *out = g_scratch[dev];
    return hipSuccess;
}

}  // namespace pic
