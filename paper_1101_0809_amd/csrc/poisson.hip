// poisson.hip -- electrostatic initial field (Section 4.3): the discrete
// Poisson equation of Eq. poiphi for the cell-centred potential,
//   sum_a (-Phi_{c-e_a} + 2 Phi_c - Phi_{c+e_a}) / d_a^2 = 4 pi rho_c,
// on the periodic grid, then E from Eq. egradphidis,
//   E^x at face i = (Phi_{i-1} - Phi_i) / dx  (and y, z alike),
// so that div_h E = 4 pi rho cell by cell.  The operator is symmetric and
// positive definite on grid functions of zero mean; the right side has its
// mean removed (a uniform background) and conjugate gradients run on that
// subspace.  Scalars (alpha, beta, residual norms) stay on the device: each
// iteration is five launches with no host round trip; the host reads the
// residual every kCheck iterations to stop.
#include <algorithm>
#include <cmath>

#include "pic_internal.h"

namespace pic {
namespace {

constexpr int kThreads = 256;
constexpr int kBlocks = 1024;  // reduction workgroups
constexpr int kCheck = 16;

// device scalars: [0] r.r  [1] p.Ap  [2] target r.r  [4] b.b  [5] sum rho  [6] new r.r

__device__ __forceinline__ double block_sum(double v, double* sh)
{
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int w = kThreads / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    return sh[0];
}

// -Laplacian_h x at cell p
__device__ __forceinline__ double neg_lap(const GridK& g, const double* __restrict__ x, int64_t p)
{
    const int64_t row = p / g.n[0];
    const int i = (int)(p - row * g.n[0]);
    const int k = (int)(row / g.n[1]);
    const int j = (int)(row - (int64_t)k * g.n[1]);
    const int64_t sy = g.n[0], sz = (int64_t)g.n[0] * g.n[1];
    const int64_t im = i == 0 ? p + (g.n[0] - 1) : p - 1, ip = i == g.n[0] - 1 ? p - (g.n[0] - 1) : p + 1;
    const int64_t jm = j == 0 ? p + (int64_t)(g.n[1] - 1) * sy : p - sy;
    const int64_t jp = j == g.n[1] - 1 ? p - (int64_t)(g.n[1] - 1) * sy : p + sy;
    const int64_t km = k == 0 ? p + (int64_t)(g.n[2] - 1) * sz : p - sz;
    const int64_t kp = k == g.n[2] - 1 ? p - (int64_t)(g.n[2] - 1) * sz : p + sz;
    const double c = x[p];
    double r = (2.0 * c - x[im] - x[ip]) * g.inv_h[0] * g.inv_h[0] + (2.0 * c - x[jm] - x[jp]) * g.inv_h[1] * g.inv_h[1];
    if (g.n[2] > 1) r += (2.0 * c - x[km] - x[kp]) * g.inv_h[2] * g.inv_h[2];
    return r;
}

__global__ __launch_bounds__(kThreads) void k_sum(const double* __restrict__ x, int64_t n, double* __restrict__ part)
{
    __shared__ double sh[kThreads];
    double v = 0.0;
    for (int64_t p = (int64_t)blockIdx.x * kThreads + threadIdx.x; p < n; p += (int64_t)gridDim.x * kThreads) v += x[p];
    const double t = block_sum(v, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// out[slot] = sum of the nb partials (fixed order: deterministic)
__global__ __launch_bounds__(kThreads) void k_finish(const double* __restrict__ part, int nb, double* __restrict__ s,
                                                     int slot)
{
    __shared__ double sh[kThreads];
    double v = 0.0;
    for (int b = threadIdx.x; b < nb; b += kThreads) v += part[b];
    const double t = block_sum(v, sh);
    if (threadIdx.x == 0) s[slot] = t;
}

// b = 4 pi (rho - mean); r = b, p = b, phi = 0; partial b.b
__global__ __launch_bounds__(kThreads) void k_cg_init(int64_t n, const double* __restrict__ rho,
                                                      const double* __restrict__ s, double* __restrict__ phi,
                                                      double* __restrict__ r, double* __restrict__ pp,
                                                      double* __restrict__ part)
{
    __shared__ double sh[kThreads];
    const double mean = s[5] / (double)n;
    double v = 0.0;
    for (int64_t p = (int64_t)blockIdx.x * kThreads + threadIdx.x; p < n; p += (int64_t)gridDim.x * kThreads) {
        const double b = 4.0 * kPi * (rho[p] - mean);
        r[p] = b;
        pp[p] = b;
        phi[p] = 0.0;
        v += b * b;
    }
    const double t = block_sum(v, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// Ap = A p; partial p.Ap
__global__ __launch_bounds__(kThreads) void k_cg_apply(GridK g, const double* __restrict__ pp, double* __restrict__ ap,
                                                       double* __restrict__ part)
{
    __shared__ double sh[kThreads];
    double v = 0.0;
    for (int64_t p = (int64_t)blockIdx.x * kThreads + threadIdx.x; p < g.ncell; p += (int64_t)gridDim.x * kThreads) {
        const double a = neg_lap(g, pp, p);
        ap[p] = a;
        v += pp[p] * a;
    }
    const double t = block_sum(v, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// alpha = r.r / p.Ap; phi += alpha p; r -= alpha Ap; partial new r.r.  Once
// r.r has reached the target the iterate is frozen (alpha = 0): the host
// checks every kCheck iterations, and iterations past the rounding floor of
// this singular (periodic) system make p.Ap a rounding residue, alpha
// arbitrary and the residual grow again.
__global__ __launch_bounds__(kThreads) void k_cg_update(int64_t n, const double* __restrict__ s,
                                                        const double* __restrict__ pp, const double* __restrict__ ap,
                                                        double* __restrict__ phi, double* __restrict__ r,
                                                        double* __restrict__ part)
{
    __shared__ double sh[kThreads];
    const double alpha = s[0] > s[2] && s[1] > 0.0 ? s[0] / s[1] : 0.0;
    double v = 0.0;
    for (int64_t p = (int64_t)blockIdx.x * kThreads + threadIdx.x; p < n; p += (int64_t)gridDim.x * kThreads) {
        phi[p] += alpha * pp[p];
        const double rn = r[p] - alpha * ap[p];
        r[p] = rn;
        v += rn * rn;
    }
    const double t = block_sum(v, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// beta = new r.r / old r.r; p = r + beta p (reads s[0] old, s[6] new); p is
// left as it is once the iterate is frozen
__global__ __launch_bounds__(kThreads) void k_cg_direction(int64_t n, double* __restrict__ s,
                                                           const double* __restrict__ r, double* __restrict__ pp)
{
    if (!(s[0] > s[2])) return;
    const double beta = s[6] / s[0];
    for (int64_t p = (int64_t)blockIdx.x * kThreads + threadIdx.x; p < n; p += (int64_t)gridDim.x * kThreads)
        pp[p] = r[p] + beta * pp[p];
}

__global__ void k_set(double* s, int dst, int src)
{
    if (threadIdx.x == 0) s[dst] = s[src];
}
// s[dst] = f s[src]
__global__ void k_scale(double* s, int dst, int src, double f)
{
    if (threadIdx.x == 0) s[dst] = f * s[src];
}

// E from the potential (Eq. egradphidis)
__global__ __launch_bounds__(kThreads) void k_e_of_phi(GridK g, const double* __restrict__ phi, double* __restrict__ E)
{
    const int64_t p = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (p >= g.ncell) return;
    const int64_t N = g.ncell;
    const int64_t row = p / g.n[0];
    const int i = (int)(p - row * g.n[0]);
    const int k = (int)(row / g.n[1]);
    const int j = (int)(row - (int64_t)k * g.n[1]);
    const int64_t sy = g.n[0], sz = (int64_t)g.n[0] * g.n[1];
    const int64_t im = i == 0 ? p + (g.n[0] - 1) : p - 1;
    const int64_t jm = j == 0 ? p + (int64_t)(g.n[1] - 1) * sy : p - sy;
    const int64_t km = k == 0 ? p + (int64_t)(g.n[2] - 1) * sz : p - sz;
    const double c = phi[p];
    E[p] = (phi[im] - c) * g.inv_h[0];
    E[N + p] = (phi[jm] - c) * g.inv_h[1];
    E[2 * N + p] = g.n[2] > 1 ? (phi[km] - c) * g.inv_h[2] : 0.0;
}

__global__ __launch_bounds__(kThreads) void k_add_const(double* __restrict__ x, int64_t n, const double* __restrict__ s,
                                                        double scale)
{
    const double v = scale * s[5] / (double)n;
    for (int64_t p = (int64_t)blockIdx.x * kThreads + threadIdx.x; p < n; p += (int64_t)gridDim.x * kThreads) x[p] += v;
}

unsigned grid_for(int64_t n) { return (unsigned)std::min<int64_t>(kBlocks, (n + kThreads - 1) / kThreads); }

}  // namespace

hipError_t solve_poisson(Ctx& c, double* rho, bool neutralize, double tol, int64_t max_iter, int64_t* iters,
                         double* rel_residual, hipStream_t s)
{
    const int64_t n = c.k.ncell;
    // scratch: phi in bn (first plane), r, p, Ap in the adjoint planes;
    // partials and scalars in the reduction buffer
    double* phi = c.bn;
    double* r = c.adj;
    double* pp = c.adj + n;
    double* ap = c.adj + 2 * n;
    double* part = c.red;
    double* sc = c.red + kBlocks;
    const unsigned gb = grid_for(n);
    const int nb = (int)gb;
    hipLaunchKernelGGL(k_sum, dim3(gb), dim3(kThreads), 0, s, rho, n, part);
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(kThreads), 0, s, part, nb, sc, 5);
    if (neutralize)  // the uniform background: minus the mean charge density
        hipLaunchKernelGGL(k_add_const, dim3(gb), dim3(kThreads), 0, s, c.rho_bg, n, sc, -1.0);
    hipLaunchKernelGGL(k_cg_init, dim3(gb), dim3(kThreads), 0, s, n, rho, sc, phi, r, pp, part);
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(kThreads), 0, s, part, nb, sc, 4);
    hipLaunchKernelGGL(k_set, dim3(1), dim3(64), 0, s, sc, 0, 4);  // r.r = b.b at the start
    hipLaunchKernelGGL(k_scale, dim3(1), dim3(64), 0, s, sc, 2, 4, tol * tol);  // target r.r
    double host[7] = {0, 0, 0, 0, 0, 0, 0};
    hipError_t e = hipMemcpyAsync(host, sc, sizeof(host), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return e;
    const double bb = host[4];
    int64_t it = 0;
    double rr = bb;
    const double target = tol * tol * bb;
    while (bb > 0.0 && rr > target && it < max_iter) {
        for (int q = 0; q < kCheck && it < max_iter; ++q, ++it) {
            hipLaunchKernelGGL(k_cg_apply, dim3(gb), dim3(kThreads), 0, s, c.k, pp, ap, part);
            hipLaunchKernelGGL(k_finish, dim3(1), dim3(kThreads), 0, s, part, nb, sc, 1);
            hipLaunchKernelGGL(k_cg_update, dim3(gb), dim3(kThreads), 0, s, n, sc, pp, ap, phi, r, part);
            hipLaunchKernelGGL(k_finish, dim3(1), dim3(kThreads), 0, s, part, nb, sc, 6);
            hipLaunchKernelGGL(k_cg_direction, dim3(gb), dim3(kThreads), 0, s, n, sc, r, pp);
            hipLaunchKernelGGL(k_set, dim3(1), dim3(64), 0, s, sc, 0, 6);
        }
        e = hipMemcpyAsync(host, sc, sizeof(host), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return e;
        rr = host[0];
    }
    hipLaunchKernelGGL(k_e_of_phi, dim3((unsigned)((n + kThreads - 1) / kThreads)), dim3(kThreads), 0, s, c.k, phi,
                       c.fields);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    *iters = it;
    *rel_residual = bb > 0.0 ? std::sqrt(rr / bb) : 0.0;
    return hipSuccess;
}

}  // namespace pic
