// fields.hip -- staggered-grid (Yee) field updates of the paper's Appendix:
// the B half step (Eq. updateB) and the E update (Eq. escheme).
//
// Storage (see pic.h): FP64 planes [k][j][i], i fastest, periodic.
//   Ex(i, j+1/2, k+1/2)  Ey(i+1/2, j, k+1/2)  Ez(i+1/2, j+1/2, k)
//   Bx(i+1/2, j, k)      By(i, j+1/2, k)      Bz(i, j, k+1/2)
// One thread per cell, consecutive threads on consecutive i, so every plane is
// streamed with unit stride; the backward / forward neighbours along y and z
// are re-reads of rows that the same or a neighbouring workgroup just fetched
// and are served from L2.  Both kernels are HBM-bound (9 or 12 FP64 values
// moved per cell).
#include <algorithm>

#include "pic_internal.h"

namespace pic {
namespace {

constexpr int kFieldThreads = 256;

struct CellIdx {
    int64_t p;
    int i, j, k;
};

__device__ __forceinline__ CellIdx cell_of(int64_t p, const GridK& g)
{
    CellIdx c;
    c.p = p;
    const int64_t row = p / g.n[0];
    c.i = (int)(p - row * g.n[0]);
    c.k = (int)(row / g.n[1]);
    c.j = (int)(row - (int64_t)c.k * g.n[1]);
    return c;
}

// B <- B - (1/2) curl_h E
__global__ __launch_bounds__(kFieldThreads) void k_half_b(GridK g, double* __restrict__ f)
{
    const int64_t p = (int64_t)blockIdx.x * kFieldThreads + threadIdx.x;
    if (p >= g.ncell) return;
    const CellIdx c = cell_of(p, g);
    const int64_t N = g.ncell;
    const double* Ex = f;
    const double* Ey = f + N;
    const double* Ez = f + 2 * N;
    double* Bx = f + 3 * N;
    double* By = f + 4 * N;
    double* Bz = f + 5 * N;
    const int64_t sx = 1, sy = g.n[0], sz = (int64_t)g.n[0] * g.n[1];
    const int64_t im = c.i == 0 ? p + (g.n[0] - 1) * sx : p - sx;
    const int64_t jm = c.j == 0 ? p + (int64_t)(g.n[1] - 1) * sy : p - sy;
    const int64_t km = c.k == 0 ? p + (int64_t)(g.n[2] - 1) * sz : p - sz;
    const double ex = Ex[p], ey = Ey[p], ez = Ez[p];
    const double hx = g.half_cfl[0], hy = g.half_cfl[1], hz = g.half_cfl[2];
    Bx[p] = Bx[p] - hy * (ez - Ez[jm]) + hz * (ey - Ey[km]);
    By[p] = By[p] - hz * (ex - Ex[km]) + hx * (ez - Ez[im]);
    double bz = Bz[p] - hx * (ey - Ey[im]) + hy * (ex - Ex[jm]);
    if (g.src_kind == 1 && c.i == g.src_plane)  // B^z at the plane is scattered-field:
        bz += hx * g.aux[2];                   // remove the incident E^y of face plane+1/2
    Bz[p] = bz;
}

// Both B half steps of a time step at once (they use the same E^n): B^n =
// B^{n-1/2} - (1/2) curl_h E^n to bn, then B^{n+1/2} = B^n - (1/2) curl_h E^n
// in place, each half step with the same expression and rounding as k_half_b.
// With the open x boundary (mur != null, pic_grid_desc.xbc): the planes one
// cell inside the walls save their B^y, B^z of n - 1/2 to mur ([side][y, z]
// [ny nz], side 0 the plane x = 1, side 1 the plane x = nx - 2), the walls
// x = 0 and x = nx - 1 keep theirs in place for k_mur_walls, and the outside
// layer's B^x is set to zero.  The walls' B^n in bn is the plain half step;
// no particle within the box reads it.
__global__ __launch_bounds__(kFieldThreads) void k_half_b_pair(GridK g, double* __restrict__ f,
                                                               double* __restrict__ bn,
                                                               unsigned long long* __restrict__ zero, int nzero,
                                                               double* __restrict__ mur)
{
    const int64_t p = (int64_t)blockIdx.x * kFieldThreads + threadIdx.x;
    if (p < nzero) zero[p] = 0;  // counters of the particle kernels that follow
    if (p >= g.ncell) return;
    const CellIdx c = cell_of(p, g);
    const int64_t N = g.ncell;
    const double* Ex = f;
    const double* Ey = f + N;
    const double* Ez = f + 2 * N;
    double* Bx = f + 3 * N;
    double* By = f + 4 * N;
    double* Bz = f + 5 * N;
    const int64_t sx = 1, sy = g.n[0], sz = (int64_t)g.n[0] * g.n[1];
    const int64_t im = c.i == 0 ? p + (g.n[0] - 1) * sx : p - sx;
    const int64_t jm = c.j == 0 ? p + (int64_t)(g.n[1] - 1) * sy : p - sy;
    const int64_t km = c.k == 0 ? p + (int64_t)(g.n[2] - 1) * sz : p - sz;
    const double ex = Ex[p], ey = Ey[p], ez = Ez[p];
    const double hx = g.half_cfl[0], hy = g.half_cfl[1], hz = g.half_cfl[2];
    const double cx = hy * (ez - Ez[jm]), dx = hz * (ey - Ey[km]);
    const double cy = hz * (ex - Ex[km]), dy = hx * (ez - Ez[im]);
    const double cz = hx * (ey - Ey[im]), dz = hy * (ex - Ex[jm]);
    const bool src = g.src_kind == 1 && c.i == g.src_plane;
    const double sc = hx * g.aux[2];
    double bx = Bx[p] - cx + dx;
    double by = By[p] - cy + dy;
    double bz = Bz[p] - cz + dz;
    if (src) bz += sc;
    bn[p] = bx;
    bn[N + p] = by;
    bn[2 * N + p] = bz;
    bx = bx - cx + dx;
    by = by - cy + dy;
    bz = bz - cz + dz;
    if (src) bz += sc;
    if (mur) {
        const int nx = g.n[0];
        const int64_t nyz = (int64_t)g.n[1] * g.n[2], q = (int64_t)c.k * g.n[1] + c.j;
        if (c.i == 1 || c.i == nx - 2) {
            double* sv = mur + (c.i == 1 ? 0 : 2 * nyz);
            sv[q] = By[p];
            sv[nyz + q] = Bz[p];
        }
        if (c.i == 0 || c.i == nx - 1) {  // walls: k_mur_walls sets B^y, B^z
            Bx[p] = c.i == 0 ? bx : 0.0;
            return;
        }
    }
    Bx[p] = bx;
    By[p] = by;
    Bz[p] = bz;
}

// Open x boundary: Mur's first-order condition on the walls' B^y, B^z,
// B_wall^{n+1/2} = B_in^{n-1/2} + k (B_in^{n+1/2} - B_wall^{n-1/2}), with
// B_in^{n-1/2} from mur and B_wall^{n-1/2} still in place (k_half_b_pair).
// One thread per wall point: side = blockIdx.y.
__global__ __launch_bounds__(kFieldThreads) void k_mur_walls(GridK g, double* __restrict__ f,
                                                             const double* __restrict__ mur, double kmur)
{
    const int64_t nyz = (int64_t)g.n[1] * g.n[2];
    const int64_t q = (int64_t)blockIdx.x * kFieldThreads + threadIdx.x;
    if (q >= nyz) return;
    const int side = blockIdx.y;
    const int nx = g.n[0];
    const int64_t N = g.ncell;
    const int64_t pw = q * nx + (side == 0 ? 0 : nx - 1);
    const int64_t pi = q * nx + (side == 0 ? 1 : nx - 2);
    double* By = f + 4 * N;
    double* Bz = f + 5 * N;
    const double* sv = mur + 2 * nyz * side;
    By[pw] = sv[q] + kmur * (By[pi] - By[pw]);
    Bz[pw] = sv[nyz + q] + kmur * (Bz[pi] - Bz[pw]);
}

// The source's auxiliary line, advanced by a one-workgroup kernel after each
// grid kernel: the grid's B correction uses the line's E^y of time n, its E
// correction the line's B^z of time n + 1/2, the values before each advance.
__device__ void aux_half_b(const GridK& g)
{
    double* ey = g.aux;
    double* bz = g.aux + PIC_AUX;
    const double hx = g.half_cfl[0];
    for (int a = 1 + threadIdx.x; a < PIC_AUX; a += kFieldThreads) bz[a] = bz[a] - hx * (ey[a] - ey[a - 1]);
}

__device__ void aux_update_e(const GridK& g, double t)
{
    double* ey = g.aux;
    const double* bz = g.aux + PIC_AUX;
    const double cx = g.cfl[0];
    for (int a = 1 + threadIdx.x; a < PIC_AUX - 1; a += kFieldThreads) ey[a] = ey[a] - cx * (bz[a + 1] - bz[a]);
    if (threadIdx.x == 0) {
        double ramp = 1.0;
        if (t < g.src_ramp) {
            const double s = sin(0.5 * kPi * t / g.src_ramp);
            ramp = s * s;
        }
        ey[0] = g.src_amp * ramp * sin(g.src_omega * t);
    }
}

__global__ __launch_bounds__(kFieldThreads) void k_aux_half_b(GridK g) { aux_half_b(g); }
__global__ __launch_bounds__(kFieldThreads) void k_aux_half_b_pair(GridK g)
{
    aux_half_b(g);
    __syncthreads();
    aux_half_b(g);
}
__global__ __launch_bounds__(kFieldThreads) void k_aux_update_e(GridK g, double t) { aux_update_e(g, t); }

// E <- E - 4 pi dt J + curl_h B ; J <- 0.  open: the open x boundary's
// outside layer x in [nx - 1, nx) gets E^y = E^z = 0.
__global__ __launch_bounds__(kFieldThreads) void k_update_e(GridK g, double* __restrict__ f, int open)
{
    const int64_t p = (int64_t)blockIdx.x * kFieldThreads + threadIdx.x;
    if (p >= g.ncell) return;
    const CellIdx c = cell_of(p, g);
    const int64_t N = g.ncell;
    double* Ex = f;
    double* Ey = f + N;
    double* Ez = f + 2 * N;
    const double* Bx = f + 3 * N;
    const double* By = f + 4 * N;
    const double* Bz = f + 5 * N;
    double* Jx = f + 6 * N;
    double* Jy = f + 7 * N;
    double* Jz = f + 8 * N;
    const int64_t sx = 1, sy = g.n[0], sz = (int64_t)g.n[0] * g.n[1];
    const int64_t ip = c.i == g.n[0] - 1 ? p - (g.n[0] - 1) * sx : p + sx;
    const int64_t jp = c.j == g.n[1] - 1 ? p - (int64_t)(g.n[1] - 1) * sy : p + sy;
    const int64_t kp = c.k == g.n[2] - 1 ? p - (int64_t)(g.n[2] - 1) * sz : p + sz;
    const double bx = Bx[p], by = By[p], bz = Bz[p];
    const double cx = g.cfl[0], cy = g.cfl[1], cz = g.cfl[2];
    Ex[p] = Ex[p] - g.fourpidt * Jx[p] + cy * (Bz[jp] - bz) - cz * (By[kp] - by);
    double ey = Ey[p] - g.fourpidt * Jy[p] + cz * (Bx[kp] - bx) - cx * (Bz[ip] - bz);
    if (g.src_kind == 1 && c.i == g.src_plane)  // E^y at face plane+1/2 is total-field:
        ey += cx * g.aux[PIC_AUX + 2];         // add the incident B^z of node plane
    double ez = Ez[p] - g.fourpidt * Jz[p] + cx * (By[ip] - by) - cy * (Bx[jp] - bx);
    if (open && c.i == g.n[0] - 1) ey = ez = 0.0;
    Ey[p] = ey;
    Ez[p] = ez;
    Jx[p] = 0.0;
    Jy[p] = 0.0;
    Jz[p] = 0.0;
}

// ---------------------------------------------------------------------------
// Vector-potential form (Section 4.2, Eq. dadt): A at the E points,
// A^{n+1/2} = A^{n-1/2} - c dt E^n, and B = curl_h A with the same backward
// differences as the B update: B^x = (A^z - A^z_{j-1})/dy - (A^y - A^y_{k-1})/dz,
// B^y = (A^x - A^x_{k-1})/dz - (A^z - A^z_{i-1})/dx,
// B^z = (A^y - A^y_{i-1})/dx - (A^x - A^x_{j-1})/dy.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kFieldThreads) void k_advance_a(GridK g, const double* __restrict__ f,
                                                             double* __restrict__ A,
                                                             unsigned long long* __restrict__ zero, int nzero)
{
    const int64_t p = (int64_t)blockIdx.x * kFieldThreads + threadIdx.x;
    if (p < nzero) zero[p] = 0;  // counters of the particle kernels that follow
    if (p >= g.ncell) return;
    const int64_t N = g.ncell;
    const double cdt = g.c * g.dt;
    for (int a = 0; a < 3; ++a) A[a * N + p] -= cdt * f[a * N + p];
}

// curl_h of (A + s E) at cell p (s = c dt / 2 gives A^n from A^{n+1/2}).
__device__ __forceinline__ void curl_a(const GridK& g, const double* __restrict__ A, const double* __restrict__ E,
                                       double s, const CellIdx& c, double out[3])
{
    const int64_t N = g.ncell, p = c.p;
    const int64_t sy = g.n[0], sz = (int64_t)g.n[0] * g.n[1];
    const int64_t im = c.i == 0 ? p + (g.n[0] - 1) : p - 1;
    const int64_t jm = c.j == 0 ? p + (int64_t)(g.n[1] - 1) * sy : p - sy;
    const int64_t km = c.k == 0 ? p + (int64_t)(g.n[2] - 1) * sz : p - sz;
    auto v = [&](int comp, int64_t q) { return A[comp * N + q] + s * E[comp * N + q]; };
    out[0] = (v(2, p) - v(2, jm)) * g.inv_h[1] - (v(1, p) - v(1, km)) * g.inv_h[2];
    out[1] = (v(0, p) - v(0, km)) * g.inv_h[2] - (v(2, p) - v(2, im)) * g.inv_h[0];
    out[2] = (v(1, p) - v(1, im)) * g.inv_h[0] - (v(0, p) - v(0, jm)) * g.inv_h[1];
}

// B^n = curl_h A^n into bn (A^n = A^{n+1/2} + (c dt / 2) E^n) and B^{n+1/2} =
// curl_h A^{n+1/2} into the field buffer (bn may be null: B planes only).
__global__ __launch_bounds__(kFieldThreads) void k_b_of_a(GridK g, double* __restrict__ f, const double* __restrict__ A,
                                                          double* __restrict__ bn)
{
    const int64_t p = (int64_t)blockIdx.x * kFieldThreads + threadIdx.x;
    if (p >= g.ncell) return;
    const int64_t N = g.ncell;
    const CellIdx c = cell_of(p, g);
    double b[3];
    if (bn) {
        curl_a(g, A, f, 0.5 * g.c * g.dt, c, b);
        for (int a = 0; a < 3; ++a) bn[a * N + p] = b[a];
    }
    curl_a(g, A, f, 0.0, c, b);
    for (int a = 0; a < 3; ++a) f[(3 + a) * N + p] = b[a];
}

}  // namespace

hipError_t launch_field_half_b(const Ctx& c, hipStream_t s)
{
    const unsigned blocks = (unsigned)((c.k.ncell + kFieldThreads - 1) / kFieldThreads);
    hipLaunchKernelGGL(k_half_b, dim3(blocks), dim3(kFieldThreads), 0, s, c.k, c.fields);
    if (c.k.src_kind == 1)  // after the grid kernel, which reads the line's E^y only
        hipLaunchKernelGGL(k_aux_half_b, dim3(1), dim3(kFieldThreads), 0, s, c.k);
    return hipGetLastError();
}

// The open x boundary's walls: B^{n-1/2} of the inside planes goes to the
// adjoint scratch (4 ny nz doubles of its 3 nx ny nz), which an open-boundary
// context never uses for the adjoint.
hipError_t launch_field_half_b_pair(const Ctx& c, hipStream_t s, unsigned long long* zero, int nzero)
{
    const unsigned blocks = (unsigned)((std::max<int64_t>(c.k.ncell, nzero) + kFieldThreads - 1) / kFieldThreads);
    double* mur = c.g.xbc == 1 ? c.adj : nullptr;
    hipLaunchKernelGGL(k_half_b_pair, dim3(blocks), dim3(kFieldThreads), 0, s, c.k, c.fields, c.bn, zero, nzero,
                       mur);
    if (mur) {
        const int64_t nyz = (int64_t)c.k.n[1] * c.k.n[2];
        const double cdt = c.g.c * c.g.dt;
        hipLaunchKernelGGL(k_mur_walls, dim3((unsigned)((nyz + kFieldThreads - 1) / kFieldThreads), 2),
                           dim3(kFieldThreads), 0, s, c.k, c.fields, (const double*)mur,
                           (cdt - c.g.dx) / (cdt + c.g.dx));
    }
    if (c.k.src_kind == 1)  // the line's two half steps, after the grid kernel read its E^y
        hipLaunchKernelGGL(k_aux_half_b_pair, dim3(1), dim3(kFieldThreads), 0, s, c.k);
    return hipGetLastError();
}

hipError_t launch_field_update_e(const Ctx& c, hipStream_t s, int64_t step)
{
    const unsigned blocks = (unsigned)((c.k.ncell + kFieldThreads - 1) / kFieldThreads);
    hipLaunchKernelGGL(k_update_e, dim3(blocks), dim3(kFieldThreads), 0, s, c.k, c.fields, c.g.xbc == 1 ? 1 : 0);
    if (c.k.src_kind == 1)  // the line's E^y at t = (step + 1) dt
        hipLaunchKernelGGL(k_aux_update_e, dim3(1), dim3(kFieldThreads), 0, s, c.k,
                           (double)(step + 1) * c.k.dt);
    return hipGetLastError();
}

}  // namespace pic

namespace pic {

hipError_t launch_field_half_a_pair(const Ctx& c, hipStream_t s, unsigned long long* zero, int nzero)
{
    const unsigned blocks = (unsigned)((std::max<int64_t>(c.k.ncell, nzero) + kFieldThreads - 1) / kFieldThreads);
    hipLaunchKernelGGL(k_advance_a, dim3(blocks), dim3(kFieldThreads), 0, s, c.k, c.fields, c.avec, zero, nzero);
    const unsigned cb = (unsigned)((c.k.ncell + kFieldThreads - 1) / kFieldThreads);
    hipLaunchKernelGGL(k_b_of_a, dim3(cb), dim3(kFieldThreads), 0, s, c.k, c.fields, c.avec, c.bn);
    return hipGetLastError();
}

hipError_t launch_b_of_a(const Ctx& c, hipStream_t s)
{
    const unsigned cb = (unsigned)((c.k.ncell + kFieldThreads - 1) / kFieldThreads);
    hipLaunchKernelGGL(k_b_of_a, dim3(cb), dim3(kFieldThreads), 0, s, c.k, c.fields, (const double*)c.avec,
                       (double*)nullptr);
    return hipGetLastError();
}

}  // namespace pic
