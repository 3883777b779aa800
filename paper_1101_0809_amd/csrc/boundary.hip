// boundary.hip -- particle side of the open x boundary (pic_grid_desc.xbc =
// 1): after a step's deposit, a particle whose new position lies within
// PIC_ABSORB cells of a wall, x < PIC_ABSORB or x >= nx - 1 - PIC_ABSORB, is
// absorbed by setting its weight to zero.  It stays in the arrays and moves on
// without charge, so the sort and the particle kernels need no compaction.
// The decision reads the x cell only: the FP64 position's floor, or the FP32
// mode's packed cell, the same cell the particle kernels use.  One pass over
// the 4- or 8-byte x data in 16-byte loads, with a store only for the
// particles absorbed.
#include <algorithm>

#include "boundary.h"
#include "pic_math.h"

namespace pic {
namespace {

constexpr int kAbsorbThreads = 256;

// The x cells of particles 4q .. 4q+3 from one 16-byte load (FP32 mode: the
// packed cell words) or two (FP64: the positions).
template <class R>
__device__ __forceinline__ void x_cells4(const StepArgs& a, int64_t q, int c[4]);
template <>
__device__ __forceinline__ void x_cells4<float>(const StepArgs& a, int64_t q, int c[4])
{
    const uint4 v = ((const uint4*)a.cell)[q];
    const uint32_t w[4] = {v.x, v.y, v.z, v.w};
    for (int k = 0; k < 4; ++k) {
        int i[3];
        unpack_cell(w[k], i);
        c[k] = i[0];
    }
}
template <>
__device__ __forceinline__ void x_cells4<double>(const StepArgs& a, int64_t q, int c[4])
{
    const double2 u = ((const double2*)a.pos[0])[2 * q];
    const double2 v = ((const double2*)a.pos[0])[2 * q + 1];
    c[0] = (int)floor(u.x);
    c[1] = (int)floor(u.y);
    c[2] = (int)floor(v.x);
    c[3] = (int)floor(v.y);
}

// Four particles per thread (vec: the x array is 16-byte aligned); the last
// n % 4, or all of them without vec, one each.
template <class R, int D>
__global__ __launch_bounds__(kAbsorbThreads) void k_absorb(StepArgs a, int64_t n, int lo, int hi,
                                                           R* __restrict__ weight, int vec)
{
    const int64_t n4 = vec ? n / 4 : 0;
    const int64_t stride = (int64_t)gridDim.x * kAbsorbThreads;
    for (int64_t q = (int64_t)blockIdx.x * kAbsorbThreads + threadIdx.x; q < n4; q += stride) {
        int c[4];
        x_cells4<R>(a, q, c);
        for (int k = 0; k < 4; ++k)
            if ((c[k] < lo || c[k] >= hi) && weight[4 * q + k] != R(0)) weight[4 * q + k] = R(0);
    }
    for (int64_t p = 4 * n4 + (int64_t)blockIdx.x * kAbsorbThreads + threadIdx.x; p < n; p += stride) {
        int i[3];
        PosIO<R, D>::cell(a, p, i);
        if ((i[0] < lo || i[0] >= hi) && weight[p] != R(0)) weight[p] = R(0);
    }
}

template <class R, int D>
hipError_t absorb(const Species& sp, int nx, hipStream_t s)
{
    StepArgs a{};
    for (int ax = 0; ax < 3; ++ax) a.pos[ax] = sp.cur.pos[ax];
    a.cell = sp.cur.cell;
    const void* xs = sizeof(R) == 4 ? (const void*)a.cell : a.pos[0];
    const int vec = ((uintptr_t)xs & 15) == 0 ? 1 : 0;
    const int64_t want = ((vec ? sp.n / 4 : sp.n) + kAbsorbThreads) / kAbsorbThreads;
    const unsigned blocks = (unsigned)std::max<int64_t>(1, std::min<int64_t>(want, 8192));
    hipLaunchKernelGGL((k_absorb<R, D>), dim3(blocks), dim3(kAbsorbThreads), 0, s, a, sp.n, PIC_ABSORB,
                       nx - 1 - PIC_ABSORB, (R*)sp.cur.weight, vec);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_absorb(const Ctx& c, const Species& sp, hipStream_t s)
{
    if (sp.n == 0) return hipSuccess;
    const int nx = c.k.n[0];
    if (c.g.precision == PIC_FP64)
        return c.k.dims == 3 ? absorb<double, 3>(sp, nx, s) : absorb<double, 2>(sp, nx, s);
    return c.k.dims == 3 ? absorb<float, 3>(sp, nx, s) : absorb<float, 2>(sp, nx, s);
}

}  // namespace pic
