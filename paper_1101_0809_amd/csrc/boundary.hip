// boundary.hip -- particle side of the open x boundary (pic_grid_desc.xbc =
// 1): after a step's deposit, a particle whose new position lies within
// PIC_ABSORB cells of a wall, x < PIC_ABSORB or x >= nx - 1 - PIC_ABSORB, is
// absorbed by setting its weight to zero.  It stays in the arrays and moves on
// without charge, so the sort and the particle kernels need no compaction.
// The decision reads the x cell only: the FP64 position's floor, or the FP32
// mode's packed cell, the same cell the particle kernels use.  One pass over
// the 4- or 8-byte x data, with a store only for the particles absorbed.
#include <algorithm>

#include "boundary.h"
#include "pic_math.h"

namespace pic {
namespace {

constexpr int kAbsorbThreads = 256;

template <class R, int D>
__global__ __launch_bounds__(kAbsorbThreads) void k_absorb(StepArgs a, int64_t n, int lo, int hi,
                                                           R* __restrict__ weight)
{
    for (int64_t p = (int64_t)blockIdx.x * kAbsorbThreads + threadIdx.x; p < n;
         p += (int64_t)gridDim.x * kAbsorbThreads) {
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
    const int64_t want = (sp.n + kAbsorbThreads - 1) / kAbsorbThreads;
    const unsigned blocks = (unsigned)std::max<int64_t>(1, std::min<int64_t>(want, 8192));
    hipLaunchKernelGGL((k_absorb<R, D>), dim3(blocks), dim3(kAbsorbThreads), 0, s, a, sp.n, PIC_ABSORB,
                       nx - 1 - PIC_ABSORB, (R*)sp.cur.weight);
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
