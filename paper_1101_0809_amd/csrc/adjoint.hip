// adjoint.hip -- reverse-mode derivative (adjoint) of one time step (paper
// Appendix): gather (Eqs. alphax, betax), push (Eq. p2), position advance
// (Eq. coordscheme), charge-conserving current (Eq. current) and the Yee
// updates (Eqs. updateB, escheme), FP64.
//
// One step maps (E^n, B^{n-1/2}, x^n, w^{n-1/2}) to (E^{n+1}, B^{n+1/2},
// x^{n+1}, w^{n+1/2}) through
//   B^n = B^{n-1/2} - (1/2) C E^n,  B^{n+1/2} = B^n - (1/2) C E^n,
//   per particle: (E_p, B_p) = gather(x^n; E^n, B^n) + B_ext, w^{n+1/2} =
//   push(w^{n-1/2}, E_p, B_p), x^{n+1} = x^n + V(w^{n+1/2}), J += deposit,
//   E^{n+1} = E^n - 4 pi dt J + D B^{n+1/2},
// with C the curl that takes E to B (backward differences) and D the one
// that takes B to E (forward differences).  The curl is symmetric: the
// transpose of a backward difference is minus the forward one, and the two
// terms of each curl component swap places with opposite signs, so C^T = D
// and D^T = C.  Given the adjoints lambda of the state after the step, the
// adjoint of the state before it is
//   lambda_J = -4 pi dt lambda_E',          lambda_B2 = lambda_B' + C lambda_E',
//   lambda_E = lambda_E' - (1/2) D lambda_B2 + (particles) - (1/2) D lambda_Bn,
//   lambda_Bn = lambda_B2 + (particles),     lambda_B = lambda_Bn,
// and per particle the derivatives of its gather, push, move and deposit,
// evaluated by the same formulas as the step (pic_math.h) on forward-mode dual
// numbers.  The particle part adds alpha lambda_Ep into lambda_E and beta
// lambda_Bp into lambda_B (atomics) and sums lambda_Bp into the external-field
// gradient.
#include "pic_math.h"

namespace pic {
namespace {

// ---------------------------------------------------------------------------
// Forward-mode dual number: a value and its N partial derivatives.
// ---------------------------------------------------------------------------
template <int N>
struct Dual {
    double v;
    double d[N];
    __device__ Dual() : v(0.0)
    {
        for (int i = 0; i < N; ++i) d[i] = 0.0;
    }
    __device__ Dual(double x) : v(x)
    {
        for (int i = 0; i < N; ++i) d[i] = 0.0;
    }
    __device__ static Dual var(double x, int k)
    {
        Dual r(x);
        r.d[k] = 1.0;
        return r;
    }
    __device__ Dual& operator+=(const Dual& b)
    {
        v += b.v;
        for (int i = 0; i < N; ++i) d[i] += b.d[i];
        return *this;
    }
    __device__ Dual& operator-=(const Dual& b)
    {
        v -= b.v;
        for (int i = 0; i < N; ++i) d[i] -= b.d[i];
        return *this;
    }
    __device__ Dual& operator*=(const Dual& b)
    {
        for (int i = 0; i < N; ++i) d[i] = d[i] * b.v + v * b.d[i];
        v *= b.v;
        return *this;
    }
};

template <int N>
__device__ __forceinline__ Dual<N> operator+(Dual<N> a, const Dual<N>& b) { return a += b; }
template <int N>
__device__ __forceinline__ Dual<N> operator-(Dual<N> a, const Dual<N>& b) { return a -= b; }
template <int N>
__device__ __forceinline__ Dual<N> operator-(const Dual<N>& a)
{
    Dual<N> r(-a.v);
    for (int i = 0; i < N; ++i) r.d[i] = -a.d[i];
    return r;
}
template <int N>
__device__ __forceinline__ Dual<N> operator*(Dual<N> a, const Dual<N>& b) { return a *= b; }
template <int N>
__device__ __forceinline__ Dual<N> operator*(const Dual<N>& a, double b)
{
    Dual<N> r(a.v * b);
    for (int i = 0; i < N; ++i) r.d[i] = a.d[i] * b;
    return r;
}
template <int N>
__device__ __forceinline__ Dual<N> operator*(double b, const Dual<N>& a) { return a * b; }
template <int N>
__device__ __forceinline__ Dual<N> operator/(const Dual<N>& a, const Dual<N>& b)
{
    const double q = a.v / b.v;
    Dual<N> r(q);
    for (int i = 0; i < N; ++i) r.d[i] = (a.d[i] - q * b.d[i]) / b.v;
    return r;
}
template <int N>
__device__ __forceinline__ Dual<N> sqrt(const Dual<N>& a)
{
    const double s = ::sqrt(a.v);
    Dual<N> r(s);
    for (int i = 0; i < N; ++i) r.d[i] = a.d[i] * (0.5 / s);
    return r;
}

__device__ __forceinline__ void grid_add(double* p, double v) { unsafeAtomicAdd(p, v); }

constexpr int kAdjThreads = 256;
constexpr int kCurlThreads = 256;

struct CellNb {
    int64_t p, im, jm, km, ip, jp, kp;
};

__device__ __forceinline__ CellNb neighbours(int64_t p, const GridK& g)
{
    CellNb c;
    c.p = p;
    const int64_t row = p / g.n[0];
    const int i = (int)(p - row * g.n[0]);
    const int k = (int)(row / g.n[1]);
    const int j = (int)(row - (int64_t)k * g.n[1]);
    const int64_t sy = g.n[0], sz = (int64_t)g.n[0] * g.n[1];
    c.im = i == 0 ? p + (g.n[0] - 1) : p - 1;
    c.jm = j == 0 ? p + (int64_t)(g.n[1] - 1) * sy : p - sy;
    c.km = k == 0 ? p + (int64_t)(g.n[2] - 1) * sz : p - sz;
    c.ip = i == g.n[0] - 1 ? p - (g.n[0] - 1) : p + 1;
    c.jp = j == g.n[1] - 1 ? p - (int64_t)(g.n[1] - 1) * sy : p + sy;
    c.kp = k == g.n[2] - 1 ? p - (int64_t)(g.n[2] - 1) * sz : p + sz;
    return c;
}

// (C E) at cell c, component-wise: B <- B - (1/2) C E is the half step.
__device__ __forceinline__ void curl_c(const GridK& g, const double* E, const CellNb& c, double out[3])
{
    const int64_t N = g.ncell;
    const double* Ex = E;
    const double* Ey = E + N;
    const double* Ez = E + 2 * N;
    const double cx = g.cfl[0], cy = g.cfl[1], cz = g.cfl[2];
    out[0] = cy * (Ez[c.p] - Ez[c.jm]) - cz * (Ey[c.p] - Ey[c.km]);
    out[1] = cz * (Ex[c.p] - Ex[c.km]) - cx * (Ez[c.p] - Ez[c.im]);
    out[2] = cx * (Ey[c.p] - Ey[c.im]) - cy * (Ex[c.p] - Ex[c.jm]);
}

// (D B) at cell c: E <- E - 4 pi dt J + D B is the E update.
__device__ __forceinline__ void curl_d(const GridK& g, const double* B, const CellNb& c, double out[3])
{
    const int64_t N = g.ncell;
    const double* Bx = B;
    const double* By = B + N;
    const double* Bz = B + 2 * N;
    const double cx = g.cfl[0], cy = g.cfl[1], cz = g.cfl[2];
    out[0] = cy * (Bz[c.jp] - Bz[c.p]) - cz * (By[c.kp] - By[c.p]);
    out[1] = cz * (Bx[c.kp] - Bx[c.p]) - cx * (Bz[c.ip] - Bz[c.p]);
    out[2] = cx * (By[c.ip] - By[c.p]) - cy * (Bx[c.jp] - Bx[c.p]);
}

// B^n of the state (E^n, B^{n-1/2}) into bn, the state untouched.  Same
// expression as the step's first half step.
__global__ __launch_bounds__(kCurlThreads) void k_adj_bn(GridK g, const double* __restrict__ f,
                                                         double* __restrict__ bn)
{
    const int64_t p = (int64_t)blockIdx.x * kCurlThreads + threadIdx.x;
    if (p >= g.ncell) return;
    const int64_t N = g.ncell;
    const CellNb c = neighbours(p, g);
    const double *Ex = f, *Ey = f + N, *Ez = f + 2 * N;
    const double hx = g.half_cfl[0], hy = g.half_cfl[1], hz = g.half_cfl[2];
    bn[p] = f[3 * N + p] - hy * (Ez[p] - Ez[c.jm]) + hz * (Ey[p] - Ey[c.km]);
    bn[N + p] = f[4 * N + p] - hz * (Ex[p] - Ex[c.km]) + hx * (Ez[p] - Ez[c.im]);
    bn[2 * N + p] = f[5 * N + p] - hx * (Ey[p] - Ey[c.im]) + hy * (Ex[p] - Ex[c.jm]);
}

// lambda_J = -4 pi dt lambda_E';  lambda_B <- lambda_B' + C lambda_E' (the
// transpose of D is C: both are the curl, with backward and forward differences).
__global__ __launch_bounds__(kCurlThreads) void k_adj_pre(GridK g, const double* __restrict__ lamE,
                                                          double* __restrict__ lamB,
                                                          double* __restrict__ lamJ)
{
    const int64_t p = (int64_t)blockIdx.x * kCurlThreads + threadIdx.x;
    if (p >= g.ncell) return;
    const int64_t N = g.ncell;
    const CellNb c = neighbours(p, g);
    double ce[3];
    curl_c(g, lamE, c, ce);
    for (int k = 0; k < 3; ++k) {
        lamJ[k * N + p] = -g.fourpidt * lamE[k * N + p];
        lamB[k * N + p] += ce[k];
    }
}

// lambda_E <- lambda_E - (1/2) D lambda_B (B <- B - (1/2) C E, transpose of C = D).
__global__ __launch_bounds__(kCurlThreads) void k_adj_curl(GridK g, double* __restrict__ lamE,
                                                           const double* __restrict__ lamB)
{
    const int64_t p = (int64_t)blockIdx.x * kCurlThreads + threadIdx.x;
    if (p >= g.ncell) return;
    const CellNb c = neighbours(p, g);
    double db[3];
    curl_d(g, lamB, c, db);
    for (int k = 0; k < 3; ++k) lamE[k * g.ncell + p] -= 0.5 * db[k];
}

// Loss L = V/(8 pi) sum E^2 + (B^n)^2, B^n = B - (1/2) C E:
// dL/dB = 2 k B^n, dL/dE = 2 k E - k D B^n, k = V/(8 pi).  First kernel:
// B^n into tmp and lambda_B; second: lambda_E.
__global__ __launch_bounds__(kCurlThreads) void k_adj_seed_b(GridK g, const double* __restrict__ f,
                                                             double* __restrict__ lam,
                                                             double* __restrict__ tmp)
{
    const int64_t p = (int64_t)blockIdx.x * kCurlThreads + threadIdx.x;
    if (p >= g.ncell) return;
    const int64_t N = g.ncell;
    const CellNb c = neighbours(p, g);
    double ce[3];
    curl_c(g, f, c, ce);
    const double k2 = 2.0 / (8.0 * kPi * g.inv_vol);
    for (int k = 0; k < 3; ++k) {
        const double bn = f[(3 + k) * N + p] - 0.5 * ce[k];
        tmp[k * N + p] = bn;
        lam[(3 + k) * N + p] = k2 * bn;
    }
}

__global__ __launch_bounds__(kCurlThreads) void k_adj_seed_e(GridK g, const double* __restrict__ f,
                                                             double* __restrict__ lam,
                                                             const double* __restrict__ tmp)
{
    const int64_t p = (int64_t)blockIdx.x * kCurlThreads + threadIdx.x;
    if (p >= g.ncell) return;
    const CellNb c = neighbours(p, g);
    double db[3];
    curl_d(g, tmp, c, db);
    const double k1 = 1.0 / (8.0 * kPi * g.inv_vol);
    for (int k = 0; k < 3; ++k) lam[k * g.ncell + p] = 2.0 * k1 * f[k * g.ncell + p] - k1 * db[k];
}

struct AdjArgs {
    const double* pos[3];
    const double* mom[3];
    const double* weight;
    const int64_t* id;
    int64_t n;       // particles of the species
    int64_t count;   // row stride of lam_x, lam_w
    double q, qm;
    const double* E;     // E^n (3 planes)
    const double* Bn;    // B^n (3 planes)
    const double* lamJ;  // 3 planes
    double* lamE;        // 3 planes, accumulated
    double* lamB;        // 3 planes, accumulated
    double* lam_x;       // 3 x count, by particle id
    double* lam_w;       // 3 x count, by particle id
    double* lam_bext;    // 3, accumulated
};

// Add w * lam at the stencil points of one field component: per axis the node
// weights f (offsets 0, 1) or the cell weights s (offsets -1, 0, 1); in 2D the
// z axis is collapsed onto the single plane.
template <int D, bool NX, bool NY, bool NZ>
__device__ __forceinline__ void scatter_comp(double* dst, const Axis<double> (&w)[3], const int xi[3],
                                             const int yj[3], const int64_t zk[3], double lam)
{
    constexpr int ZLO = D == 3 ? (NZ ? 0 : -1) : 0, ZHI = D == 3 ? 1 : 0;
    for (int c = ZLO; c <= ZHI; ++c) {
        const double wz = D == 3 ? (NZ ? w[2].f[c] : w[2].s[c + 1]) : 1.0;
        for (int b = NY ? 0 : -1; b <= 1; ++b) {
            const double wy = NY ? w[1].f[b] : w[1].s[b + 1];
            for (int a = NX ? 0 : -1; a <= 1; ++a) {
                const double wx = NX ? w[0].f[a] : w[0].s[a + 1];
                grid_add(&dst[zk[c + 1] + yj[b + 1] + xi[a + 1]], wx * wy * wz * lam);
            }
        }
    }
}

template <int D>
__global__ __launch_bounds__(kAdjThreads) void k_adj_particles(GridK g, AdjArgs a)
{
    __shared__ double sb[3];
    if (threadIdx.x < 3) sb[threadIdx.x] = 0.0;
    __syncthreads();
    const int64_t p = (int64_t)blockIdx.x * kAdjThreads + threadIdx.x;
    double lbp[3] = {0.0, 0.0, 0.0};
    if (p < a.n) {
        const int64_t N = g.ncell;
        const int nx = g.n[0], ny = g.n[1], nz = g.n[2];
        const double c = g.c, c2 = c * c;
        int i0[3] = {0, 0, 0};
        double d0[3] = {0.0, 0.0, 0.0};
        for (int ax = 0; ax < D; ++ax) {
            const double x = a.pos[ax][p];
            const double fl = floor(x);
            i0[ax] = (int)fl;
            d0[ax] = x - fl;
        }
        const int64_t id = a.id[p];
        double w0[3];
        for (int k = 0; k < 3; ++k) w0[k] = a.mom[k][p];
        const double qp = a.q * a.weight[p];

        // gather, with the derivatives in the start offsets d0
        using DG = Dual<D>;
        Axis<DG> ax0[3];
        for (int ax = 0; ax < D; ++ax) ax0[ax] = form_factor<DG>(DG::var(d0[ax], ax));
        if (D == 2) ax0[2] = form_factor<DG>(DG(0.0));
        int xi[3], yj[3];
        int64_t zk[3];
        for (int o = 0; o < 3; ++o) {
            xi[o] = wrapi(i0[0] + o - 1, nx);
            yj[o] = wrapi(i0[1] + o - 1, ny) * nx;
            zk[o] = D == 3 ? (int64_t)wrapi(i0[2] + o - 1, nz) * nx * ny : 0;
        }
        auto F = [&](int comp, int da, int db, int dc) -> double {
            const int64_t cell = zk[dc + 1] + yj[db + 1] + xi[da + 1];
            return comp < 3 ? a.E[comp * N + cell] : a.Bn[(comp - 3) * N + cell];
        };
        DG Eg[3], Bg[3];
        if (D == 3) gather3<DG>(ax0, F, Eg, Bg);
        else gather2<DG>(ax0, F, Eg, Bg);

        // push, with the derivatives in (w, E_p, B_p)
        using DP = Dual<9>;
        DP wv[3], Ev[3], Bv[3];
        for (int k = 0; k < 3; ++k) {
            wv[k] = DP::var(w0[k], k);
            Ev[k] = DP::var(Eg[k].v, 3 + k);
            Bv[k] = DP::var(Bg[k].v + g.bext[k], 6 + k);
        }
        push<DP>(DP(0.5 * a.qm * g.dt), DP(c2), Ev, Bv, wv);
        double w1[3];
        for (int k = 0; k < 3; ++k) w1[k] = wv[k].v;

        // position advance: values only (d1 = d0 + disp - delta)
        const double inv = 1.0 / ::sqrt(w1[0] * w1[0] + w1[1] * w1[1] + w1[2] * w1[2] + c2);
        double disp[3];
        for (int ax = 0; ax < 3; ++ax) disp[ax] = w1[ax] * inv * g.cfl[ax];
        double d1[3] = {0.0, 0.0, 0.0};
        int delta[3] = {0, 0, 0};
        StepArgs none{};
        PosIO<double, D>::move(none, p, g, i0, d0, disp, d1, delta, false);

        // current, with the derivatives in (d0, d1[, w^{n+1/2} in 2D]), each
        // contribution weighted by lambda_J at its cell
        constexpr int NV = D == 3 ? 6 : 7;
        using DD = Dual<NV>;
        DD dm[3][4], dp[3][4];
        for (int ax = 0; ax < D; ++ax) {
            DD s0[3], s1[3];
            cell_weights<DD>(DD::var(d0[ax], ax), s0);
            cell_weights<DD>(DD::var(d1[ax], D + ax), s1);
            window<DD>(s0, s1, delta[ax], dm[ax], dp[ax]);
        }
        DD jfac[3];
        for (int k = 0; k < 3; ++k) jfac[k] = DD(g.jscale[k] * qp);
        DD jz2(0.0);
        if (D == 2) {
            DD wz[3];
            for (int k = 0; k < 3; ++k) wz[k] = DD::var(w1[k], 2 * D + k);
            const DD invd = DD(1.0) / sqrt(wz[0] * wz[0] + wz[1] * wz[1] + wz[2] * wz[2] + DD(c2));
            jz2 = DD(qp) * DD(0.25 * g.inv_vol) * DD(c) * wz[2] * invd;
        }
        int cxs[4], cys[4];
        int64_t czs[4];
        for (int o = 0; o < 4; ++o) {
            const int sx = i0[0] + (delta[0] < 0 ? -1 : 0) - 1;
            const int sy = i0[1] + (delta[1] < 0 ? -1 : 0) - 1;
            const int sz = i0[2] + (delta[2] < 0 ? -1 : 0) - 1;
            cxs[o] = wrapi(sx + o, nx);
            cys[o] = wrapi(sy + o, ny) * nx;
            czs[o] = D == 3 ? (int64_t)wrapi(sz + o, nz) * nx * ny : 0;
        }
        double gd[NV];
        for (int k = 0; k < NV; ++k) gd[k] = 0.0;
        auto S = [&](int comp, int ix, int iy, int iz, const DD& v) {
            const double lj = a.lamJ[comp * N + czs[iz] + cys[iy] + cxs[ix]];
            for (int k = 0; k < NV; ++k) gd[k] += lj * v.d[k];
        };
        if (D == 3) deposit3<DD>(dm, dp, jfac, S);
        else deposit2<DD>(dm, dp, jfac, jz2, S);

        // reverse assembly
        double lx1[3] = {0.0, 0.0, 0.0}, lw1[3];
        for (int ax = 0; ax < D; ++ax) lx1[ax] = a.lam_x[ax * a.count + id];
        for (int k = 0; k < 3; ++k) lw1[k] = a.lam_w[k * a.count + id];
        double ld1[3] = {0.0, 0.0, 0.0}, ld0[3] = {0.0, 0.0, 0.0};
        for (int ax = 0; ax < D; ++ax) ld1[ax] = lx1[ax] + gd[D + ax];
        const double inv3 = inv * inv * inv;
        double lw[3];
        for (int k = 0; k < 3; ++k) {
            lw[k] = lw1[k] + (D == 2 ? gd[2 * D + k] : 0.0);
            for (int ax = 0; ax < D; ++ax)
                lw[k] += ld1[ax] * g.cfl[ax] * ((ax == k ? inv : 0.0) - w1[ax] * w1[k] * inv3);
        }
        for (int ax = 0; ax < D; ++ax) ld0[ax] = gd[ax] + ld1[ax];
        double l9[9];
        for (int j = 0; j < 9; ++j) {
            l9[j] = 0.0;
            for (int k = 0; k < 3; ++k) l9[j] += lw[k] * wv[k].d[j];
        }
        for (int ax = 0; ax < D; ++ax)
            for (int k = 0; k < 3; ++k) ld0[ax] += l9[3 + k] * Eg[k].d[ax] + l9[6 + k] * Bg[k].d[ax];

        // fields: alpha lambda_Ep into lambda_E, beta lambda_Bp into lambda_B
        Axis<double> wv0[3];
        for (int ax = 0; ax < 3; ++ax) {
            for (int k = 0; k < 2; ++k) wv0[ax].f[k] = ax0[ax].f[k].v;
            for (int k = 0; k < 3; ++k) wv0[ax].s[k] = ax0[ax].s[k].v;
        }
        scatter_comp<D, true, false, false>(a.lamE, wv0, xi, yj, zk, l9[3]);
        scatter_comp<D, false, true, false>(a.lamE + N, wv0, xi, yj, zk, l9[4]);
        scatter_comp<D, false, false, true>(a.lamE + 2 * N, wv0, xi, yj, zk, l9[5]);
        scatter_comp<D, false, true, true>(a.lamB, wv0, xi, yj, zk, l9[6]);
        scatter_comp<D, true, false, true>(a.lamB + N, wv0, xi, yj, zk, l9[7]);
        scatter_comp<D, true, true, false>(a.lamB + 2 * N, wv0, xi, yj, zk, l9[8]);
        for (int k = 0; k < 3; ++k) lbp[k] = l9[6 + k];

        for (int ax = 0; ax < 3; ++ax) a.lam_x[ax * a.count + id] = ax < D ? ld0[ax] : 0.0;
        for (int k = 0; k < 3; ++k) a.lam_w[k * a.count + id] = l9[k];
    }
    for (int k = 0; k < 3; ++k)
        if (lbp[k] != 0.0) atomicAdd(&sb[k], lbp[k]);
    __syncthreads();
    if (threadIdx.x < 3) grid_add(&a.lam_bext[threadIdx.x], sb[threadIdx.x]);
}

unsigned cells_blocks(int64_t n) { return (unsigned)((n + kCurlThreads - 1) / kCurlThreads); }

}  // namespace

hipError_t launch_adjoint_seed(const Ctx& c, double* lam, hipStream_t s)
{
    const unsigned b = cells_blocks(c.k.ncell);
    hipLaunchKernelGGL(k_adj_seed_b, dim3(b), dim3(kCurlThreads), 0, s, c.k, c.fields, lam, c.adj);
    hipLaunchKernelGGL(k_adj_seed_e, dim3(b), dim3(kCurlThreads), 0, s, c.k, c.fields, lam, c.adj);
    return hipGetLastError();
}

hipError_t launch_adjoint_step(const Ctx& c, double* lam, double* const* lam_x, double* const* lam_w,
                               double* lam_bext, hipStream_t s)
{
    const int64_t N = c.k.ncell;
    const unsigned b = cells_blocks(N);
    hipLaunchKernelGGL(k_adj_bn, dim3(b), dim3(kCurlThreads), 0, s, c.k, c.fields, c.bn);
    hipLaunchKernelGGL(k_adj_pre, dim3(b), dim3(kCurlThreads), 0, s, c.k, lam, lam + 3 * N, c.adj);
    hipLaunchKernelGGL(k_adj_curl, dim3(b), dim3(kCurlThreads), 0, s, c.k, lam, lam + 3 * N);
    for (int i = 0; i < c.nsp; ++i) {
        const Species& sp = c.sp[i];
        if (!sp.d.mobile || sp.n == 0) continue;
        AdjArgs a{};
        for (int ax = 0; ax < 3; ++ax) {
            a.pos[ax] = (const double*)sp.cur.pos[ax];
            a.mom[ax] = (const double*)sp.cur.mom[ax];
        }
        a.weight = (const double*)sp.cur.weight;
        a.id = sp.cur.id;
        a.n = sp.n;
        a.count = sp.n;
        a.q = sp.d.q;
        a.qm = sp.d.q / sp.d.m;
        a.E = c.fields;
        a.Bn = c.bn;
        a.lamJ = c.adj;
        a.lamE = lam;
        a.lamB = lam + 3 * N;
        a.lam_x = lam_x[i];
        a.lam_w = lam_w[i];
        a.lam_bext = lam_bext;
        const unsigned pb = (unsigned)((sp.n + kAdjThreads - 1) / kAdjThreads);
        if (c.k.dims == 3)
            hipLaunchKernelGGL(k_adj_particles<3>, dim3(pb), dim3(kAdjThreads), 0, s, c.k, a);
        else
            hipLaunchKernelGGL(k_adj_particles<2>, dim3(pb), dim3(kAdjThreads), 0, s, c.k, a);
    }
    hipLaunchKernelGGL(k_adj_curl, dim3(b), dim3(kCurlThreads), 0, s, c.k, lam, lam + 3 * N);
    return hipGetLastError();
}

}  // namespace pic
