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
// and per particle the reverse of its gather, push, move and deposit: the
// forward values are recomputed by the step's own formulas (pic_math.h); the
// current and the push are reversed by hand (contractions of lambda_J with the
// window sums and differences; cross-product identities), and the gather's
// derivative in the start offsets comes from forward-mode dual numbers (2D,
// and the generic kernel) or from separable partial sums over the stencil in
// a second pass that also does the scatter (3D tile kernel).  The
// particle part adds alpha lambda_Ep into lambda_E and beta lambda_Bp into
// lambda_B (in LDS per tile, or with atomics) and sums lambda_Bp into the
// external-field gradient.
//
// Kernels: k_adj_seed_b/e (loss seed), k_adj_pre (B^n, lambda_J, lambda_B),
// k_adj_curl (lambda_E), k_adj_tile2 / k_adj_tile3 (particles by tile),
// k_adj_particles (particles of an unsorted context), k_copy_segments
// (records), k_inverse / k_permute (particle adjoints between orders).
#include <algorithm>

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

// First kernel of a reverse step, per cell: B^n of the state (E^n,
// B^{n-1/2}) into bn (same expression as the step's first half step; the
// state is untouched); lambda_J = -4 pi dt lambda_E'; lambda_B <- lambda_B' +
// C lambda_E' (the transpose of D is C: both are the curl, with backward and
// forward differences).
__global__ __launch_bounds__(kCurlThreads) void k_adj_pre(GridK g, const double* __restrict__ f,
                                                          double* __restrict__ bn, const double* __restrict__ lamE,
                                                          double* __restrict__ lamB, double* __restrict__ lamJ)
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
    double* lam_x;       // 3 x count, by particle id (by_id) or storage position
    double* lam_w;       // 3 x count, likewise
    double* lam_bext;    // 3, accumulated
    double* scr[6];      // per storage position, n each: lambda_Ep, lambda_Bp (3D tile kernel)
    int64_t* qslot;      // per storage position: 16 x class rank + class, or -1 (3D tile kernel)
    int by_id;
};

// Reverse of the momentum advance (Appendix, Eq. p2): recompute the forward
// intermediates, then carry lw1 = dL/dw^{n+1/2} back to dL/dw^{n-1/2} (lw0),
// dL/dE_p (lE) and dL/dB_p (lB).  For f = m . (u x v): df/du = v x m and
// df/dv = m x u.
__device__ __forceinline__ void cross(const double u[3], const double v[3], double r[3])
{
    r[0] = u[1] * v[2] - u[2] * v[1];
    r[1] = u[2] * v[0] - u[0] * v[2];
    r[2] = u[0] * v[1] - u[1] * v[0];
}

__device__ __forceinline__ void push_reverse(double qmdt2, double c2, const double E[3], const double B[3],
                                             const double w[3], const double lw1[3], double lw0[3],
                                             double lE[3], double lB[3])
{
    double e[3], wt[3], b[3], wp[3], cr[3];
    for (int a = 0; a < 3; ++a) e[a] = qmdt2 * E[a];
    for (int a = 0; a < 3; ++a) wt[a] = w[a] + e[a];
    const double g = ::sqrt(wt[0] * wt[0] + wt[1] * wt[1] + wt[2] * wt[2] + c2);
    const double k = qmdt2 / g;
    for (int a = 0; a < 3; ++a) b[a] = k * B[a];
    cross(wt, b, cr);
    for (int a = 0; a < 3; ++a) wp[a] = wt[a] + cr[a];
    const double s = 2.0 / (1.0 + b[0] * b[0] + b[1] * b[1] + b[2] * b[2]);
    // w1 = wt + e + s (wp x b)
    cross(wp, b, cr);
    const double ls = lw1[0] * cr[0] + lw1[1] * cr[1] + lw1[2] * cr[2];
    double m[3], lwp[3], lb[3], lwt[3], t[3];
    for (int a = 0; a < 3; ++a) m[a] = s * lw1[a];
    cross(b, m, lwp);
    cross(m, wp, lb);
    for (int a = 0; a < 3; ++a) lb[a] -= s * s * ls * b[a];  // ds/db = -s^2 b
    // wp = wt + wt x b
    cross(b, lwp, t);
    for (int a = 0; a < 3; ++a) lwt[a] = lw1[a] + lwp[a] + t[a];
    cross(lwp, wt, t);
    for (int a = 0; a < 3; ++a) lb[a] += t[a];
    // b = (qmdt2 / g) B, g = sqrt(wt^2 + c^2)
    const double lk = lb[0] * B[0] + lb[1] * B[1] + lb[2] * B[2];
    const double lg = -lk * k / g;
    for (int a = 0; a < 3; ++a) {
        lB[a] = k * lb[a];
        lwt[a] += lg * wt[a] / g;
        lw0[a] = lwt[a];
        lE[a] = qmdt2 * (lw1[a] + lwt[a]);  // e enters w1 directly and through wt
    }
}

// 2D reverse of the quarter-form current (Eq. current as in deposit2):
// L(comp, ix, iy, 0) returns lambda_J at a window position; the derivatives
// of sum lambda_J J with respect to the window differences dm and sums dp are
// added into ldm, ldp, and with respect to the J^z factor into ljz.
template <int D, class LJ>
__device__ __forceinline__ void deposit_reverse(const double (&dm)[3][4], const double (&dp)[3][4],
                                                const double jfac[3], double jz, LJ L,
                                                double (&ldm)[3][4], double (&ldp)[3][4], double& ljz)
{
    static_assert(D == 2, "the 3D reverse current is deposit_reverse3");
    const double third = 1.0 / 3.0;
    for (int comp = 0; comp < 2; ++comp) {
        const int u = 1 - comp;
        const double K = 2.0 * jfac[comp];
        const double P[3] = {dm[comp][0], dm[comp][0] + dm[comp][1], -dm[comp][3]};
        double lP[3] = {0.0, 0.0, 0.0};
        for (int b = 0; b < 4; ++b) {
            double lb = 0.0;
            for (int t = 0; t < 3; ++t) {
                int ij[2];
                ij[comp] = t + 1;
                ij[u] = b;
                const double l = L(comp, ij[0], ij[1], 0);
                lP[t] += l * dp[u][b];
                lb += l * P[t];
            }
            ldp[u][b] += K * lb;
        }
        ldm[comp][0] += K * (lP[0] + lP[1]);
        ldm[comp][1] += K * lP[1];
        ldm[comp][3] -= K * lP[2];
    }
    for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b) {
            const double l = L(2, a, b, 0);
            ljz += l * (dp[0][a] * dp[1][b] + third * dm[0][a] * dm[1][b]);
            const double lj = jz * l;
            ldp[0][a] += lj * dp[1][b];
            ldp[1][b] += lj * dp[0][a];
            ldm[0][a] += third * lj * dm[1][b];
            ldm[1][b] += third * lj * dm[0][a];
        }
}

// 3D reverse of the quarter-form current (Eq. current as in deposit3).  J of
// component comp at window position (t+1 along comp, b, c across) is jfac P_t
// (dp_u[b] dp_v[c] + dm_u[b] dm_v[c] / 3); L(comp, ix, iy, iz) returns lambda_J
// there.  The derivatives of sum lambda_J J with respect to the window sums
// are added into ldp, and three times those with respect to the differences
// into ldm3: with jfac folded into P and the transverse product taken three
// times over, the inner loop has no 1/3 and no jfac product.
template <class LJ>
__device__ __forceinline__ void deposit_reverse3(const double (&dm)[3][4], const double (&dp)[3][4],
                                                 const double jfac[3], LJ L, double (&ldm3)[3][4],
                                                 double (&ldp)[3][4])
{
#pragma unroll
    for (int comp = 0; comp < 3; ++comp) {
        const int u = (comp + 1) % 3, v = (comp + 2) % 3;
        const double P[3] = {jfac[comp] * dm[comp][0], jfac[comp] * (dm[comp][0] + dm[comp][1]),
                             -jfac[comp] * dm[comp][3]};
        double lP3[3] = {0.0, 0.0, 0.0};  // sum over b, c of lambda_J times 3 x the transverse product
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const double dp3 = 3.0 * dp[u][b];
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const double tr3 = dp3 * dp[v][c] + dm[u][b] * dm[v][c];
                double ltr = 0.0;
#pragma unroll
                for (int t = 0; t < 3; ++t) {
                    int ijk[3];
                    ijk[comp] = t + 1;
                    ijk[u] = b;
                    ijk[v] = c;
                    const double l = L(comp, ijk[0], ijk[1], ijk[2]);
                    lP3[t] += l * tr3;
                    ltr += l * P[t];
                }
                ldp[u][b] += ltr * dp[v][c];
                ldp[v][c] += ltr * dp[u][b];
                ldm3[u][b] += ltr * dm[v][c];
                ldm3[v][c] += ltr * dm[u][b];
                // three lambda_J reads in flight per window column: the
                // reverse step runs two waves per SIMD in 256 registers
                __builtin_amdgcn_sched_barrier(0);
            }
        }
        ldm3[comp][0] += jfac[comp] * (lP3[0] + lP3[1]);
        ldm3[comp][1] += jfac[comp] * lP3[1];
        ldm3[comp][3] -= jfac[comp] * lP3[2];
        __builtin_amdgcn_sched_barrier(0);
    }
}

// d/dd of the cell weights (1/2 (1-d)^2, 3/4 - (1/2-d)^2, 1/2 d^2), contracted
// with their adjoints.
__device__ __forceinline__ double cell_weights_reverse(double d, const double ls[3])
{
    return ls[0] * (d - 1.0) + ls[1] * (1.0 - 2.0 * d) + ls[2] * d;
}

// Where a particle's reverse step reads and writes grid values.  Field
// component comp (0..2 = E, 3..5 = B^n) at offset (da, db, dc) in {-1, 0, 1}
// from the particle cell (F reads, add accumulates the adjoint); lambda_J at
// window position (ix, iy, iz) in 0..3 from the window start (L).
template <int D>
struct GlobalAcc {
    const GridK& g;
    const AdjArgs& a;
    // byte offsets within one plane (a plane is below 4 GiB): the plane base
    // is uniform once the component is known at compile time, so each load
    // takes a scalar base and one 32-bit offset register
    uint32_t xi[3], yj[3], zk[3], cx[4], cy[4], cz[4];
    __device__ GlobalAcc(const GridK& g_, const AdjArgs& a_) : g(g_), a(a_) {}
    __device__ void at(const int i0[3])
    {
        const uint32_t rx = 8u * (uint32_t)g.n[0], rxy = rx * (uint32_t)g.n[1];
        for (int o = 0; o < 3; ++o) {
            xi[o] = 8u * (uint32_t)wrapi(i0[0] + o - 1, g.n[0]);
            yj[o] = (uint32_t)wrapi(i0[1] + o - 1, g.n[1]) * rx;
            zk[o] = D == 3 ? (uint32_t)wrapi(i0[2] + o - 1, g.n[2]) * rxy : 0u;
        }
    }
    __device__ void window(const int i0[3], const int delta[3])
    {
        const int sx = i0[0] + (delta[0] < 0 ? -1 : 0) - 1;
        const int sy = i0[1] + (delta[1] < 0 ? -1 : 0) - 1;
        const int sz = i0[2] + (delta[2] < 0 ? -1 : 0) - 1;
        const uint32_t rx = 8u * (uint32_t)g.n[0], rxy = rx * (uint32_t)g.n[1];
        for (int o = 0; o < 4; ++o) {
            cx[o] = 8u * (uint32_t)wrapi(sx + o, g.n[0]);
            cy[o] = (uint32_t)wrapi(sy + o, g.n[1]) * rx;
            cz[o] = D == 3 ? (uint32_t)wrapi(sz + o, g.n[2]) * rxy : 0u;
        }
    }
    static __device__ __forceinline__ const double& at_byte(const double* plane, uint32_t off)
    {
        return *reinterpret_cast<const double*>(reinterpret_cast<const char*>(plane) + off);
    }
    __device__ const double* fplane(int comp) const
    {
        return comp < 3 ? a.E + comp * g.ncell : a.Bn + (comp - 3) * g.ncell;
    }
    __device__ double F(int comp, int da, int db, int dc) const
    {
        return at_byte(fplane(comp), zk[dc + 1] + yj[db + 1] + xi[da + 1]);
    }
    __device__ double L(int comp, int ix, int iy, int iz) const
    {
        return at_byte(a.lamJ + comp * g.ncell, cz[iz] + cy[iy] + cx[ix]);
    }
    __device__ void add(int comp, int da, int db, int dc, double v) const
    {
        double* plane = comp < 3 ? a.lamE + comp * g.ncell : a.lamB + (comp - 3) * g.ncell;
        grid_add(const_cast<double*>(&at_byte(plane, zk[dc + 1] + yj[db + 1] + xi[da + 1])), v);
    }
};

// Add w * lam at the stencil points of field component comp (Eqs. alphax,
// betax: per axis the node weights f at offsets 0, 1 or the cell weights s
// at -1, 0, 1; in 2D the z axis is the single plane).
template <int D, int comp, class Acc>
__device__ __forceinline__ void scatter_comp(Acc& acc, const Axis<double> (&w)[3], double lam)
{
    // node axes of each component: E^x x, E^y y, E^z z, B^x y z, B^y x z, B^z x y
    constexpr bool NX = comp == 0 || comp == 4 || comp == 5;
    constexpr bool NY = comp == 1 || comp == 3 || comp == 5;
    constexpr bool NZ = comp == 2 || comp == 3 || comp == 4;
    constexpr int ZLO = D == 3 ? (NZ ? 0 : -1) : 0, ZHI = D == 3 ? 1 : 0;
    for (int c = ZLO; c <= ZHI; ++c) {
        const double wz = D == 3 ? (NZ ? w[2].f[c] : w[2].s[c + 1]) : 1.0;
        for (int b = NY ? 0 : -1; b <= 1; ++b) {
            const double wy = NY ? w[1].f[b] : w[1].s[b + 1];
            for (int a = NX ? 0 : -1; a <= 1; ++a) {
                const double wx = NX ? w[0].f[a] : w[0].s[a + 1];
                acc.add(comp, a, b, c, wx * wy * wz * lam);
            }
        }
    }
}

// The 2D particle's part of the reverse step: recompute its gather, push and
// move, take lambda_J over its current window back to its start and end
// offsets and new momentum, then through the push to its old momentum and the
// fields it gathered; add those into lambda_E, lambda_B (acc) and lbp.  The
// gather's derivatives in the start offsets come from dual numbers.
template <int D, class Acc>
__device__ __forceinline__ void adj_particle(const GridK& g, const AdjArgs& a, Acc& acc, const int i0[3],
                                             const double d0[3], const double w0[3], double qp, int64_t li,
                                             double lbp[3])
{
    static_assert(D == 2, "the 3D particle's reverse step is adj_particle3");
    const double c = g.c, c2 = c * c;
    acc.at(i0);
    // gather, with the derivatives in the start offsets d0
    using DG = Dual<D>;
    Axis<DG> ax0[3];
    for (int ax = 0; ax < D; ++ax) ax0[ax] = form_factor<DG>(DG::var(d0[ax], ax));
    if (D == 2) ax0[2] = form_factor<DG>(DG(0.0));
    auto F = [&](int comp, int da, int db, int dc) -> double { return acc.F(comp, da, db, dc); };
    DG Eg[3], Bg[3];
    gather2<DG>(ax0, F, Eg, Bg);
    double Ep[3], Bp[3];
    for (int k = 0; k < 3; ++k) {
        Ep[k] = Eg[k].v;
        Bp[k] = Bg[k].v + g.bext[k];
    }

    // forward push and position advance, values only
    const double qmdt2 = 0.5 * a.qm * g.dt;
    double w1[3] = {w0[0], w0[1], w0[2]};
    push<double>(qmdt2, c2, Ep, Bp, w1);
    const double inv = 1.0 / ::sqrt(w1[0] * w1[0] + w1[1] * w1[1] + w1[2] * w1[2] + c2);
    double disp[3];
    for (int ax = 0; ax < 3; ++ax) disp[ax] = w1[ax] * inv * g.cfl[ax];
    double d1[3] = {0.0, 0.0, 0.0};
    int delta[3] = {0, 0, 0};
    StepArgs none{};
    PosIO<double, D>::move(none, 0, g, i0, d0, disp, d1, delta, false);

    // reverse of the current: lambda_J over the particle's window
    double dm[3][4], dp[3][4], ldm[3][4], ldp[3][4];
    for (int ax = 0; ax < 3; ++ax)
        for (int t = 0; t < 4; ++t) {
            dm[ax][t] = dp[ax][t] = 0.0;
            ldm[ax][t] = ldp[ax][t] = 0.0;
        }
#pragma unroll
    for (int ax = 0; ax < D; ++ax) {
        double s0[3], s1[3];
        cell_weights<double>(d0[ax], s0);
        cell_weights<double>(d1[ax], s1);
        window<double>(s0, s1, delta[ax], dm[ax], dp[ax]);
    }
    double jfac[3];
    for (int k = 0; k < 3; ++k) jfac[k] = g.jscale[k] * qp;
    const double jzc = qp * 0.25 * g.inv_vol * c;  // J^z factor per unit u_z = w_z / gamma
    const double jz = D == 2 ? jzc * w1[2] * inv : 0.0;
    acc.window(i0, delta);
    double ljz = 0.0;
    auto L = [&](int comp, int ix, int iy, int iz) -> double { return acc.L(comp, ix, iy, iz); };
    deposit_reverse<D>(dm, dp, jfac, jz, L, ldm, ldp, ljz);

    // back through the window to the start and end offsets
    double gd0[3] = {0.0, 0.0, 0.0}, gd1[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int ax = 0; ax < D; ++ax) {
        // start weights sit one window cell right when delta < 0, end weights
        // when delta > 0 (two-way selects, no indexed access)
        const bool o0 = delta[ax] < 0, o1 = delta[ax] > 0;
        double ls0[3], ls1[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            ls0[k] = o0 ? ldp[ax][k + 1] - ldm[ax][k + 1] : ldp[ax][k] - ldm[ax][k];
            ls1[k] = o1 ? ldp[ax][k + 1] + ldm[ax][k + 1] : ldp[ax][k] + ldm[ax][k];
        }
        gd0[ax] = cell_weights_reverse(d0[ax], ls0);
        gd1[ax] = cell_weights_reverse(d1[ax], ls1);
    }

    // x^{n+1} = x^n + V(w^{n+1/2}): d1 = d0 + disp - delta
    double ld1[3] = {0.0, 0.0, 0.0}, ld0[3] = {0.0, 0.0, 0.0};
    for (int ax = 0; ax < D; ++ax) {
        ld1[ax] = a.lam_x[ax * a.count + li] + gd1[ax];
        ld0[ax] = gd0[ax] + ld1[ax];
    }
    const double inv3 = inv * inv * inv;
    double lw1[3];
    for (int k = 0; k < 3; ++k) {
        lw1[k] = a.lam_w[k * a.count + li];
        if (D == 2) lw1[k] += ljz * jzc * ((k == 2 ? inv : 0.0) - w1[2] * w1[k] * inv3);
        for (int ax = 0; ax < D; ++ax)
            lw1[k] += ld1[ax] * g.cfl[ax] * ((ax == k ? inv : 0.0) - w1[ax] * w1[k] * inv3);
    }

    // push
    double lw0[3], lE[3], lB[3];
    push_reverse(qmdt2, c2, Ep, Bp, w0, lw1, lw0, lE, lB);

    // gather: offsets, and alpha lambda_Ep into lambda_E, beta lambda_Bp
    // into lambda_B
    for (int ax = 0; ax < D; ++ax)
        for (int k = 0; k < 3; ++k) ld0[ax] += lE[k] * Eg[k].d[ax] + lB[k] * Bg[k].d[ax];
    Axis<double> wv0[3];
    for (int ax = 0; ax < 3; ++ax) {
        for (int k = 0; k < 2; ++k) wv0[ax].f[k] = ax0[ax].f[k].v;
        for (int k = 0; k < 3; ++k) wv0[ax].s[k] = ax0[ax].s[k].v;
    }
    scatter_comp<D, 0>(acc, wv0, lE[0]);
    scatter_comp<D, 1>(acc, wv0, lE[1]);
    scatter_comp<D, 2>(acc, wv0, lE[2]);
    scatter_comp<D, 3>(acc, wv0, lB[0]);
    scatter_comp<D, 4>(acc, wv0, lB[1]);
    scatter_comp<D, 5>(acc, wv0, lB[2]);
    for (int k = 0; k < 3; ++k) lbp[k] += lB[k];

    for (int ax = 0; ax < 3; ++ax) a.lam_x[ax * a.count + li] = ax < D ? ld0[ax] : 0.0;
    for (int k = 0; k < 3; ++k) a.lam_w[k * a.count + li] = lw0[k];
}

// Derivative in d of the form factor of one axis (Eqs. alphax, betax):
// node factors 1 - d, d; cell factors (1 - d)^2 / 2, 3/4 - (1/2 - d)^2, d^2 / 2.
__device__ __forceinline__ Axis<double> form_factor_d(double d)
{
    Axis<double> a;
    a.f[0] = -1.0;
    a.f[1] = 1.0;
    a.s[0] = d - 1.0;
    a.s[1] = 1.0 - 2.0 * d;
    a.s[2] = d;
    return a;
}

// Reverse of one gathered component, lam being the adjoint of its value at
// the particle: lam times the form factor goes into the component's adjoint
// at each stencil point (acc.add, when SCATTER), and lam times the derivatives of the
// gathered value in the three offsets into ld0.  The derivatives are
// separable partial sums over the stencil (innermost z, then y, then x) with
// one axis's factor replaced by its derivative.
template <int comp, bool SCATTER, class Acc>
__device__ __forceinline__ void gather_comp_reverse(Acc& acc, const Axis<double> (&w)[3], const Axis<double> (&dw)[3],
                                                    double lam, double (&ld0)[3])
{
    constexpr bool NX = comp == 0 || comp == 4 || comp == 5;
    constexpr bool NY = comp == 1 || comp == 3 || comp == 5;
    constexpr bool NZ = comp == 2 || comp == 3 || comp == 4;
    double tx = 0.0, ty = 0.0, tz = 0.0;
#pragma unroll
    for (int a = NX ? 0 : -1; a <= 1; ++a) {
        const double wx = NX ? w[0].f[a] : w[0].s[a + 1];
        double sa = 0.0, say = 0.0, saz = 0.0;
#pragma unroll
        for (int b = NY ? 0 : -1; b <= 1; ++b) {
            const double wy = NY ? w[1].f[b] : w[1].s[b + 1];
            const double lxy = SCATTER ? lam * wx * wy : 0.0;
            double sb = 0.0, sbz = 0.0;
#pragma unroll
            for (int c = NZ ? 0 : -1; c <= 1; ++c) {
                const double wz = NZ ? w[2].f[c] : w[2].s[c + 1];
                const double f = acc.F(comp, a, b, c);
                sb += wz * f;
                sbz += (NZ ? dw[2].f[c] : dw[2].s[c + 1]) * f;
                if constexpr (SCATTER) acc.add(comp, a, b, c, lxy * wz);
            }
            sa += wy * sb;
            say += (NY ? dw[1].f[b] : dw[1].s[b + 1]) * sb;
            saz += wy * sbz;
        }
        tx += (NX ? dw[0].f[a] : dw[0].s[a + 1]) * sa;
        ty += wx * say;
        tz += wx * saz;
    }
    ld0[0] += lam * tx;
    ld0[1] += lam * ty;
    ld0[2] += lam * tz;
}

// The 3D particle's part of the reverse step, arranged to keep few values
// live: a gather of values only feeds the push and the move; the reverse
// current and the reverse push run on that state; a second pass over the
// stencil then adds the form factor times lambda_Ep, lambda_Bp into lambda_E,
// lambda_B and the gathered values' derivatives in the start offsets into
// lambda_x.  Without SCATTER the second pass only takes the derivatives and
// lambda_Ep, lambda_Bp are returned in lEB for a later scatter.  The
// derivatives of the gathered values are separable partial sums over the
// stencil (gather_comp_reverse), not dual numbers.
template <bool SCATTER, class Acc>
__device__ __forceinline__ void adj_particle3(const GridK& g, const AdjArgs& a, Acc& acc, const int i0[3],
                                              const double d0[3], const double w0[3], double qp, int64_t li,
                                              double lbp[3], double lEB[6])
{
    const double c = g.c, c2 = c * c;
    acc.at(i0);
    double Ep[3], Bp[3];
    {
        Axis<double> w[3];
        for (int ax = 0; ax < 3; ++ax) w[ax] = form_factor<double>(d0[ax]);
        auto F = [&](int comp, int da, int db, int dc) -> double { return acc.F(comp, da, db, dc); };
        gather3<double>(w, F, Ep, Bp);
    }
    for (int k = 0; k < 3; ++k) Bp[k] += g.bext[k];

    // forward push and position advance, values only
    const double qmdt2 = 0.5 * a.qm * g.dt;
    double w1[3] = {w0[0], w0[1], w0[2]};
    push<double>(qmdt2, c2, Ep, Bp, w1);
    const double inv = 1.0 / ::sqrt(w1[0] * w1[0] + w1[1] * w1[1] + w1[2] * w1[2] + c2);
    double disp[3];
    for (int ax = 0; ax < 3; ++ax) disp[ax] = w1[ax] * inv * g.cfl[ax];
    double d1[3] = {0.0, 0.0, 0.0};
    int delta[3] = {0, 0, 0};
    StepArgs none{};
    PosIO<double, 3>::move(none, 0, g, i0, d0, disp, d1, delta, false);
    __builtin_amdgcn_sched_barrier(0);

    // reverse of the current over the particle's window
    double ld0[3], ld1[3];
    {
        double dm[3][4], dp[3][4], ldm[3][4], ldp[3][4];
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
            double s0[3], s1[3];
            cell_weights<double>(d0[ax], s0);
            cell_weights<double>(d1[ax], s1);
            window<double>(s0, s1, delta[ax], dm[ax], dp[ax]);
            for (int t = 0; t < 4; ++t) ldm[ax][t] = ldp[ax][t] = 0.0;
        }
        double jfac[3];
        for (int k = 0; k < 3; ++k) jfac[k] = g.jscale[k] * qp;
        const double third = 1.0 / 3.0;
        acc.window(i0, delta);
        auto L = [&](int comp, int ix, int iy, int iz) -> double { return acc.L(comp, ix, iy, iz); };
        deposit_reverse3(dm, dp, jfac, L, ldm, ldp);  // ldm holds 3 x the difference adjoints
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
            // start weights sit one window cell right when delta < 0, end
            // weights when delta > 0 (two-way selects, no indexed access)
            const bool o0 = delta[ax] < 0, o1 = delta[ax] > 0;
            double ls0[3], ls1[3];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                ls0[k] = o0 ? ldp[ax][k + 1] - third * ldm[ax][k + 1] : ldp[ax][k] - third * ldm[ax][k];
                ls1[k] = o1 ? ldp[ax][k + 1] + third * ldm[ax][k + 1] : ldp[ax][k] + third * ldm[ax][k];
            }
            // x^{n+1} = x^n + V(w^{n+1/2}): d1 = d0 + disp - delta
            ld1[ax] = a.lam_x[ax * a.count + li] + cell_weights_reverse(d1[ax], ls1);
            ld0[ax] = cell_weights_reverse(d0[ax], ls0) + ld1[ax];
        }
    }
    const double inv3 = inv * inv * inv;
    double lw1[3];
    for (int k = 0; k < 3; ++k) {
        lw1[k] = a.lam_w[k * a.count + li];
        for (int ax = 0; ax < 3; ++ax)
            lw1[k] += ld1[ax] * g.cfl[ax] * ((ax == k ? inv : 0.0) - w1[ax] * w1[k] * inv3);
    }

    // push
    double lw0[3], lE[3], lB[3];
    push_reverse(qmdt2, c2, Ep, Bp, w0, lw1, lw0, lE, lB);
    for (int k = 0; k < 3; ++k) lbp[k] += lB[k];
    __builtin_amdgcn_sched_barrier(0);

    // gather, reversed
    Axis<double> w[3], dw[3];
    for (int ax = 0; ax < 3; ++ax) {
        w[ax] = form_factor<double>(d0[ax]);
        dw[ax] = form_factor_d(d0[ax]);
    }
    gather_comp_reverse<0, SCATTER>(acc, w, dw, lE[0], ld0);
    __builtin_amdgcn_sched_barrier(0);
    gather_comp_reverse<1, SCATTER>(acc, w, dw, lE[1], ld0);
    __builtin_amdgcn_sched_barrier(0);
    gather_comp_reverse<2, SCATTER>(acc, w, dw, lE[2], ld0);
    __builtin_amdgcn_sched_barrier(0);
    gather_comp_reverse<3, SCATTER>(acc, w, dw, lB[0], ld0);
    __builtin_amdgcn_sched_barrier(0);
    gather_comp_reverse<4, SCATTER>(acc, w, dw, lB[1], ld0);
    __builtin_amdgcn_sched_barrier(0);
    gather_comp_reverse<5, SCATTER>(acc, w, dw, lB[2], ld0);
    for (int k = 0; k < 3; ++k) {
        lEB[k] = lE[k];
        lEB[3 + k] = lB[k];
    }

    for (int ax = 0; ax < 3; ++ax) a.lam_x[ax * a.count + li] = ld0[ax];
    for (int k = 0; k < 3; ++k) a.lam_w[k * a.count + li] = lw0[k];
}

template <int D>
__device__ __forceinline__ void load_particle(const AdjArgs& a, int64_t p, int i0[3], double d0[3],
                                              double w0[3], double& qp, int64_t& li)
{
    for (int ax = 0; ax < 3; ++ax) {
        i0[ax] = 0;
        d0[ax] = 0.0;
    }
    for (int ax = 0; ax < D; ++ax) {
        const double x = a.pos[ax][p];
        const double fl = floor(x);
        i0[ax] = (int)fl;
        d0[ax] = x - fl;
    }
    li = a.by_id ? a.id[p] : p;  // where the particle's adjoint is kept
    for (int k = 0; k < 3; ++k) w0[k] = a.mom[k][p];
    qp = a.q * a.weight[p];
}

// Sum lbp over the block into lam_bext.
__device__ __forceinline__ void flush_bext(double* sb, const double lbp[3], double* lam_bext)
{
    for (int k = 0; k < 3; ++k)
        if (lbp[k] != 0.0) atomicAdd(&sb[k], lbp[k]);
    __syncthreads();
    if (threadIdx.x < 3) grid_add(&lam_bext[threadIdx.x], sb[threadIdx.x]);
}

// One thread per particle, every grid access in global memory (any order of
// the particles; 3D, and 2D before the first sort).
template <int D>
__global__ __launch_bounds__(kAdjThreads) void k_adj_particles(GridK g, AdjArgs a)
{
    __shared__ double sb[3];
    if (threadIdx.x < 3) sb[threadIdx.x] = 0.0;
    __syncthreads();
    const int64_t p = (int64_t)blockIdx.x * kAdjThreads + threadIdx.x;
    double lbp[3] = {0.0, 0.0, 0.0};
    if (p < a.n) {
        int i0[3];
        double d0[3], w0[3], qp;
        int64_t li;
        load_particle<D>(a, p, i0, d0, w0, qp, li);
        GlobalAcc<D> acc(g, a);
        double lEB[6];
        if constexpr (D == 3) adj_particle3<true>(g, a, acc, i0, d0, w0, qp, li, lbp, lEB);
        else adj_particle<D>(g, a, acc, i0, d0, w0, qp, li, lbp);
    }
    flush_bext(sb, lbp, a.lam_bext);
}

// 2D tile kernel.  The particles are grouped by the tiles of the last sort
// (tile_start); kAdjSplit blocks share a tile's particles.  Each block stages
// E, B^n (cells T0-1-M .. T0+T+M) and lambda_J (T0-2-M .. T0+T+1+M) of its
// tile in LDS and accumulates lambda_E, lambda_B over the field region in LDS,
// added to the grid once at the end; a particle more than M cells outside its
// tile (it moved since the sort) uses the global-memory accessor instead.
constexpr int kAdjT2 = kTile2;
constexpr int kAdjM2 = 3;
constexpr int kAdjLF2 = kAdjT2 + 2 + 2 * kAdjM2;
constexpr int kAdjLJ2 = kAdjT2 + 4 + 2 * kAdjM2;
constexpr int kAdjNF2 = kAdjLF2 * kAdjLF2;
constexpr int kAdjNJ2 = kAdjLJ2 * kAdjLJ2;

struct LdsAcc2 {
    const double* sf;  // 6 x kAdjNF2
    const double* sj;  // 3 x kAdjNJ2
    double* sacc;      // 6 x kAdjNF2
    int r0, r1;        // particle cell relative to the tile origin
    int fo, jo;        // particle cell in the field region, window start in the current region
    __device__ void at(const int*) { fo = (r1 + 1 + kAdjM2) * kAdjLF2 + r0 + 1 + kAdjM2; }
    __device__ void window(const int*, const int delta[3])
    {
        jo = (r1 + 1 + kAdjM2 + (delta[1] < 0 ? -1 : 0)) * kAdjLJ2 + r0 + 1 + kAdjM2 + (delta[0] < 0 ? -1 : 0);
    }
    __device__ double F(int comp, int da, int db, int) const
    {
        return sf[comp * kAdjNF2 + fo + db * kAdjLF2 + da];
    }
    __device__ double L(int comp, int ix, int iy, int) const
    {
        return sj[comp * kAdjNJ2 + jo + iy * kAdjLJ2 + ix];
    }
    __device__ void add(int comp, int da, int db, int, double v) const
    {
        atomicAdd(&sacc[comp * kAdjNF2 + fo + db * kAdjLF2 + da], v);
    }
};

__global__ __launch_bounds__(kAdjThreads) __attribute__((amdgpu_waves_per_eu(2))) void k_adj_tile2(GridK g, AdjArgs a, const int64_t* __restrict__ tile_start,
                                                        int split)
{
    constexpr int T = kAdjT2, M = kAdjM2, LF = kAdjLF2, LJ = kAdjLJ2, NF = kAdjNF2, NJ = kAdjNJ2;
    __shared__ double sf[6 * NF];
    __shared__ double sj[3 * NJ];
    __shared__ double sacc[6 * NF];
    __shared__ double sb[3];
    const int unit = xcd_tile(blockIdx.x, g.ntiles * split);
    const int tile = unit / split, part = unit - tile * split;
    const int T0[2] = {(tile % g.nt[0]) * T, (tile / g.nt[0]) * T};
    const int64_t N = g.ncell;
    const int nx = g.n[0], ny = g.n[1];
    for (int e = threadIdx.x; e < 6 * NF; e += kAdjThreads) {
        const int comp = e / NF, r = e - comp * NF;
        const int gx = wrapi(T0[0] - 1 - M + r % LF, nx), gy = wrapi(T0[1] - 1 - M + r / LF, ny);
        const int64_t cell = (int64_t)gy * nx + gx;
        sf[e] = comp < 3 ? a.E[comp * N + cell] : a.Bn[(comp - 3) * N + cell];
        sacc[e] = 0.0;
    }
    for (int e = threadIdx.x; e < 3 * NJ; e += kAdjThreads) {
        const int comp = e / NJ, r = e - comp * NJ;
        const int gx = wrapi(T0[0] - 2 - M + r % LJ, nx), gy = wrapi(T0[1] - 2 - M + r / LJ, ny);
        sj[e] = a.lamJ[comp * N + (int64_t)gy * nx + gx];
    }
    if (threadIdx.x < 3) sb[threadIdx.x] = 0.0;
    __syncthreads();

    double lbp[3] = {0.0, 0.0, 0.0};
    const int64_t begin = tile_start[tile], end = tile_start[tile + 1];
    for (int64_t p = begin + part * kAdjThreads + threadIdx.x; p < end; p += (int64_t)split * kAdjThreads) {
        int i0[3];
        double d0[3], w0[3], qp;
        int64_t li;
        load_particle<2>(a, p, i0, d0, w0, qp, li);
        int rel[2];
        bool inside = true;
        for (int ax = 0; ax < 2; ++ax) {
            int r = i0[ax] - T0[ax];
            const int n = g.n[ax];
            if (r > n / 2) r -= n;
            if (r < -(n / 2)) r += n;
            rel[ax] = r;
            inside = inside && r >= -M && r <= T - 1 + M;
        }
        if (inside) {
            LdsAcc2 acc;
            acc.sf = sf;
            acc.sj = sj;
            acc.sacc = sacc;
            acc.r0 = rel[0];
            acc.r1 = rel[1];
            adj_particle<2>(g, a, acc, i0, d0, w0, qp, li, lbp);
        } else {
            GlobalAcc<2> acc(g, a);
            adj_particle<2>(g, a, acc, i0, d0, w0, qp, li, lbp);
        }
    }
    __syncthreads();
    for (int e = threadIdx.x; e < 6 * NF; e += kAdjThreads) {
        const double v = sacc[e];
        if (v == 0.0) continue;
        const int comp = e / NF, r = e - comp * NF;
        const int gx = wrapi(T0[0] - 1 - M + r % LF, nx), gy = wrapi(T0[1] - 1 - M + r / LF, ny);
        const int64_t cell = (int64_t)gy * nx + gx;
        grid_add(comp < 3 ? &a.lamE[comp * N + cell] : &a.lamB[(comp - 3) * N + cell], v);
    }
    flush_bext(sb, lbp, a.lam_bext);
}

// 3D tile kernel, in two phases over the tile's particles that share one LDS
// area.  Phase 1 stages E, B^n over the field region (cells T0-1-M .. T0+T+M,
// 83 KB) and lambda_J over the particles' windows (T0-2-M .. T0+T+1+M, 66 KB)
// and runs each particle's reverse step from LDS, except the scatter:
// lambda_Ep, lambda_Bp go to a scratch row per particle.  Phase 2 reuses the
// area for lambda_E, lambda_B over the field region, scatters every
// particle's lambda_Ep, lambda_Bp into it with LDS atomics, and adds it to
// the grid once.  A particle more than M = 1 cell outside its tile runs
// entirely in phase 1 from global memory, with global atomics, after the
// others: it is queued in the class queue's array (idle until phase 2), so
// that a wave runs the LDS form or the global one, not both (inline when
// that array is full or the tile holds more than 65536).  The particle
// work fits 256 registers, so the 512 threads run as two waves per SIMD.
//
// Phase 2 hands particles to lanes by class, the residue of the particle's
// field-region cell modulo 16: phase 1 ranks each particle within its class
// (LDS counters; rank and class kept in the spare copy's id row), a short
// pass writes the 16-bit tile offsets into an LDS queue grouped by class,
// and phase 2 takes slot s = 16 r + c as the r-th particle of class c.  The
// 16 lanes of one LDS pass then hold 16 distinct classes, so the same
// stencil offset lands in 16 distinct banks and the atomics do not conflict.
// A block with more than kAdjQ3 particles in its tile, or a tile of more
// than 65536, scatters in storage order instead.
constexpr int kAdjT3 = kTile3;
constexpr int kAdjM3 = 1;
constexpr int kAdjLF3 = kAdjT3 + 2 + 2 * kAdjM3;
constexpr int kAdjLJ3 = kAdjT3 + 4 + 2 * kAdjM3;
constexpr int kAdjNF3 = kAdjLF3 * kAdjLF3 * kAdjLF3;
constexpr int kAdjNJ3 = kAdjLJ3 * kAdjLJ3 * kAdjLJ3;
constexpr int kAdjThreads3 = 512;
constexpr int kAdjC3 = 16;      // lane classes: 16 lanes of 8-byte values per LDS pass
constexpr int kAdjQ3 = 7168;    // class-queue entries (16-bit tile offsets)
static_assert((6 * kAdjNF3 + 3 * kAdjNJ3 + 3) * 8 + (2 * kAdjC3 + 1) * 4 + kAdjQ3 * 2 <= 160 * 1024,
              "3D reverse-step LDS over 160 KB");

// Phase-1 reads: fields and lambda_J in LDS (the particle within M of its tile).
struct TileRead3 {
    const double* sf;  // 6 x kAdjNF3
    const double* sj;  // 3 x kAdjNJ3
    int rel[3];        // particle cell relative to the tile origin
    int fo;            // particle cell in the field region
    int jo;            // window start in the lambda_J region
    __device__ TileRead3(const double* f, const double* j, const int r[3]) : sf(f), sj(j)
    {
        for (int ax = 0; ax < 3; ++ax) rel[ax] = r[ax];
        fo = (r[0] + 1 + kAdjM3) + (r[1] + 1 + kAdjM3) * kAdjLF3 + (r[2] + 1 + kAdjM3) * kAdjLF3 * kAdjLF3;
    }
    __device__ void at(const int[3]) {}
    __device__ double F(int comp, int da, int db, int dc) const
    {
        return sf[comp * kAdjNF3 + fo + da + db * kAdjLF3 + dc * kAdjLF3 * kAdjLF3];
    }
    __device__ void window(const int[3], const int delta[3])
    {
        int o[3];
        for (int ax = 0; ax < 3; ++ax) o[ax] = rel[ax] + 1 + kAdjM3 + (delta[ax] < 0 ? -1 : 0);
        jo = o[0] + o[1] * kAdjLJ3 + o[2] * kAdjLJ3 * kAdjLJ3;
    }
    __device__ double L(int comp, int ix, int iy, int iz) const
    {
        return sj[comp * kAdjNJ3 + jo + ix + iy * kAdjLJ3 + iz * kAdjLJ3 * kAdjLJ3];
    }
};

// Phase-2 adds: lambda_E, lambda_B accumulated in LDS.
struct TileAdd3 {
    double* sacc;  // 6 x kAdjNF3
    int fo;
    __device__ void add(int comp, int da, int db, int dc, double v) const
    {
        atomicAdd(&sacc[comp * kAdjNF3 + fo + da + db * kAdjLF3 + dc * kAdjLF3 * kAdjLF3], v);
    }
};

// Cell and offsets of particle p and its cell relative to the tile origin;
// true when within M cells of the tile (the LDS regions cover it).
__device__ __forceinline__ bool tile_place3(const GridK& g, const AdjArgs& a, int64_t p, const int T0[3], int i0[3],
                                            double d0[3], int rel[3])
{
    bool inside = true;
    for (int ax = 0; ax < 3; ++ax) {
        const double x = a.pos[ax][p];
        const double fl = floor(x);
        i0[ax] = (int)fl;
        d0[ax] = x - fl;
        int r = i0[ax] - T0[ax];
        const int n = g.n[ax];
        if (r > n / 2) r -= n;
        if (r < -(n / 2)) r += n;
        rel[ax] = r;
        inside = inside && r >= -kAdjM3 && r <= kAdjT3 - 1 + kAdjM3;
    }
    return inside;
}

__global__ __launch_bounds__(kAdjThreads3) void k_adj_tile3(GridK g, AdjArgs a, const int64_t* __restrict__ tile_start,
                                                            int split)
{
    constexpr int T = kAdjT3, M = kAdjM3, LF = kAdjLF3, LJ = kAdjLJ3, NF = kAdjNF3, NJ = kAdjNJ3, NT = kAdjThreads3;
    constexpr int C = kAdjC3;
    static_assert((C & (C - 1)) == 0 && NT % 64 == 0, "16-lane groups of one class set per wave");
    __shared__ double lds[6 * NF + 3 * NJ];
    __shared__ double sb[3];
    __shared__ unsigned int qn[C], qoff[C], nout;
    __shared__ unsigned short queue[kAdjQ3];  // phase 1: the particles off the tile; phase 2: the class queue
    double* const sf = lds;  // phase 1: E, B^n; phase 2: lambda_E, lambda_B
    double* const sj = lds + 6 * NF;
    const int unit = xcd_tile(blockIdx.x, g.ntiles * split);
    const int tile = unit / split, part = unit - tile * split;
    const int T0[3] = {(tile % g.nt[0]) * T, ((tile / g.nt[0]) % g.nt[1]) * T, (tile / (g.nt[0] * g.nt[1])) * T};
    const int64_t N = g.ncell;
    const int nx = g.n[0], ny = g.n[1], nz = g.n[2];
    for (int e = threadIdx.x; e < 6 * NF; e += NT) {
        const int comp = e / NF, r = e - comp * NF;
        const int gx = wrapi(T0[0] - 1 - M + r % LF, nx);
        const int gy = wrapi(T0[1] - 1 - M + (r / LF) % LF, ny);
        const int gz = wrapi(T0[2] - 1 - M + r / (LF * LF), nz);
        const int64_t cell = ((int64_t)gz * ny + gy) * nx + gx;
        sf[e] = comp < 3 ? a.E[comp * N + cell] : a.Bn[(comp - 3) * N + cell];
    }
    for (int e = threadIdx.x; e < 3 * NJ; e += NT) {
        const int comp = e / NJ, r = e - comp * NJ;
        const int gx = wrapi(T0[0] - 2 - M + r % LJ, nx);
        const int gy = wrapi(T0[1] - 2 - M + (r / LJ) % LJ, ny);
        const int gz = wrapi(T0[2] - 2 - M + r / (LJ * LJ), nz);
        sj[e] = a.lamJ[comp * N + ((int64_t)gz * ny + gy) * nx + gx];
    }
    if (threadIdx.x < 3) sb[threadIdx.x] = 0.0;
    if (threadIdx.x < C) qn[threadIdx.x] = 0u;
    if (threadIdx.x == 0) nout = 0u;
    __syncthreads();

    // phase 1
    double lbp[3] = {0.0, 0.0, 0.0};
    const int64_t begin = tile_start[tile], end = tile_start[tile + 1];
    for (int64_t p = begin + part * NT + threadIdx.x; p < end; p += (int64_t)split * NT) {
        int i0[3], rel[3];
        double d0[3], w0[3], qp, lEB[6];
        int64_t li;
        load_particle<3>(a, p, i0, d0, w0, qp, li);
        const bool inside = tile_place3(g, a, p, T0, i0, d0, rel);
        if (inside) {
            TileRead3 acc(sf, sj, rel);
            adj_particle3<false>(g, a, acc, i0, d0, w0, qp, li, lbp, lEB);
            for (int k = 0; k < 6; ++k) a.scr[k][p] = lEB[k];
            const int cls = acc.fo & (C - 1);
            a.qslot[p] = (int64_t)atomicAdd(&qn[cls], 1u) * C + cls;
        } else {
            // drifted more than one cell out of the tile: queued, so that a
            // wave runs the LDS form or the global one, not both
            const unsigned int slot = end - begin <= 65536 ? atomicAdd(&nout, 1u) : (unsigned int)kAdjQ3;
            if (slot < (unsigned int)kAdjQ3) {
                queue[slot] = (unsigned short)(p - begin);
            } else {
                GlobalAcc<3> acc(g, a);
                adj_particle3<true>(g, a, acc, i0, d0, w0, qp, li, lbp, lEB);
            }
            a.qslot[p] = -1;
        }
    }
    __syncthreads();
    const unsigned int nq = nout < (unsigned int)kAdjQ3 ? nout : (unsigned int)kAdjQ3;
    for (unsigned int q = threadIdx.x; q < nq; q += NT) {
        const int64_t p = begin + queue[q];
        int i0[3];
        double d0[3], w0[3], qp, lEB[6];
        int64_t li;
        load_particle<3>(a, p, i0, d0, w0, qp, li);
        GlobalAcc<3> acc(g, a);
        adj_particle3<true>(g, a, acc, i0, d0, w0, qp, li, lbp, lEB);
    }
    __syncthreads();

    // the class queue (or storage order when it does not fit)
    unsigned int rows = 0, total = 0;
    for (int k = 0; k < C; ++k) {
        rows = qn[k] > rows ? qn[k] : rows;
        total += qn[k];
    }
    const bool classed = total <= (unsigned)kAdjQ3 && end - begin <= 65536;
    if (threadIdx.x == 0) {
        unsigned int o = 0;
        for (int k = 0; k < C; ++k) {
            qoff[k] = o;
            o += qn[k];
        }
    }
    for (int e = threadIdx.x; e < 6 * NF; e += NT) sf[e] = 0.0;
    __syncthreads();
    if (classed)
        for (int64_t p = begin + part * NT + threadIdx.x; p < end; p += (int64_t)split * NT) {
            const int64_t q = a.qslot[p];
            if (q >= 0) queue[qoff[q & (C - 1)] + q / C] = (unsigned short)(p - begin);
        }
    __syncthreads();

    // phase 2
    int64_t nslot = (int64_t)rows * C;
    if (!classed) {
        // storage order: the strides of phase 1
        const int64_t rem = end - begin - (int64_t)part * NT, stride = (int64_t)split * NT;
        nslot = rem > 0 ? (rem + stride - 1) / stride * NT : 0;
    }
    for (int64_t sl = threadIdx.x; sl < nslot; sl += NT) {
        int64_t p;
        if (classed) {
            const int cls = (int)(sl & (C - 1));
            const unsigned int r = (unsigned int)(sl / C);
            if (r >= qn[cls]) continue;
            p = begin + queue[qoff[cls] + r];
        } else {
            p = begin + part * NT + (sl / NT) * split * NT + sl % NT;
            if (p >= end) continue;
        }
        int i0[3], rel[3];
        double d0[3];
        if (!tile_place3(g, a, p, T0, i0, d0, rel)) continue;
        Axis<double> w[3];
        for (int ax = 0; ax < 3; ++ax) w[ax] = form_factor<double>(d0[ax]);
        const TileAdd3 acc{sf, (rel[0] + 1 + M) + (rel[1] + 1 + M) * LF + (rel[2] + 1 + M) * LF * LF};
        scatter_comp<3, 0>(acc, w, a.scr[0][p]);
        scatter_comp<3, 1>(acc, w, a.scr[1][p]);
        scatter_comp<3, 2>(acc, w, a.scr[2][p]);
        scatter_comp<3, 3>(acc, w, a.scr[3][p]);
        scatter_comp<3, 4>(acc, w, a.scr[4][p]);
        scatter_comp<3, 5>(acc, w, a.scr[5][p]);
    }
    __syncthreads();
    for (int e = threadIdx.x; e < 6 * NF; e += NT) {
        const double v = sf[e];
        if (v == 0.0) continue;
        const int comp = e / NF, r = e - comp * NF;
        const int gx = wrapi(T0[0] - 1 - M + r % LF, nx);
        const int gy = wrapi(T0[1] - 1 - M + (r / LF) % LF, ny);
        const int gz = wrapi(T0[2] - 1 - M + r / (LF * LF), nz);
        const int64_t cell = ((int64_t)gz * ny + gy) * nx + gx;
        grid_add(comp < 3 ? &a.lamE[comp * N + cell] : &a.lamB[(comp - 3) * N + cell], v);
    }
    flush_bext(sb, lbp, a.lam_bext);
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

namespace {

// ---------------------------------------------------------------------------
// The state a reverse step reads: E^n, B^{n-1/2} (6 planes) and per species
// the particles in storage order with the tile table of their last sort
// (tiles false: no valid table).  Either the context itself or a record.
// ---------------------------------------------------------------------------
struct PartView {
    const double* pos[3];
    const double* mom[3];
    const double* weight;
    const int64_t* id;
    const int64_t* tile_start;
    bool tiles;
};

struct StateView {
    const double* fields;
    PartView sp[kMaxSpecies];
};

StateView context_view(const Ctx& c)
{
    StateView v{};
    v.fields = c.fields;
    for (int i = 0; i < c.nsp; ++i) {
        const Species& sp = c.sp[i];
        for (int ax = 0; ax < 3; ++ax) {
            v.sp[i].pos[ax] = (const double*)sp.cur.pos[ax];
            v.sp[i].mom[ax] = (const double*)sp.cur.mom[ax];
        }
        v.sp[i].weight = (const double*)sp.cur.weight;
        v.sp[i].id = sp.cur.id;
        v.sp[i].tile_start = sp.tile_start;
        v.sp[i].tiles = sp.sorted;
    }
    return v;
}

// Record layout (each array 256-byte aligned): E, B (6 N doubles); then per
// mobile species with particles, in species order: x (dims rows of n),
// w (3 rows), weight, id, tile table (ntiles + 1).  Carve with base ==
// nullptr to size it.
size_t carve_record(const Ctx& c, char* base, StateView* v)
{
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char* r = base ? base + off : nullptr;
        off += align_up(bytes, kAlign);
        return r;
    };
    const size_t N = (size_t)c.k.ncell;
    char* f = take(6 * N * 8);
    if (v) v->fields = (const double*)f;
    for (int i = 0; i < c.nsp; ++i) {
        const Species& sp = c.sp[i];
        if (!sp.d.mobile || sp.n == 0) continue;
        const size_t n = (size_t)sp.n;
        PartView pv{};
        for (int ax = 0; ax < c.k.dims; ++ax) pv.pos[ax] = (const double*)take(n * 8);
        for (int k = 0; k < 3; ++k) pv.mom[k] = (const double*)take(n * 8);
        pv.weight = (const double*)take(n * 8);
        pv.id = (const int64_t*)take(n * 8);
        pv.tile_start = (const int64_t*)take(((size_t)c.k.ntiles + 1) * 8);
        pv.tiles = true;
        if (v) v->sp[i] = pv;
    }
    return off;
}

// Copy of up to kMaxSeg arrays of 8-byte words in one launch (blockIdx.y =
// array).  src == nullptr: write the tile table of an unsorted species, an
// even split of its `fill` particles over count - 1 tiles (any particle may
// be processed in any tile; the table only spreads the work).
struct CopySeg {
    const uint64_t* src;
    uint64_t* dst;
    int64_t count;
    int64_t fill;
};
constexpr int kMaxSeg = 1 + kMaxSpecies * 8;
struct CopySegs {
    CopySeg s[kMaxSeg];
};

__global__ __launch_bounds__(256) void k_copy_segments(CopySegs segs)
{
    const CopySeg sg = segs.s[blockIdx.y];
    const int64_t stride = (int64_t)gridDim.x * 256;
    if (sg.src) {
        for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < sg.count; i += stride) sg.dst[i] = sg.src[i];
    } else {
        const int64_t tiles = sg.count - 1;
        for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < sg.count; i += stride)
            sg.dst[i] = (uint64_t)(i * sg.fill / tiles);
    }
}

// Particle adjoints from one order to another: pos_from[id] = k for the
// particle at position k of the source order (k_inverse), then
// out[j] = in[pos_from[id_to[j]]] (k_permute).  A null id array is id order.
__global__ __launch_bounds__(256) void k_inverse(const int64_t* __restrict__ id, int64_t n, uint32_t* __restrict__ pos)
{
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (k < n) pos[id[k]] = (uint32_t)k;
}

__global__ __launch_bounds__(256) void k_permute(const int64_t* __restrict__ id_to, const uint32_t* __restrict__ pos_from,
                                              int64_t n, const double* __restrict__ in_x, const double* __restrict__ in_w,
                                              double* __restrict__ out_x, double* __restrict__ out_w)
{
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= n) return;
    const int64_t pid = id_to ? id_to[j] : j;
    const int64_t src = pos_from ? (int64_t)pos_from[pid] : pid;
    for (int k = 0; k < 3; ++k) {
        out_x[k * n + j] = in_x[k * n + src];
        out_w[k * n + j] = in_w[k * n + src];
    }
}

}  // namespace

size_t adjoint_record_bytes(const Ctx& c) { return carve_record(c, nullptr, nullptr); }

hipError_t launch_adjoint_record(const Ctx& c, void* record, hipStream_t s)
{
    StateView v{};
    carve_record(c, (char*)record, &v);
    CopySegs segs{};
    int ns = 0;
    int64_t longest = 0;
    auto add = [&](const void* src, const void* dst, int64_t count, int64_t fill) {
        segs.s[ns++] = CopySeg{(const uint64_t*)src, (uint64_t*)dst, count, fill};
        longest = std::max(longest, count);
    };
    add(c.fields, v.fields, 6 * c.k.ncell, 0);
    for (int i = 0; i < c.nsp; ++i) {
        const Species& sp = c.sp[i];
        if (!sp.d.mobile || sp.n == 0) continue;
        const PartView& pv = v.sp[i];
        for (int ax = 0; ax < c.k.dims; ++ax) add(sp.cur.pos[ax], pv.pos[ax], sp.n, 0);
        for (int k = 0; k < 3; ++k) add(sp.cur.mom[k], pv.mom[k], sp.n, 0);
        add(sp.cur.weight, pv.weight, sp.n, 0);
        add(sp.cur.id, pv.id, sp.n, 0);
        add(sp.sorted ? sp.tile_start : nullptr, pv.tile_start, (int64_t)c.k.ntiles + 1, sp.n);
    }
    const unsigned gx = (unsigned)std::min<int64_t>(1024, std::max<int64_t>(1, (longest + 255) / 256));
    hipLaunchKernelGGL(k_copy_segments, dim3(gx, (unsigned)ns), dim3(256), 0, s, segs);
    return hipGetLastError();
}

hipError_t launch_adjoint_reorder(Ctx& c, const void* from, const void* to, const double* const* in_x,
                                  const double* const* in_w, double* const* out_x, double* const* out_w,
                                  hipStream_t s)
{
    StateView vf{}, vt{};
    if (from) carve_record(c, (char*)from, &vf);
    if (to) carve_record(c, (char*)to, &vt);
    for (int i = 0; i < c.nsp; ++i) {
        Species& sp = c.sp[i];
        if (!sp.d.mobile || sp.n == 0) continue;
        const unsigned pb = (unsigned)((sp.n + 255) / 256);
        uint32_t* pos = nullptr;
        if (from) {
            pos = sp.key;  // sort scratch, capacity >= n entries
            hipLaunchKernelGGL(k_inverse, dim3(pb), dim3(256), 0, s, vf.sp[i].id, sp.n, pos);
        }
        hipLaunchKernelGGL(k_permute, dim3(pb), dim3(256), 0, s, to ? vt.sp[i].id : nullptr, pos, sp.n, in_x[i],
                           in_w[i], out_x[i], out_w[i]);
    }
    return hipGetLastError();
}

hipError_t launch_adjoint_step(const Ctx& c, const void* record, bool by_id, double* lam, double* const* lam_x,
                               double* const* lam_w, double* lam_bext, hipStream_t s)
{
    StateView v{};
    if (record) carve_record(c, (char*)record, &v);
    else v = context_view(c);
    const int64_t N = c.k.ncell;
    const unsigned b = cells_blocks(N);
    hipLaunchKernelGGL(k_adj_pre, dim3(b), dim3(kCurlThreads), 0, s, c.k, v.fields, c.bn, lam, lam + 3 * N, c.adj);
    hipLaunchKernelGGL(k_adj_curl, dim3(b), dim3(kCurlThreads), 0, s, c.k, lam, lam + 3 * N);
    for (int i = 0; i < c.nsp; ++i) {
        const Species& sp = c.sp[i];
        if (!sp.d.mobile || sp.n == 0) continue;
        const PartView& pv = v.sp[i];
        AdjArgs a{};
        for (int ax = 0; ax < 3; ++ax) {
            a.pos[ax] = pv.pos[ax];
            a.mom[ax] = pv.mom[ax];
        }
        a.weight = pv.weight;
        a.id = pv.id;
        a.n = sp.n;
        a.count = sp.n;
        a.q = sp.d.q;
        a.qm = sp.d.q / sp.d.m;
        a.E = v.fields;
        a.Bn = c.bn;
        a.lamJ = c.adj;
        a.lamE = lam;
        a.lamB = lam + 3 * N;
        a.lam_x = lam_x[i];
        a.lam_w = lam_w[i];
        a.lam_bext = lam_bext;
        a.by_id = by_id ? 1 : 0;
        // the spare particle copy is free between sorts: lambda_Ep, lambda_Bp rows
        for (int k = 0; k < 3; ++k) {
            a.scr[k] = static_cast<double*>(sp.alt.pos[k]);
            a.scr[3 + k] = static_cast<double*>(sp.alt.mom[k]);
        }
        a.qslot = sp.alt.id;
        const unsigned pb = (unsigned)((sp.n + kAdjThreads - 1) / kAdjThreads);
        if (c.k.dims == 3 && pv.tiles) {
            const int split = (int)std::min<int64_t>(8, std::max<int64_t>(1, (512 + c.k.ntiles - 1) / c.k.ntiles));
            hipLaunchKernelGGL(k_adj_tile3, dim3((unsigned)(c.k.ntiles * split)), dim3(kAdjThreads3), 0, s, c.k, a,
                               pv.tile_start, split);
        } else if (c.k.dims == 3) {
            hipLaunchKernelGGL(k_adj_particles<3>, dim3(pb), dim3(kAdjThreads), 0, s, c.k, a);
        } else if (pv.tiles) {
            // enough workgroups to fill the chip: several per tile when tiles are few
            const int split = (int)std::min<int64_t>(8, std::max<int64_t>(1, (512 + c.k.ntiles - 1) / c.k.ntiles));
            hipLaunchKernelGGL(k_adj_tile2, dim3((unsigned)(c.k.ntiles * split)), dim3(kAdjThreads), 0, s, c.k, a,
                               pv.tile_start, split);
        } else {
            hipLaunchKernelGGL(k_adj_particles<2>, dim3(pb), dim3(kAdjThreads), 0, s, c.k, a);
        }
    }
    hipLaunchKernelGGL(k_adj_curl, dim3(b), dim3(kCurlThreads), 0, s, c.k, lam, lam + 3 * N);
    return hipGetLastError();
}

}  // namespace pic
