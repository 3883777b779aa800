// pic_math.h -- the per-particle arithmetic of one time step (paper
// Appendix), shared by the step kernels and by their adjoint: form factors
// (Section 4.5), gather (Eqs. alphax, betax), momentum and position advance
// (Eqs. p2, coordscheme), the charge-conserving current window (Eq. current)
// and the particle representations.  Templates on the arithmetic type R, so
// that the adjoint can evaluate the same formulas on dual numbers.
#pragma once

#include "pic_internal.h"

namespace pic {
namespace {

// ---------------------------------------------------------------------------
// Order-1 1/2 alternating form factor of one axis (Section 4.5): with
// i = floor(x), d = x - i, node weights (1-d; d) at nodes i, i+1 and cell
// weights ((1-d)^2/2; 3/4 - (1/2-d)^2; d^2/2) at cells i-1, i, i+1.
// ---------------------------------------------------------------------------
template <class R>
struct Axis {
    R f[2];
    R s[3];
};

template <class R>
__device__ __forceinline__ Axis<R> form_factor(R d)
{
    Axis<R> a;
    const R e = R(1) - d;
    const R h = R(0.5) - d;
    a.f[0] = e;
    a.f[1] = d;
    a.s[0] = R(0.5) * e * e;
    a.s[1] = R(0.75) - h * h;
    a.s[2] = R(0.5) * d * d;
    return a;
}

// Cell weights only (the end point of the move).
template <class R>
__device__ __forceinline__ void cell_weights(R d, R s[3])
{
    const R e = R(1) - d;
    const R h = R(0.5) - d;
    s[0] = R(0.5) * e * e;
    s[1] = R(0.75) - h * h;
    s[2] = R(0.5) * d * d;
}

// ---------------------------------------------------------------------------
// Gather (Eqs. alphax, betax).  F(comp, a, b, c) returns the grid value of
// component comp (0..2 = Ex..Ez, 3..5 = Bx..Bz) at offset (a, b, c) from the
// particle cell (a, b, c in {-1, 0, 1}; node factors use 0, 1).
// ---------------------------------------------------------------------------
template <class R, class Acc>
__device__ __forceinline__ void gather3(const Axis<R> (&w)[3], Acc F, R E[3], R B[3])
{
    const Axis<R>& X = w[0];
    const Axis<R>& Y = w[1];
    const Axis<R>& Z = w[2];
    // E^x: f_x(node) S_y S_z
    {
        R acc = 0;
        for (int a = 0; a < 2; ++a) {
            R sa = 0;
            for (int b = -1; b <= 1; ++b) {
                R sb = 0;
                for (int c = -1; c <= 1; ++c) sb += Z.s[c + 1] * F(0, a, b, c);
                sa += Y.s[b + 1] * sb;
            }
            acc += X.f[a] * sa;
        }
        E[0] = acc;
    }
    // E^y: S_x f_y S_z
    {
        R acc = 0;
        for (int a = -1; a <= 1; ++a) {
            R sa = 0;
            for (int b = 0; b < 2; ++b) {
                R sb = 0;
                for (int c = -1; c <= 1; ++c) sb += Z.s[c + 1] * F(1, a, b, c);
                sa += Y.f[b] * sb;
            }
            acc += X.s[a + 1] * sa;
        }
        E[1] = acc;
    }
    // E^z: S_x S_y f_z
    {
        R acc = 0;
        for (int a = -1; a <= 1; ++a) {
            R sa = 0;
            for (int b = -1; b <= 1; ++b) {
                R sb = Z.f[0] * F(2, a, b, 0) + Z.f[1] * F(2, a, b, 1);
                sa += Y.s[b + 1] * sb;
            }
            acc += X.s[a + 1] * sa;
        }
        E[2] = acc;
    }
    // B^x: S_x f_y f_z
    {
        R acc = 0;
        for (int a = -1; a <= 1; ++a) {
            R sa = 0;
            for (int b = 0; b < 2; ++b) {
                R sb = Z.f[0] * F(3, a, b, 0) + Z.f[1] * F(3, a, b, 1);
                sa += Y.f[b] * sb;
            }
            acc += X.s[a + 1] * sa;
        }
        B[0] = acc;
    }
    // B^y: f_x S_y f_z
    {
        R acc = 0;
        for (int a = 0; a < 2; ++a) {
            R sa = 0;
            for (int b = -1; b <= 1; ++b) {
                R sb = Z.f[0] * F(4, a, b, 0) + Z.f[1] * F(4, a, b, 1);
                sa += Y.s[b + 1] * sb;
            }
            acc += X.f[a] * sa;
        }
        B[1] = acc;
    }
    // B^z: f_x f_y S_z
    {
        R acc = 0;
        for (int a = 0; a < 2; ++a) {
            R sa = 0;
            for (int b = 0; b < 2; ++b) {
                R sb = 0;
                for (int c = -1; c <= 1; ++c) sb += Z.s[c + 1] * F(5, a, b, c);
                sa += Y.f[b] * sb;
            }
            acc += X.f[a] * sa;
        }
        B[2] = acc;
    }
}

// 2D3V: nothing depends on z, so every z sum of a partition of unity is 1.
template <class R, class Acc>
__device__ __forceinline__ void gather2(const Axis<R> (&w)[3], Acc F, R E[3], R B[3])
{
    const Axis<R>& X = w[0];
    const Axis<R>& Y = w[1];
    R ex = 0, ey = 0, ez = 0, bx = 0, by = 0, bz = 0;
    for (int a = 0; a < 2; ++a) {
        R s = 0;
        for (int b = -1; b <= 1; ++b) s += Y.s[b + 1] * F(0, a, b, 0);
        ex += X.f[a] * s;
    }
    for (int a = -1; a <= 1; ++a) {
        ey += X.s[a + 1] * (Y.f[0] * F(1, a, 0, 0) + Y.f[1] * F(1, a, 1, 0));
        R s = 0;
        for (int b = -1; b <= 1; ++b) s += Y.s[b + 1] * F(2, a, b, 0);
        ez += X.s[a + 1] * s;
        bx += X.s[a + 1] * (Y.f[0] * F(3, a, 0, 0) + Y.f[1] * F(3, a, 1, 0));
    }
    for (int a = 0; a < 2; ++a) {
        R s = 0;
        for (int b = -1; b <= 1; ++b) s += Y.s[b + 1] * F(4, a, b, 0);
        by += X.f[a] * s;
        bz += X.f[a] * (Y.f[0] * F(5, a, 0, 0) + Y.f[1] * F(5, a, 1, 0));
    }
    E[0] = ex;
    E[1] = ey;
    E[2] = ez;
    B[0] = bx;
    B[1] = by;
    B[2] = bz;
}

// ---------------------------------------------------------------------------
// a / sqrt(x) and a / x: correctly rounded in FP64 (the parity mode); in FP32
// through the hardware reciprocal square root and reciprocal (about 1 ulp),
// whose error stays far below what the FP32 representation of the particle
// already carries.
// ---------------------------------------------------------------------------
template <class R>
__device__ __forceinline__ R over_sqrt(R a, R x) { return a / sqrt(x); }
template <>
__device__ __forceinline__ float over_sqrt<float>(float a, float x) { return a * __builtin_amdgcn_rsqf(x); }
template <class R>
__device__ __forceinline__ R over(R a, R x) { return a / x; }
template <>
__device__ __forceinline__ float over<float>(float a, float x) { return a * __builtin_amdgcn_rcpf(x); }

// ---------------------------------------------------------------------------
// Momentum advance (Appendix): e = q dt E/(2m); w~ = w + e;
// b = q dt B / (2 m sqrt(w~^2 + c^2)); w' = w~ + w~ x b;
// w_new = w~ + e + 2 (w' x b)/(1 + b^2).
// ---------------------------------------------------------------------------
template <class R>
__device__ __forceinline__ void push(R qmdt2, R c2, const R E[3], const R B[3], R w[3])
{
    R e[3], wt[3], b[3];
    for (int a = 0; a < 3; ++a) e[a] = qmdt2 * E[a];
    for (int a = 0; a < 3; ++a) wt[a] = w[a] + e[a];
    const R k = over_sqrt<R>(qmdt2, wt[0] * wt[0] + wt[1] * wt[1] + wt[2] * wt[2] + c2);
    for (int a = 0; a < 3; ++a) b[a] = k * B[a];
    const R wp0 = wt[0] + (wt[1] * b[2] - wt[2] * b[1]);
    const R wp1 = wt[1] + (wt[2] * b[0] - wt[0] * b[2]);
    const R wp2 = wt[2] + (wt[0] * b[1] - wt[1] * b[0]);
    const R s = over<R>(R(2), R(1) + b[0] * b[0] + b[1] * b[1] + b[2] * b[2]);
    w[0] = wt[0] + e[0] + s * (wp1 * b[2] - wp2 * b[1]);
    w[1] = wt[1] + e[1] + s * (wp2 * b[0] - wp0 * b[2]);
    w[2] = wt[2] + e[2] + s * (wp0 * b[1] - wp1 * b[0]);
}

// ---------------------------------------------------------------------------
// Current of one particle (Eq. current, one-quarter form).  Per axis the
// start and end cell weights are placed on a common window of 4 cells
// starting at s = min(i0, i1) - 1; dm = S1 - S0, dp = S1 + S0 on the window;
// the cumulative difference at face s+t+1 is P_t = sum_{t' <= t} dm_t'
// (t = 0..2; the face s+4 gets sum of all dm = 0).  The last prefix is taken
// as -dm_3, which is the same value and exactly zero whenever the window's
// last cell is empty.  A contribution is the face factor P_t times the
// transverse factor; both are converted to FP64 once and the product is
// formed there (exact for FP32 factors), and handed to the sink as FP64.
// ---------------------------------------------------------------------------
template <class R>
__device__ __forceinline__ void window(const R s0[3], const R s1[3], int delta, R dm[4], R dp[4])
{
    const bool o0 = delta < 0;  // start weights shifted one cell right in the window
    const bool o1 = delta > 0;  // end weights shifted one cell right
    const R a0 = o0 ? R(0) : s0[0], a1 = o0 ? s0[0] : s0[1], a2 = o0 ? s0[1] : s0[2],
            a3 = o0 ? s0[2] : R(0);
    const R b0 = o1 ? R(0) : s1[0], b1 = o1 ? s1[0] : s1[1], b2 = o1 ? s1[1] : s1[2],
            b3 = o1 ? s1[2] : R(0);
    dm[0] = b0 - a0;
    dm[1] = b1 - a1;
    dm[2] = b2 - a2;
    dm[3] = b3 - a3;
    dp[0] = b0 + a0;
    dp[1] = b1 + a1;
    dp[2] = b2 + a2;
    dp[3] = b3 + a3;
}

// Sink(comp, ix, iy, iz, v) adds v to component comp at window position
// (ix, iy, iz), each in 0..3 (window cells s..s+3; the face s+t+1 of the
// component's own axis is position t+1).
template <class R, class Sink>
__device__ __forceinline__ void deposit3(const R (&dm)[3][4], const R (&dp)[3][4],
                                         const R jfac[3], Sink S)
{
    const R third = R(1) / R(3);
    R m3[3][4];
    for (int a = 0; a < 3; ++a)
        for (int t = 0; t < 4; ++t) m3[a][t] = dm[a][t] * third;
    for (int comp = 0; comp < 3; ++comp) {
        const int u = (comp + 1) % 3, v = (comp + 2) % 3;
        double P[3];
        P[0] = dm[comp][0] * jfac[comp];
        P[1] = (dm[comp][0] + dm[comp][1]) * jfac[comp];
        P[2] = -dm[comp][3] * jfac[comp];
        for (int b = 0; b < 4; ++b)
            for (int c = 0; c < 4; ++c) {
                const double tr = dp[u][b] * dp[v][c] + m3[u][b] * dm[v][c];
                for (int t = 0; t < 3; ++t) {
                    int ijk[3];
                    ijk[comp] = t + 1;
                    ijk[u] = b;
                    ijk[v] = c;
                    S(comp, ijk[0], ijk[1], ijk[2], P[t] * tr);
                }
            }
    }
}

// A particle that stays in its cell (shift 0 on every axis) has start and end
// weights on the same three cells per axis, so the window's fourth cell and
// the face s+3 carry exactly zero: only faces s+1, s+2 and cells s..s+2 remain,
// 2 x 3 x 3 = 18 contributions per component.  The values are those of
// deposit3 on the same window.
template <class R, class Sink>
__device__ __forceinline__ void deposit3_still(const R (&s0)[3][3], const R (&s1)[3][3],
                                               const R jfac[3], Sink S)
{
    const R third = R(1) / R(3);
    R dm[3][3], dp[3][3], m3[3][3];
    for (int a = 0; a < 3; ++a)
        for (int k = 0; k < 3; ++k) {
            dm[a][k] = s1[a][k] - s0[a][k];
            dp[a][k] = s1[a][k] + s0[a][k];
            m3[a][k] = dm[a][k] * third;
        }
    for (int comp = 0; comp < 3; ++comp) {
        const int u = (comp + 1) % 3, v = (comp + 2) % 3;
        const double P0 = dm[comp][0] * jfac[comp];
        const double P1 = (dm[comp][0] + dm[comp][1]) * jfac[comp];
        for (int b = 0; b < 3; ++b)
            for (int c = 0; c < 3; ++c) {
                const double tr = dp[u][b] * dp[v][c] + m3[u][b] * dm[v][c];
                int ijk[3];
                ijk[u] = b;
                ijk[v] = c;
                ijk[comp] = 1;
                S(comp, ijk[0], ijk[1], ijk[2], P0 * tr);
                ijk[comp] = 2;
                S(comp, ijk[0], ijk[1], ijk[2], P1 * tr);
            }
    }
}

// A particle that crosses a cell face along axis A only (shift 0 on the other
// two axes): on those axes the window's fourth cell and the face s+3 carry
// exactly zero, leaving 3 x 3 x 3 contributions for the component along A and
// 2 x 4 x 3 for each other component (75 in all).  The values are those of
// deposit3 on the same window.
template <int A, class R, class Sink>
__device__ __forceinline__ void deposit3_axis(const R (&dm)[3][4], const R (&dp)[3][4], const R jfac[3],
                                              Sink S)
{
    const R third = R(1) / R(3);
    for (int comp = 0; comp < 3; ++comp) {
        const int u = (comp + 1) % 3, v = (comp + 2) % 3;
        const int nt = comp == A ? 3 : 2;
        const int nb = u == A ? 4 : 3, nc = v == A ? 4 : 3;
        double P[3];
        P[0] = dm[comp][0] * jfac[comp];
        P[1] = (dm[comp][0] + dm[comp][1]) * jfac[comp];
        P[2] = -dm[comp][3] * jfac[comp];
        for (int b = 0; b < nb; ++b)
            for (int c = 0; c < nc; ++c) {
                const double tr = dp[u][b] * dp[v][c] + (dm[u][b] * third) * dm[v][c];
                for (int t = 0; t < nt; ++t) {
                    int ijk[3];
                    ijk[comp] = t + 1;
                    ijk[u] = b;
                    ijk[v] = c;
                    S(comp, ijk[0], ijk[1], ijk[2], P[t] * tr);
                }
            }
    }
}

// 2D3V: the z sums collapse (sum of dp_z = 2, sum of dm_z = 0, sum over the
// z faces of P_z = z0 - z1), leaving 12 + 12 + 16 contributions.  jz is the
// J^z factor per unit transverse weight: (q/V) u_z / 4.
template <class R, class Sink>
__device__ __forceinline__ void deposit2(const R (&dm)[3][4], const R (&dp)[3][4],
                                         const R jfac[3], R jz, Sink S)
{
    const R third = R(1) / R(3);
    for (int comp = 0; comp < 2; ++comp) {
        const int u = 1 - comp;
        R P[3];
        P[0] = dm[comp][0];
        P[1] = dm[comp][0] + dm[comp][1];
        P[2] = -dm[comp][3];
        for (int t = 0; t < 3; ++t) P[t] *= R(2) * jfac[comp];
        for (int b = 0; b < 4; ++b)
            for (int t = 0; t < 3; ++t) {
                int ij[2];
                ij[comp] = t + 1;
                ij[u] = b;
                S(comp, ij[0], ij[1], 0, (double)(P[t] * dp[u][b]));
            }
    }
    for (int a = 0; a < 4; ++a) {
        const R mx = dm[0][a] * third;
        for (int b = 0; b < 4; ++b) S(2, a, b, 0, (double)(jz * (dp[0][a] * dp[1][b] + mx * dm[1][b])));
    }
}

// ---------------------------------------------------------------------------
// Alternating order 2 1/2 (Section 4.5): with i = int(x + 1/2) and
// d = x + 1/2 - i, the node factors f_{i-1:i+1} are the quadratic spline
// ((1-d)^2/2; 3/4-(1/2-d)^2; d^2/2) and the cell factors
// Delta F_{i-3/2:i+3/2} the cubic one ((1-d)^3/6; (2-d)^3/6-2(1-d)^3/3;
// (1+d)^3/6-2d^3/3; d^3/6).  Positions are stored as cell c = floor(x) and
// offset d0 = x - c; then i = c + h with h = (d0 >= 1/2), so node k of the
// table sits at offset h - 1 + k from c and cell k at offset h - 2 + k.
// ---------------------------------------------------------------------------
template <class R>
struct Axis2 {
    R f[3];  // nodes c+h-1 .. c+h+1
    R s[4];  // cells c+h-2 .. c+h+1
    int h;
};

template <class R>
__device__ __forceinline__ void cell_weights2(R d, R s[4])
{
    const R e = R(1) - d;
    const R e3 = e * e * e, d3 = d * d * d;
    const R t = R(2) - d, u = R(1) + d;
    s[0] = e3 * R(1.0 / 6.0);
    s[1] = t * t * t * R(1.0 / 6.0) - R(2.0 / 3.0) * e3;
    s[2] = u * u * u * R(1.0 / 6.0) - R(2.0 / 3.0) * d3;
    s[3] = d3 * R(1.0 / 6.0);
}

// d0 in [0, 1): the offset from the cell.
template <class R>
__device__ __forceinline__ Axis2<R> form_factor2(R d0)
{
    Axis2<R> a;
    a.h = d0 >= R(0.5) ? 1 : 0;
    const R d = d0 + R(0.5) - R(a.h);
    const R e = R(1) - d;
    const R m = R(0.5) - d;
    a.f[0] = R(0.5) * e * e;
    a.f[1] = R(0.75) - m * m;
    a.f[2] = R(0.5) * d * d;
    cell_weights2<R>(d, a.s);
    return a;
}

// Gather (Eqs. alphax, betax) at order 2 1/2: F(comp, oa, ob, oc) returns the
// grid value at offsets (oa, ob, oc) in [-2, 2] from the particle cell.  3D:
// 48 points for each E component and 36 for each B component.
template <class R, class Acc>
__device__ __forceinline__ void gather3_o2(const Axis2<R> (&w)[3], Acc F, R E[3], R B[3])
{
    const Axis2<R>& X = w[0];
    const Axis2<R>& Y = w[1];
    const Axis2<R>& Z = w[2];
    const int nx = X.h - 1, ny = Y.h - 1, nz = Z.h - 1;  // first node offset
    const int cx = X.h - 2, cy = Y.h - 2, cz = Z.h - 2;  // first cell offset
    R ex = 0, ey = 0, ez = 0, bx = 0, by = 0, bz = 0;
    for (int c = 0; c < 4; ++c) {
        R sx = 0, sy = 0;
        for (int b = 0; b < 4; ++b) {
            R t = 0;
            for (int a = 0; a < 3; ++a) t += X.f[a] * F(0, nx + a, cy + b, cz + c);
            sx += Y.s[b] * t;
        }
        ex += Z.s[c] * sx;
        for (int b = 0; b < 3; ++b) {
            R t = 0;
            for (int a = 0; a < 4; ++a) t += X.s[a] * F(1, cx + a, ny + b, cz + c);
            sy += Y.f[b] * t;
        }
        ey += Z.s[c] * sy;
    }
    for (int c = 0; c < 3; ++c) {
        R sz = 0, sbx = 0, sby = 0;
        for (int b = 0; b < 4; ++b) {
            R t = 0;
            for (int a = 0; a < 4; ++a) t += X.s[a] * F(2, cx + a, cy + b, nz + c);
            sz += Y.s[b] * t;
        }
        ez += Z.f[c] * sz;
        for (int b = 0; b < 3; ++b) {
            R t = 0;
            for (int a = 0; a < 4; ++a) t += X.s[a] * F(3, cx + a, ny + b, nz + c);
            sbx += Y.f[b] * t;
        }
        bx += Z.f[c] * sbx;
        for (int b = 0; b < 4; ++b) {
            R t = 0;
            for (int a = 0; a < 3; ++a) t += X.f[a] * F(4, nx + a, cy + b, nz + c);
            sby += Y.s[b] * t;
        }
        by += Z.f[c] * sby;
    }
    for (int c = 0; c < 4; ++c) {
        R s = 0;
        for (int b = 0; b < 3; ++b) {
            R t = 0;
            for (int a = 0; a < 3; ++a) t += X.f[a] * F(5, nx + a, ny + b, cz + c);
            s += Y.f[b] * t;
        }
        bz += Z.s[c] * s;
    }
    E[0] = ex;
    E[1] = ey;
    E[2] = ez;
    B[0] = bx;
    B[1] = by;
    B[2] = bz;
}

// 2D3V: the z factors sum to one on the single plane.
template <class R, class Acc>
__device__ __forceinline__ void gather2_o2(const Axis2<R> (&w)[3], Acc F, R E[3], R B[3])
{
    const Axis2<R>& X = w[0];
    const Axis2<R>& Y = w[1];
    const int nx = X.h - 1, ny = Y.h - 1, cx = X.h - 2, cy = Y.h - 2;
    R ex = 0, ey = 0, ez = 0, bx = 0, by = 0, bz = 0;
    for (int b = 0; b < 4; ++b) {
        R t0 = 0, t2 = 0, t4 = 0;
        for (int a = 0; a < 3; ++a) {
            t0 += X.f[a] * F(0, nx + a, cy + b, 0);
            t4 += X.f[a] * F(4, nx + a, cy + b, 0);
        }
        for (int a = 0; a < 4; ++a) t2 += X.s[a] * F(2, cx + a, cy + b, 0);
        ex += Y.s[b] * t0;
        ez += Y.s[b] * t2;
        by += Y.s[b] * t4;
    }
    for (int b = 0; b < 3; ++b) {
        R t1 = 0, t3 = 0, t5 = 0;
        for (int a = 0; a < 4; ++a) {
            t1 += X.s[a] * F(1, cx + a, ny + b, 0);
            t3 += X.s[a] * F(3, cx + a, ny + b, 0);
        }
        for (int a = 0; a < 3; ++a) t5 += X.f[a] * F(5, nx + a, ny + b, 0);
        ey += Y.f[b] * t1;
        bx += Y.f[b] * t3;
        bz += Y.f[b] * t5;
    }
    E[0] = ex;
    E[1] = ey;
    E[2] = ez;
    B[0] = bx;
    B[1] = by;
    B[2] = bz;
}

// Current window at order 2 1/2: start and end cell factors (4 cells each,
// from i0 - 2 and i1 - 2 with i = int(x + 1/2)) on a common window of 5 cells
// starting at s = min(i0, i1) - 2; shift = i1 - i0 in {-1, 0, 1}.
template <class R>
__device__ __forceinline__ void window5(const R s0[4], const R s1[4], int shift, R dm[5], R dp[5])
{
    // start (end) weights one window cell right when shift < 0 (> 0); two-way
    // selects, since a store at a run-time index becomes a chain of compares
    const bool o0 = shift < 0, o1 = shift > 0;
    R a[5], b[5];
#pragma unroll
    for (int t = 0; t < 5; ++t) {
        a[t] = o0 ? (t > 0 ? s0[t - 1] : R(0)) : (t < 4 ? s0[t] : R(0));
        b[t] = o1 ? (t > 0 ? s1[t - 1] : R(0)) : (t < 4 ? s1[t] : R(0));
    }
#pragma unroll
    for (int t = 0; t < 5; ++t) {
        dm[t] = b[t] - a[t];
        dp[t] = b[t] + a[t];
    }
}

// Current of one particle at order 2 1/2 (Eq. current, one-quarter form):
// the same formula as deposit3 on 5-cell windows, faces s+1 .. s+4 (the face
// s+5 gets the sum of all dm = 0); 4 x 5 x 5 = 100 contributions per
// component.  Sink(comp, ix, iy, iz, v) as for deposit3.
template <class R, class Sink>
__device__ __forceinline__ void deposit3_o2(const R (&dm)[3][5], const R (&dp)[3][5], const R jfac[3], Sink S)
{
    const R third = R(1) / R(3);
    for (int comp = 0; comp < 3; ++comp) {
        const int u = (comp + 1) % 3, v = (comp + 2) % 3;
        R P[4];
        P[0] = dm[comp][0];
        P[1] = P[0] + dm[comp][1];
        P[2] = P[1] + dm[comp][2];
        P[3] = -dm[comp][4];
        for (int t = 0; t < 4; ++t) P[t] *= jfac[comp];
        for (int b = 0; b < 5; ++b)
            for (int c = 0; c < 5; ++c) {
                const R tr = dp[u][b] * dp[v][c] + (dm[u][b] * third) * dm[v][c];
                for (int t = 0; t < 4; ++t) {
                    int ijk[3];
                    ijk[comp] = t + 1;
                    ijk[u] = b;
                    ijk[v] = c;
                    S(comp, ijk[0], ijk[1], ijk[2], P[t] * tr);
                }
            }
    }
}

// A particle whose int(x + 1/2) stays the same on every axis has start and
// end factors on the same 4 cells per axis: the window's fifth cell and the
// face s+4 carry exactly zero, leaving 3 x 4 x 4 contributions per component
// (144 in all).  The values are those of deposit3_o2 on the same window.
template <class R, class Sink>
__device__ __forceinline__ void deposit3_o2_still(const R (&dm)[3][5], const R (&dp)[3][5], const R jfac[3],
                                                  Sink S)
{
    const R third = R(1) / R(3);
    for (int comp = 0; comp < 3; ++comp) {
        const int u = (comp + 1) % 3, v = (comp + 2) % 3;
        R P[3];
        P[0] = dm[comp][0];
        P[1] = P[0] + dm[comp][1];
        P[2] = P[1] + dm[comp][2];
        for (int t = 0; t < 3; ++t) P[t] *= jfac[comp];
        for (int b = 0; b < 4; ++b)
            for (int c = 0; c < 4; ++c) {
                const R tr = dp[u][b] * dp[v][c] + (dm[u][b] * third) * dm[v][c];
                for (int t = 0; t < 3; ++t) {
                    int ijk[3];
                    ijk[comp] = t + 1;
                    ijk[u] = b;
                    ijk[v] = c;
                    S(comp, ijk[0], ijk[1], ijk[2], P[t] * tr);
                }
            }
    }
}

// 2D3V at order 2 1/2: 20 + 20 + 25 contributions (z collapsed as in
// deposit2).
template <class R, class Sink>
__device__ __forceinline__ void deposit2_o2(const R (&dm)[3][5], const R (&dp)[3][5], const R jfac[3], R jz,
                                            Sink S)
{
    const R third = R(1) / R(3);
    for (int comp = 0; comp < 2; ++comp) {
        const int u = 1 - comp;
        R P[4];
        P[0] = dm[comp][0];
        P[1] = P[0] + dm[comp][1];
        P[2] = P[1] + dm[comp][2];
        P[3] = -dm[comp][4];
        for (int t = 0; t < 4; ++t) P[t] *= R(2) * jfac[comp];
        for (int b = 0; b < 5; ++b)
            for (int t = 0; t < 4; ++t) {
                int ij[2];
                ij[comp] = t + 1;
                ij[u] = b;
                S(comp, ij[0], ij[1], 0, P[t] * dp[u][b]);
            }
    }
    for (int a = 0; a < 5; ++a) {
        const R mx = dm[0][a] * third;
        for (int b = 0; b < 5; ++b) S(2, a, b, 0, jz * (dp[0][a] * dp[1][b] + mx * dm[1][b]));
    }
}

// ---------------------------------------------------------------------------
// The "conventional" uniform-order interpolation of Eq. wrong1 (the comparison
// of Section 5): along a component's node axes the weight of node n is the
// mean of the order-1 1/2 cell factors of the two cells that share it,
// (Delta F_{n-1/2} + Delta F_{n+1/2}) / 2, on nodes c-1 .. c+2; along its
// cell axes it is Delta F on cells c-1 .. c+1.  3D: 36 points per E
// component, 48 per B component.  The charge and current are those of the
// order-1 1/2 scheme.
// ---------------------------------------------------------------------------
template <class R>
struct AxisC {
    R g[4];  // nodes c-1 .. c+2
    R s[3];  // cells c-1 .. c+1
};

template <class R>
__device__ __forceinline__ AxisC<R> form_factor_conv(R d)
{
    AxisC<R> a;
    cell_weights<R>(d, a.s);
    a.g[0] = R(0.5) * a.s[0];
    a.g[1] = R(0.5) * (a.s[0] + a.s[1]);
    a.g[2] = R(0.5) * (a.s[1] + a.s[2]);
    a.g[3] = R(0.5) * a.s[2];
    return a;
}

// F(comp, oa, ob, oc): grid value at offsets in [-1, 2] from the particle cell.
template <class R, class Acc>
__device__ __forceinline__ void gather3_conv(const AxisC<R> (&w)[3], Acc F, R E[3], R B[3])
{
    const AxisC<R>& X = w[0];
    const AxisC<R>& Y = w[1];
    const AxisC<R>& Z = w[2];
    R ex = 0, ey = 0, ez = 0, bx = 0, by = 0, bz = 0;
    for (int c = 0; c < 3; ++c) {
        R sx = 0, sy = 0;
        for (int b = 0; b < 3; ++b) {
            R t = 0;
            for (int a = 0; a < 4; ++a) t += X.g[a] * F(0, a - 1, b - 1, c - 1);
            sx += Y.s[b] * t;
        }
        ex += Z.s[c] * sx;
        for (int b = 0; b < 4; ++b) {
            R t = 0;
            for (int a = 0; a < 3; ++a) t += X.s[a] * F(1, a - 1, b - 1, c - 1);
            sy += Y.g[b] * t;
        }
        ey += Z.s[c] * sy;
    }
    for (int c = 0; c < 4; ++c) {
        R sz = 0, sbx = 0, sby = 0;
        for (int b = 0; b < 3; ++b) {
            R t = 0;
            for (int a = 0; a < 3; ++a) t += X.s[a] * F(2, a - 1, b - 1, c - 1);
            sz += Y.s[b] * t;
        }
        ez += Z.g[c] * sz;
        for (int b = 0; b < 4; ++b) {
            R t = 0;
            for (int a = 0; a < 3; ++a) t += X.s[a] * F(3, a - 1, b - 1, c - 1);
            sbx += Y.g[b] * t;
        }
        bx += Z.g[c] * sbx;
        for (int b = 0; b < 3; ++b) {
            R t = 0;
            for (int a = 0; a < 4; ++a) t += X.g[a] * F(4, a - 1, b - 1, c - 1);
            sby += Y.s[b] * t;
        }
        by += Z.g[c] * sby;
    }
    for (int c = 0; c < 3; ++c) {
        R s = 0;
        for (int b = 0; b < 4; ++b) {
            R t = 0;
            for (int a = 0; a < 4; ++a) t += X.g[a] * F(5, a - 1, b - 1, c - 1);
            s += Y.g[b] * t;
        }
        bz += Z.s[c] * s;
    }
    E[0] = ex;
    E[1] = ey;
    E[2] = ez;
    B[0] = bx;
    B[1] = by;
    B[2] = bz;
}

// 2D3V: the z weights sum to one on the single plane.
template <class R, class Acc>
__device__ __forceinline__ void gather2_conv(const AxisC<R> (&w)[3], Acc F, R E[3], R B[3])
{
    const AxisC<R>& X = w[0];
    const AxisC<R>& Y = w[1];
    R ex = 0, ey = 0, ez = 0, bx = 0, by = 0, bz = 0;
    for (int b = 0; b < 3; ++b) {
        R t0 = 0, t2 = 0, t4 = 0;
        for (int a = 0; a < 4; ++a) {
            t0 += X.g[a] * F(0, a - 1, b - 1, 0);
            t4 += X.g[a] * F(4, a - 1, b - 1, 0);
        }
        for (int a = 0; a < 3; ++a) t2 += X.s[a] * F(2, a - 1, b - 1, 0);
        ex += Y.s[b] * t0;
        ez += Y.s[b] * t2;
        by += Y.s[b] * t4;
    }
    for (int b = 0; b < 4; ++b) {
        R t1 = 0, t3 = 0, t5 = 0;
        for (int a = 0; a < 3; ++a) {
            t1 += X.s[a] * F(1, a - 1, b - 1, 0);
            t3 += X.s[a] * F(3, a - 1, b - 1, 0);
        }
        for (int a = 0; a < 4; ++a) t5 += X.g[a] * F(5, a - 1, b - 1, 0);
        ey += Y.g[b] * t1;
        bx += Y.g[b] * t3;
        bz += Y.g[b] * t5;
    }
    E[0] = ex;
    E[1] = ey;
    E[2] = ez;
    B[0] = bx;
    B[1] = by;
    B[2] = bz;
}

// Workgroup -> tile map: consecutive workgroup ids are dealt round-robin to
// the 8 XCDs, so give each XCD a contiguous run of tiles (neighbouring tiles
// share field rows and J guard cells in that XCD's L2).
__device__ __forceinline__ int xcd_tile(int bid, int ntiles)
{
    const int per = ntiles / kXcds, rem = ntiles % kXcds;
    const int x = bid % kXcds, local = bid / kXcds;
    return x < rem ? x * (per + 1) + local : rem * (per + 1) + (x - rem) * per + local;
}

// ---------------------------------------------------------------------------
// Particle representations.
// ---------------------------------------------------------------------------
struct StepArgs {
    void* pos[3];
    void* mom[3];
    const void* weight;
    uint32_t* cell;
    const int64_t* tile_start;
    double q;        // charge per unit weight
    double qm;       // q / m
    unsigned long long* counters;
    // queue of the tile's cell-crossing particles, kept in the spare copy of
    // the particle arrays (idle between sorts) at the tile's own index range:
    // start offsets qd0[a] and one packed word per entry
    void* qd0[3];
    int64_t* qword;
    // 3D: the class map of the crossing queue (32-bit entry offsets), in the
    // spare copy's weight array, and the migrants whose bucket was full
    // (32-bit slot offsets), in its third momentum array
    void* qmap;
    void* qother;
    // 3D: the tile's migrant list (slot offsets; rank and neighbour code), in
    // the spare copy's first two momentum arrays
    void* mlist;
    void* mlist2;
    // 3D migrant buckets: mig_cap particle indices per tile at mig + tile *
    // mig_cap, filled through the per-tile counters mig_n (zero between
    // launches: the migrant kernel clears the counter it reads)
    uint32_t* mig;
    unsigned int* mig_n;
    uint32_t mig_cap;
};

__device__ __forceinline__ int wrapi(int v, int n)
{
    int r = v % n;
    return r < 0 ? r + n : r;
}

// Periodic wrap of v in [-n, 2n): one compare-and-add instead of a modulo.
__device__ __forceinline__ int wrap1(int v, int n)
{
    v = v < 0 ? v + n : v;
    return v >= n ? v - n : v;
}

__device__ __forceinline__ uint32_t pack_cell(int i, int j, int k)
{
    return (uint32_t)i | ((uint32_t)j << 11) | ((uint32_t)k << 22);
}

__device__ __forceinline__ void unpack_cell(uint32_t c, int i[3])
{
    i[0] = (int)(c & 2047u);
    i[1] = (int)((c >> 11) & 2047u);
    i[2] = (int)(c >> 22);
}

// Load the start state: cell index i[a], offset d[a] in [0,1).
template <class R, int D>
struct PosIO;

template <int D>
struct PosIO<double, D> {
    static __device__ __forceinline__ void cell(const StepArgs& a, int64_t p, int i[3])
    {
        for (int ax = 0; ax < 3; ++ax) i[ax] = ax < D ? (int)floor(((const double*)a.pos[ax])[p]) : 0;
    }
    static __device__ __forceinline__ void load(const StepArgs& a, int64_t p, int i[3], double d[3])
    {
        for (int ax = 0; ax < D; ++ax) {
            const double x = ((const double*)a.pos[ax])[p];
            const double fl = floor(x);
            i[ax] = (int)fl;
            d[ax] = x - fl;
        }
        if (D == 2) {
            i[2] = 0;
            d[2] = 0.0;
        }
    }
    // Advance by disp (cell units), wrap, store; return the end offsets d1 and
    // the cell shift delta in {-1, 0, 1} consistent with the stored position.
    static __device__ __forceinline__ void move(const StepArgs& a, int64_t p, const GridK& g,
                                                const int i0[3], const double d0[3],
                                                const double disp[3], double d1[3], int delta[3],
                                                bool store)
    {
        for (int ax = 0; ax < D; ++ax) {
            const double N = (double)g.n[ax];
            double x = ((double)i0[ax] + d0[ax]) + disp[ax];
            if (x >= N) x -= N;
            if (x < 0.0) x += N;
            if (x >= N) x -= N;  // a tiny negative value can round up to N
            const double fl = floor(x);
            d1[ax] = x - fl;
            // in {-1, 0, 1} for any finite move shorter than a cell; the clamp
            // keeps window indices in range for non-finite input
            const double dd = rint((d0[ax] + disp[ax]) - d1[ax]);
            delta[ax] = dd > 0.5 ? 1 : (dd < -0.5 ? -1 : 0);
            if (store) ((double*)a.pos[ax])[p] = x;
        }
    }
};

template <int D>
struct PosIO<float, D> {
    static __device__ __forceinline__ void cell(const StepArgs& a, int64_t p, int i[3]) { unpack_cell(a.cell[p], i); }
    static __device__ __forceinline__ void load(const StepArgs& a, int64_t p, int i[3], float d[3])
    {
        unpack_cell(a.cell[p], i);
        for (int ax = 0; ax < D; ++ax) d[ax] = ((const float*)a.pos[ax])[p];
        if (D == 2) d[2] = 0.0f;
    }
    static __device__ __forceinline__ void move(const StepArgs& a, int64_t p, const GridK& g,
                                                const int i0[3], const float d0[3],
                                                const float disp[3], float d1[3], int delta[3],
                                                bool store)
    {
        int i1[3] = {i0[0], i0[1], i0[2]};
        for (int ax = 0; ax < D; ++ax) {
            float o = d0[ax] + disp[ax];
            int dl = 0;
            if (o >= 1.0f) {
                o -= 1.0f;  // exact: o is in [1, 2)
                dl = 1;
            } else if (o < 0.0f) {
                o += 1.0f;
                dl = -1;
                if (o >= 1.0f) {  // |o| below half an ulp of 1: the position is the node
                    o = 0.0f;
                    dl = 0;
                }
            }
            d1[ax] = o;
            delta[ax] = dl;
            int c = i0[ax] + dl;
            c = c < 0 ? c + g.n[ax] : (c >= g.n[ax] ? c - g.n[ax] : c);
            i1[ax] = c;
            if (store) ((float*)a.pos[ax])[p] = o;
        }
        // a particle that stays in its cell keeps its stored cell word
        if (store && (delta[0] | delta[1] | delta[2])) a.cell[p] = pack_cell(i1[0], i1[1], i1[2]);
    }
};


}  // namespace
}  // namespace pic
