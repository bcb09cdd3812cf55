// Track-to-tracklet matching for gfx950: one seed track per lane.
//
// Per layer (Sect. 3 of the paper): propagate the helix state and its
// covariance to the chamber plane, hop into the neighbouring sector frame if
// the point left the sector, add the layer's multiple scattering, open the
// covariance road, scan the tracklet cells the road overlaps (linear
// extrapolation to each chamber's radius, pad-tilt corrected y residual, dy
// exclusion at n sigma, chi2 from y and z only), keep the lexicographic best
// (chi2, tracklet index), propagate precisely to the winner's radius and run
// the Joseph-form Kalman update.
//
// TS is the precision of the state and of the candidate gates, TC that of
// the covariance.  <double,double> is the plain double-precision matcher,
// <float,float> the fast one whose tracks are re-run as <float,double> when
// the float covariance stops being positive definite.
#include "trd_internal.h"

namespace trd {

namespace {

// packed upper triangle of the symmetric 5x5 covariance, row-major
enum : int {
    YY = 0, YZ, YS, YT, YC,
    ZZ, ZS, ZT, ZC,
    SS, ST, SC,
    TT, TC_,
    CC
};

template <typename TS, typename TC>
struct Trk {
    TS y, z, s, t, c, x;
    TC C[15];
    int sec;
};

template <typename T> __device__ __forceinline__ T sq(T a) { return a * a; }

// integers in rows of the state type: bit pattern in float, value in double
__device__ __forceinline__ float as_row(int v, float) { return __int_as_float(v); }
__device__ __forceinline__ double as_row(int v, double) { return (double)v; }
__device__ __forceinline__ int int_of(float v) { return __float_as_int(v); }
__device__ __forceinline__ int int_of(double v) { return (int)v; }

// Division: the float paths take one hardware reciprocal (1 ulp) and a
// multiply instead of the IEEE division sequence (the float state is held to
// 1e-5 anyway); the double paths divide exactly.
__device__ __forceinline__ float div_(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
__device__ __forceinline__ double div_(double a, double b) { return a / b; }

// sin(u)/u, asin(h)/h and (sin d - d)/d^2 of the helix step.  The float
// forms use their Taylor series where the turning angle is small (|u| < 0.5:
// first omitted term below 3e-11; h < 0.3: below 1e-8) and the library
// functions beyond, which costs a fraction of the library's argument
// reduction; the double forms call the library (gfun: series below 0.5).
template <typename T> __device__ __forceinline__ T sinc_(T u) { return u == T(0) ? T(1) : div_(T(sin(u)), u); }
__device__ __forceinline__ float sinc_(float u)
{
    const float u2 = u * u;
    if (u2 < 0.25f)
        return 1.f + u2 * (-1.f / 6.f + u2 * (1.f / 120.f + u2 * (-1.f / 5040.f + u2 * (1.f / 362880.f))));
    return div_(sinf(u), u);
}
__device__ __forceinline__ float asin_over(float h)
{
    const float h2 = h * h;
    if (h2 < 0.09f)
        return 1.f + h2 * (1.f / 6.f + h2 * (3.f / 40.f + h2 * (5.f / 112.f + h2 * (35.f / 1152.f + h2 * (63.f / 2816.f)))));
    return div_(asinf(h), h);
}
__device__ __forceinline__ double asin_over(double h) { return h > 0.0 ? asin(h) / h : 1.0; }

__device__ __forceinline__ float gfun(float d)
{
    const float d2 = d * d;
    if (d2 < 0.25f)
        return d * (-1.f / 6.f + d2 * (1.f / 120.f + d2 * (-1.f / 5040.f + d2 * (1.f / 362880.f + d2 * (-1.f / 39916800.f)))));
    return div_(sinf(d) - d, d2);
}
// (sin d - d) / d^2; Taylor series below |d| = 0.5 where the direct form cancels
template <typename T> __device__ __forceinline__ T gfun(T d)
{
    if (fabs(d) < T(0.5)) {
        const T d2 = d * d;
        T term = div_(-d, T(6)), sum = T(0);
#pragma unroll
        for (int k = 1; k <= 8; k++) {
            sum += term;
            term *= div_(-d2, T(2 * k + 2) * T(2 * k + 3));
        }
        return sum;
    }
    return div_(T(sin(d)) - d, d * d);
}

// The exact Jacobian of the helix step dx from sin(phi) = s1 with curvature
// coefficient k (curvature k q/pT), applied to the covariance: C <- J C J^T.
// The step's sin(phi) at the end, displacement and arc come with it.
template <typename TS, typename TC>
__device__ __forceinline__ void helix_transport(TC *C, TS s1, TS t, TS c, TS dx, TS k, TS &s2o, TS &dyo,
                                                TS &arco)
{
    const TS cu = k * c;
    const TS s2 = s1 + cu * dx;
    const TS f1 = sqrt(TS(1) - s1 * s1);
    const TS f2 = sqrt(TS(1) - s2 * s2);
    const TS ff = f1 + f2;
    const TS dy = div_(dx * (s1 + s2), ff);
    const TS chord = sqrt(dx * dx + dy * dy);
    const TS h = TS(0.5) * fabs(cu) * chord;
    const TS aoh = asin_over(h);
    const TS arc = (dx >= TS(0) ? chord : -chord) * aoh;
    const TS delta = cu * arc;

    // Jacobian entries (identity elsewhere)
    const TC f12 = TC(f1) * TC(f2);
    const TC a = div_(TC(arc) * sinc_(TC(delta)), f12);                   // dy/ds
    const TC b = div_(TC(k) * sq(TC(dx)), TC(ff)) *
                 (TC(1) + div_(TC(s2) * TC(s1 + s2), TC(f2) * TC(ff)));     // dy/dc
    const TC d = div_(TC(t) * TC(dy), f12);                                 // dz/ds
    const TC e = TC(arc);                                                   // dz/dt
    const TC sh = sinc_(TC(0.5) * TC(delta));
    const TC f = TC(k) * TC(t) * sq(TC(arc)) *
                 ((TC(s2) / TC(f2)) * sh * sh * TC(0.5) + gfun(TC(delta)));  // dz/dc
    const TC gg = TC(k) * TC(dx);                                           // ds/dc
    s2o = s2;
    dyo = dy;
    arco = arc;

    // D = J C (rows y, z, s change)
    const TC D00 = C[YY] + a * C[YS] + b * C[YC];
    const TC D01 = C[YZ] + a * C[ZS] + b * C[ZC];
    const TC D02 = C[YS] + a * C[SS] + b * C[SC];
    const TC D03 = C[YT] + a * C[ST] + b * C[TC_];
    const TC D04 = C[YC] + a * C[SC] + b * C[CC];
    const TC D11 = C[ZZ] + d * C[ZS] + e * C[ZT] + f * C[ZC];
    const TC D12 = C[ZS] + d * C[SS] + e * C[ST] + f * C[SC];
    const TC D13 = C[ZT] + d * C[ST] + e * C[TT] + f * C[TC_];
    const TC D14 = C[ZC] + d * C[SC] + e * C[TC_] + f * C[CC];
    const TC D22 = C[SS] + gg * C[SC];
    const TC D23 = C[ST] + gg * C[TC_];
    const TC D24 = C[SC] + gg * C[CC];
    // C' = D J^T
    C[YY] = D00 + a * D02 + b * D04;
    C[YZ] = D01 + d * D02 + e * D03 + f * D04;
    C[YS] = D02 + gg * D04;
    C[YT] = D03;
    C[YC] = D04;
    C[ZZ] = D11 + d * D12 + e * D13 + f * D14;
    C[ZS] = D12 + gg * D14;
    C[ZT] = D13;
    C[ZC] = D14;
    C[SS] = D22 + gg * D24;
    C[ST] = D23;
    C[SC] = D24;
}

// Field of the map relative to its value on the axis at z = 0, at a point of
// any sector frame (x^2 + y^2 is the squared radius).
template <typename TS> __device__ __forceinline__ TS field_factor(TS x, TS y, TS z, const DevCfg<TS> &g)
{
    return TS(1) + g.fr * (x * x + y * y) + g.fz * z * z;
}

// d(y, z, sin phi)/dx and the field factor at (x, y, z); false if |sin phi| >= 1
template <typename TS>
__device__ __forceinline__ bool rk_deriv(TS x, TS y, TS z, TS s, TS t, TS kc, TS fr, TS fz, TS &dy, TS &dz,
                                         TS &ds, TS &fb)
{
    if (!(fabs(s) < TS(1))) return false;
    const TS rf = TS(1) / sqrt(TS(1) - s * s);
    fb = TS(1) + fr * (x * x + y * y) + fz * z * z;
    dy = s * rf;
    dz = t * rf;
    ds = kc * fb;
    return true;
}

// y += v with the rounding error of the sum carried in e (compensated
// summation: the many small steps of an integration do not lose the last
// bits of the float state)
template <typename TS> __device__ __forceinline__ void acc_add(TS &y, TS &e, TS v)
{
    const TS u = v - e;
    const TS t = y + u;
    e = (t - y) - u;
    y = t;
}

template <typename TS> struct FieldStep {
    TS y, z, s, k;
    int ok;
};

// Step in a field map, state only: classical 4th-order Runge-Kutta
// integration of y' = tan(phi), z' = tan(lambda)/cos(phi), sin(phi)' = k Bz/Bz0
// q/pT over equal x steps of at most `step` (the step count in double, as the
// double path computes it), with compensated sums of the steps.  Also the
// curvature coefficient of the mean of the Runge-Kutta weighted field
// samples, with which the caller transports the covariance.  ok = 0 if
// |sin phi| reaches snp_max.  Kept out of line (scalars in and out) so that
// the uniform-field path keeps its registers.
template <typename TS>
__device__ __noinline__ FieldStep<TS> field_step(TS x1, TS x2, TS y, TS z, TS s, TS t, TS c, TS kcurv, TS fr, TS fz,
                                                 TS snp_max, double step)
{
    FieldStep<TS> r;
    r.ok = 0;
    r.y = y;
    r.z = z;
    r.s = s;
    r.k = kcurv;
    const TS dx = x2 - x1;
    const int ns = (int)ceil(fabs((double)dx) / step);
    const TS h = ns > 0 ? div_(dx, TS(ns)) : TS(0), kc = kcurv * c;
    TS ey = TS(0), ez = TS(0), es = TS(0), fsum = TS(0);
    for (int i = 0; i < ns; i++) {
        const TS xa = x1 + TS(i) * h, xb = (i == ns - 1) ? x2 : x1 + TS(i + 1) * h;
        const TS hs = xb - xa, hh = TS(0.5) * hs, xm = xa + hh;
        TS a1, a2, a3, b1, b2, b3, c1, c2, c3, d1, d2, d3, f1, f2, f3, f4;
        if (!rk_deriv(xa, y, z, s, t, kc, fr, fz, a1, a2, a3, f1)) return r;
        if (!rk_deriv(xm, y + hh * a1, z + hh * a2, s + hh * a3, t, kc, fr, fz, b1, b2, b3, f2)) return r;
        if (!rk_deriv(xm, y + hh * b1, z + hh * b2, s + hh * b3, t, kc, fr, fz, c1, c2, c3, f3)) return r;
        if (!rk_deriv(xb, y + hs * c1, z + hs * c2, s + hs * c3, t, kc, fr, fz, d1, d2, d3, f4)) return r;
        const TS w = hs * TS(1.0 / 6.0);
        acc_add(y, ey, w * (a1 + TS(2) * b1 + TS(2) * c1 + d1));
        acc_add(z, ez, w * (a2 + TS(2) * b2 + TS(2) * c2 + d2));
        acc_add(s, es, w * (a3 + TS(2) * b3 + TS(2) * c3 + d3));
        fsum += (f1 + TS(2) * f2 + TS(2) * f3 + f4) * TS(1.0 / 6.0);
        if (!(fabs(s) < snp_max)) return r;
    }
    r.y = y;
    r.z = z;
    r.s = s;
    r.k = ns > 0 ? kcurv * div_(fsum, TS(ns)) : kcurv;
    r.ok = 1;
    return r;
}

// Helix step in the sector frame from T.x to x2, with the exact Jacobian
// applied to the covariance (in a field map: the state from field_step, the
// covariance with the helix in its mean field).  False (state untouched) if
// |sin phi| would reach snp_max.
template <typename TS, typename TC>
__device__ __forceinline__ bool propagate(Trk<TS, TC> &T, TS x2, const DevCfg<TS> &g)
{
    const TS dx = x2 - T.x;
    TS k = g.k_curv;
    FieldStep<TS> fs;
    if (g.field_on) {
        fs = field_step(T.x, x2, T.y, T.z, T.s, T.t, T.c, g.k_curv, g.fr, g.fz, g.snp_max, g.field_step);
        if (!fs.ok) return false;
        k = fs.k;
        if (!(fabs(T.s + k * T.c * dx) < TS(1))) return false;
    } else if (!(fabs(T.s + k * T.c * dx) < g.snp_max)) {
        return false;
    }
    TS s2, dy, arc;
    helix_transport(T.C, T.s, T.t, T.c, dx, k, s2, dy, arc);
    if (g.field_on) {
        T.y = fs.y;
        T.z = fs.z;
        T.s = fs.s;
    } else {
        T.y += dy;
        T.z += T.t * arc;
        T.s = s2;
    }
    T.x = x2;
    return true;
}

// Change of sector frame by +-20 degrees at the current point.
template <typename TS, typename TC>
__device__ __forceinline__ bool rotate(Trk<TS, TC> &T, bool up, const DevCfg<TS> &g)
{
    const TS ca = g.cos_sector, sa = up ? g.sin_sector : -g.sin_sector;
    const TS s = T.s, f = sqrt(TS(1) - s * s);
    const TS s1 = s * ca - f * sa;
    const TS f1 = f * ca + s * sa;
    if (!(f1 > TS(0))) return false;
    const TS x1 = T.x * ca + T.y * sa;
    const TS y1 = -T.x * sa + T.y * ca;
    const TC A = div_(TC(f), TC(f1));
    const TC B = div_(-TC(sa) * TC(T.t), TC(f1));
    const TS kf = g.field_on ? g.k_curv * field_factor(T.x, T.y, T.z, g) : g.k_curv;
    const TC Cc = -TC(kf) * TC(T.c) * TC(sa);
    const TC Dd = div_(TC(f1), TC(f));
    T.y = y1;
    T.s = s1;
    T.x = x1;
    TC *C = T.C;
    const TC c00 = C[YY], c01 = C[YZ], c02 = C[YS], c03 = C[YT], c04 = C[YC];
    const TC D10 = c01 + B * c00, D12 = C[ZS] + B * c02;
    const TC D20 = Cc * c00 + Dd * c02, D22 = Cc * c02 + Dd * C[SS];
    C[YY] = A * A * c00;
    C[YZ] = A * c01 + B * A * c00;
    C[YS] = Cc * A * c00 + Dd * A * c02;
    C[YT] = A * c03;
    C[YC] = A * c04;
    C[ZZ] = (C[ZZ] + B * c01) + B * D10;
    C[ZS] = Cc * D10 + Dd * D12;
    C[ZT] = C[ZT] + B * c03;
    C[ZC] = C[ZC] + B * c04;
    C[SS] = Cc * D20 + Dd * D22;
    C[ST] = Cc * c03 + Dd * C[ST];
    C[SC] = Cc * c04 + Dd * C[SC];
    return true;
}

// Thin scatterer (Highland width) at the current point.
template <typename TS, typename TC>
__device__ __forceinline__ void add_ms(Trk<TS, TC> &T, const DevCfg<TS> &g)
{
    const TC c = TC(T.c), t = TC(T.t), s = TC(T.s);
    if (c == TC(0) || !(g.x_over_x0 > TS(0))) return;
    const TC f = sqrt(TC(1) - s * s);
    const TC tt = TC(1) + t * t;
    const TC pp = div_(TC(sqrt(tt)), TC(fabs(c)));
    // beta p = p / sqrt(1 + m^2 / p^2), which stays finite where p^2 would overflow
    const TC pbeta = div_(pp, TC(sqrt(TC(1) + div_(TC(g.mass2), pp * pp))));
    const TC xi = div_(TC(g.x_over_x0) * TC(sqrt(tt)), f);
    const TC th0 = div_(TC(0.0136), pbeta) * sqrt(xi) * (TC(1) + TC(0.038) * log(xi));
    const TC th2 = th0 * th0;
    T.C[SS] += th2 * f * f * tt;
    T.C[TT] += th2 * tt * tt;
    T.C[CC] += th2 * c * c * t * t;
    T.C[TC_] += th2 * tt * c * t;
}

// Mean energy loss of the layer's material at the current point (Bethe
// formula without density or shell terms; rate at the momentum before the
// loss; path = thickness / (cos lambda cos phi)).  Outward the energy falls
// by it, inward (the refit) it is given back.  q/pT scales by p/p', its
// covariance row by (p/p')^3 E'/E (the loss held fixed).  False (state
// untouched): the energy would not exceed the mass.
template <typename TS, typename TC>
__device__ __forceinline__ bool eloss(Trk<TS, TC> &T, const DevCfg<TS> &g, bool outward)
{
    const TS c = T.c;
    if (!(g.eloss_xrho > TS(0)) || c == TS(0)) return true;
    const TS s = T.s, t = T.t;
    const TS f = sqrt(TS(1) - s * s), tt = TS(1) + t * t;
    const TS p2 = div_(tt, c * c);
    if (!(p2 < TS(1e30))) return true;  // |p| beyond 1e15 GeV: no loss worth a digit
    const TS e2 = p2 + g.mass2;
    const TS e = sqrt(e2), p = sqrt(p2);
    const TS bg2 = div_(p2, g.mass2), b2 = div_(p2, e2), gam = div_(e, g.mass), r = g.me_over_m;
    const TS wmax = TS(2 * 0.51099895e-3) * bg2 / (TS(1) + TS(2) * gam * r + r * r);
    TS rate = div_(g.eloss_kza, b2) * (TS(0.5) * log(TS(2 * 0.51099895e-3) * bg2 * wmax * g.inv_i2) - b2);
    rate = rate > TS(0) ? rate : TS(0);
    const TS de = rate * g.eloss_xrho * div_(sqrt(tt), f);
    const TS e1 = outward ? e - de : e + de;
    if (!(e1 > g.mass)) return false;
    const TS p1 = sqrt(e1 * e1 - g.mass2);
    const TS k = div_(p, p1);
    const TC j = TC(k) * TC(k) * TC(k) * TC(div_(e1, e));
    T.c = c * k;
    T.C[YC] *= j;
    T.C[ZC] *= j;
    T.C[SC] *= j;
    T.C[TC_] *= j;
    T.C[CC] *= j * j;
    return true;
}

// Whether the point (sector, z) of layer l lies in a chamber slot without a
// chamber (outside the stacks in z: no).
template <typename TS>
__device__ __forceinline__ bool absent_at(const DevCfg<TS> &g, int sec, int l, TS z)
{
    const TS row = floor(div_(z - g.z_min, g.pad_len));
    if (!(row >= TS(0)) || row >= TS(kStacks * g.bin.n_rows)) return false;
    return slot_absent(g.bin, sec * (kStacks * kLayers) + ((int)row / g.bin.n_rows) * kLayers + l);
}

template <typename T> __device__ __forceinline__ T cget(const T *C, int i, int j)
{
    // symmetric access into the packed upper triangle
    const int a = i < j ? i : j, b = i < j ? j : i;
    const int off = a * 5 - (a * (a - 1)) / 2 + (b - a);
    return C[off];
}

// positive definiteness of the packed covariance: all LDL^T pivots > 0
template <typename TC> __device__ __forceinline__ bool ldl_pd(const TC *C)
{
    TC L[5][5], dd[5];
#pragma unroll
    for (int j = 0; j < 5; j++) {
        TC v = cget(C, j, j);
#pragma unroll
        for (int k2 = 0; k2 < j; k2++) v -= L[j][k2] * L[j][k2] * dd[k2];
        if (!(v > TC(0))) return false;
        dd[j] = v;
#pragma unroll
        for (int i = j + 1; i < 5; i++) {
            TC w = cget(C, i, j);
#pragma unroll
            for (int k2 = 0; k2 < j; k2++) w -= L[i][k2] * L[j][k2] * dd[k2];
            L[i][j] = w / v;  // IEEE division: the check's decisions are those of plain float
        }
    }
    return true;
}

// Joseph-form update with h(p) = (y + tau (z - z_tkl), z); returns false if
// the updated covariance is not positive definite (LDL^T pivots).
template <typename TS, typename TC>
__device__ __forceinline__ bool kalman_update(Trk<TS, TC> &T, TS ry, TS rz, TS tau, TC vy, TC vz)
{
    TC *C = T.C;
    const TC tc = TC(tau);
    TC H0[5], H1[5];  // C H^T columns
#pragma unroll
    for (int i = 0; i < 5; i++) {
        H0[i] = cget(C, i, 0) + tc * cget(C, i, 1);
        H1[i] = cget(C, i, 1);
    }
    const TC S00 = H0[0] + tc * H0[1] + vy;
    const TC S01 = H1[0] + tc * H1[1];
    const TC S11 = H1[1] + vz;
    const TC det = S00 * S11 - S01 * S01;
    const TC i00 = div_(S11, det), i01 = div_(-S01, det), i11 = div_(S00, det);
    TC K0[5], K1[5];
#pragma unroll
    for (int i = 0; i < 5; i++) {
        K0[i] = H0[i] * i00 + H1[i] * i01;
        K1[i] = H0[i] * i01 + H1[i] * i11;
    }
    T.y += TS(K0[0] * TC(ry) + K1[0] * TC(rz));
    T.z += TS(K0[1] * TC(ry) + K1[1] * TC(rz));
    T.s += TS(K0[2] * TC(ry) + K1[2] * TC(rz));
    T.t += TS(K0[3] * TC(ry) + K1[3] * TC(rz));
    T.c += TS(K0[4] * TC(ry) + K1[4] * TC(rz));
    // B = (I - K H) C
    TC B[5][5];
#pragma unroll
    for (int i = 0; i < 5; i++)
#pragma unroll
        for (int j = 0; j < 5; j++) B[i][j] = cget(C, i, j) - K0[i] * H0[j] - K1[i] * H1[j];
    // C' = B (I - K H)^T + K V K^T
    TC Bh0[5];
#pragma unroll
    for (int i = 0; i < 5; i++) Bh0[i] = B[i][0] + tc * B[i][1];
    int o = 0;
#pragma unroll
    for (int i = 0; i < 5; i++)
#pragma unroll
        for (int j = i; j < 5; j++) {
            C[o++] = B[i][j] - Bh0[i] * K0[j] - B[i][1] * K1[j] + vy * K0[i] * K0[j] +
                     vz * K1[i] * K1[j];
        }
    return ldl_pd(C);
}

template <typename TS> __device__ __forceinline__ TS poly2(const TS *a, TS s)
{
    return a[0] + a[1] * s + a[2] * s * s;
}

// bin of a window edge among n bins starting at lo, clamped; NaN maps to
// bin 0 (never out of range)
__device__ __forceinline__ int bin_of(double v, double lo, double inv_w, int n)
{
    const double u = floor((v - lo) * inv_w);
    if (!(u >= 0.0)) return 0;
    return u > (double)(n - 1) ? n - 1 : (int)u;
}

// global pad-row index of a z window edge, clamped to [0, nrt - 1]
template <typename TS> __device__ __forceinline__ int zrow(TS z, const DevCfg<TS> &g, int nrt)
{
    const TS u = floor((z - g.z_min) * g.inv_pad);
    if (!(u >= TS(0))) return 0;
    return u > TS(nrt - 1) ? nrt - 1 : (int)u;
}


// ---------------------------------------------------------------------------
// per-track phases shared by the kernels
// ---------------------------------------------------------------------------

// Search road of one track at one layer.
template <typename TS>
struct Road {
    TS y, z, tphi, tz, tau, Ry, Rz, gdy, dytrk, si00, si01, si11;
    int glo, ghi;  // global pad-row range (glo > ghi: nothing to search)
    int yb0, yb1;  // y-bin range
    int db0, db1;  // deflection-bin range
    int gdet0;     // key-space chamber of stack 0: group * 540 + sector * 30 + layer
    int sdet0;     // misalignment-table chamber of stack 0: sector * 30 + layer
};

// Best candidate so far: lexicographic minimum of (chi2, input index).
template <typename TS>
struct Best {
    TS chi2;
    int idx;    // input-order tracklet index, INT_MAX if none
    int stack;  // stack of its chamber
    float y, z; // its measurement

    // keeps a passing candidate if it is the lexicographic (chi2, index) minimum
    // (bitwise, not short-circuit, logic: no branches in the record loop)
    __device__ __forceinline__ void offer(TS c, int oj, float yy, float zz, int st, bool pass)
    {
        const bool take = pass & ((c < chi2) | ((c == chi2) & (oj < idx)));
        chi2 = take ? c : chi2;
        idx = take ? oj : idx;
        stack = take ? st : stack;
        y = take ? yy : y;
        z = take ? zz : z;
    }
};

template <typename TS> __device__ __forceinline__ Best<TS> no_best()
{
    Best<TS> b;
    b.chi2 = TS(INFINITY);
    b.idx = 0x7fffffff;
    b.stack = 0;
    b.y = 0.f;
    b.z = 0.f;
    return b;
}

template <typename TS> __device__ __forceinline__ bool better(TS c, int i, const Best<TS> &b)
{
    return c < b.chi2 || (c == b.chi2 && i < b.idx);
}

// Load one seed and validate it.  0: live, 1: rejected (copied through),
// 2: the float covariance is not positive definite (queue for the re-run).
template <typename TS, typename TC, bool kQueueNotPD>
__device__ __forceinline__ int load_track(const DevCfg<TS> &g, const MatchIO &io, int64_t i,
                                          Trk<TS, TC> &T, int &grp)
{
    if (io.rows_in) {
        const TS *r = reinterpret_cast<const TS *>(io.rows_in) + i * kRowIn;
        T.y = r[0];
        T.z = r[1];
        T.s = r[2];
        T.t = r[3];
        T.c = r[4];
#pragma unroll
        for (int k = 0; k < 15; k++) T.C[k] = TC(r[5 + k]);
        T.x = r[20];
        T.sec = int_of(r[21]);
        grp = int_of(r[22]);
    } else {
        const int64_t n = io.n;
        const TS *ip = reinterpret_cast<const TS *>(io.ip);
        const TS *ic = reinterpret_cast<const TS *>(io.ic);
        const TS *ix = reinterpret_cast<const TS *>(io.ix);
        T.y = ip[i];
        T.z = ip[n + i];
        T.s = ip[2 * n + i];
        T.t = ip[3 * n + i];
        T.c = ip[4 * n + i];
        T.x = ix[i];
#pragma unroll
        for (int k = 0; k < 15; k++) T.C[k] = TC(ic[k * n + i]);
        T.sec = io.isec[i];
        grp = io.igrp ? io.igrp[i] : 0;
    }
    bool bad = !(__builtin_isfinite(T.x) && T.sec >= 0 && T.sec < kSectors && grp >= 0 &&
                 grp < g.bin.n_groups);
    bad |= !(__builtin_isfinite(T.y) && __builtin_isfinite(T.z) && __builtin_isfinite(T.s) &&
             __builtin_isfinite(T.t) && __builtin_isfinite(T.c));
#pragma unroll
    for (int k = 0; k < 15; k++) bad |= !__builtin_isfinite(T.C[k]);
    if (!bad) bad = !(fabs(T.s) < g.snp_max);
    if (!bad && !ldl_pd(T.C)) {
        if (kQueueNotPD) return 2;  // positive definite in double is decided by the re-run
        bad = true;
    }
    if (kQueueNotPD && io.force_fallback) return 2;
    return bad ? 1 : 0;
}

// Propagation to the layer plane and sector hops (predict adds the layer's
// scattering).  False: the track stopped (status set).
template <typename TS, typename TC>
__device__ __forceinline__ bool reach_plane(Trk<TS, TC> &T, int l, const DevCfg<TS> &g, uint32_t &status)
{
    const TS xl = g.x_layer[l];
    if (!propagate(T, xl, g)) {
        status |= kStopSnp;
        return false;
    }
    for (int nrot = 0;; nrot++) {
        if (fabs(T.y) <= xl * g.tan_half_sector) break;
        if (nrot == 2) {
            status |= kRotFail;
            return false;
        }
        const bool up = T.y > TS(0);
        if (!rotate(T, up, g)) {
            status |= kRotFail;
            return false;
        }
        T.sec = up ? (T.sec == kSectors - 1 ? 0 : T.sec + 1) : (T.sec == 0 ? kSectors - 1 : T.sec - 1);
        if (!propagate(T, xl, g)) {
            status |= kStopSnp;
            return false;
        }
    }
    return true;
}

template <typename TS, typename TC>
__device__ __forceinline__ bool predict(Trk<TS, TC> &T, int l, const DevCfg<TS> &g, uint32_t &status)
{
    if (!reach_plane(T, l, g, status)) return false;
    add_ms(T, g);
    if (!eloss(T, g, true)) {
        status |= kStopped;
        return false;
    }
    return true;
}

// Covariance road at layer l.  False: nothing to search (out of the
// chambers in z, or no positive definite innovation covariance).
template <typename TS, typename TC>
__device__ __forceinline__ bool open_road(const Trk<TS, TC> &T, int l, int grp, const DevCfg<TS> &g,
                                          uint32_t &status, Road<TS> &R)
{
    const TS tau = g.tilt[l];
    const TS f = sqrt(TS(1) - T.s * T.s);
    R.y = T.y;
    R.z = T.z;
    R.tau = tau;
    R.tphi = div_(T.s, f);
    R.tz = div_(T.t, f);
    const TS sy = poly2(g.sigma_y, T.s);
    const TC vy = TC(sy) * TC(sy);
    const TC Syy = T.C[YY] + TC(2) * TC(tau) * T.C[YZ] + TC(tau) * TC(tau) * T.C[ZZ] + vy;
    const TC Syz = T.C[YZ] + TC(tau) * T.C[ZZ];
    const TC Szz = T.C[ZZ] + TC(g.vz);
    const TC det = Syy * Szz - Syz * Syz;
    R.glo = 1;
    R.ghi = 0;
    if (!(Syy > TC(0) && Szz > TC(0) && det > TC(0))) {
        status |= kNotPD;
        return false;
    }
    R.si00 = TS(div_(Szz, det));
    R.si01 = TS(div_(-Syz, det));
    R.si11 = TS(div_(Syy, det));
    R.Ry = g.n_sigma_road * TS(sqrt(Syy));
    R.Rz = g.n_sigma_road * TS(sqrt(Szz));
    R.dytrk = g.drift_len * (R.tphi - g.tan_psi);
    const TS sdy = poly2(g.sigma_dy, T.s);
    const TS f3 = f * f * f;
    R.gdy = g.n_sigma_dy *
            TS(sqrt(TC(sdy) * TC(sdy) + div_(TC(g.drift_len) * TC(g.drift_len) * T.C[SS], TC(f3) * TC(f3))));
    const TS mz = g.dx_max * fabs(R.tz);
    if (T.z + R.Rz + mz < g.z_min || T.z - R.Rz - mz > g.z_max) {
        status |= kOutOfZ;
        return false;
    }
    // cells overlapping the road; the slack keeps the set a superset of the
    // gate's acceptance under rounding
    const TS slack_y = TS(1e-3) + TS(1e-5) * R.Ry, slack_z = TS(1e-3) + TS(1e-5) * R.Rz;
    const TS my = fabs(tau) * (R.Rz + mz + slack_z) + g.dx_max * fabs(R.tphi);
    const int nrt = kStacks * g.bin.n_rows;
    R.glo = zrow(T.z - R.Rz - mz - slack_z, g, nrt);
    R.ghi = zrow(T.z + R.Rz + mz + slack_z, g, nrt);
    R.yb0 = bin_of((double)(T.y - R.Ry - my - slack_y), g.bin.y_min, g.bin.inv_w, g.bin.n_yb);
    R.yb1 = bin_of((double)(T.y + R.Ry + my + slack_y), g.bin.y_min, g.bin.inv_w, g.bin.n_yb);
    const TS slack_d = TS(1e-4) + TS(1e-4) * R.gdy;
    R.db0 = bin_of((double)(R.dytrk - R.gdy - slack_d), g.bin.dy_min, g.bin.inv_wd, g.bin.n_db);
    R.db1 = bin_of((double)(R.dytrk + R.gdy + slack_d), g.bin.dy_min, g.bin.inv_wd, g.bin.n_db);
    R.sdet0 = T.sec * (kStacks * kLayers) + l;
    R.gdet0 = grp * kDet + R.sdet0;
    return true;
}

// Gates of one candidate record; chi2 valid when *pass.
template <typename TS>
__device__ __forceinline__ TS cand_chi2(const Road<TS> &R, TS ye, TS ze, const float4 &r, TS chi2_max,
                                        bool &pass)
{
    const TS ddy = TS(r.y) - R.dytrk;
    const TS zj = TS(r.z);
    const TS rz = zj - ze;
    // y of the track at the tracklet's z along the tilted pad: ye + tau (ze - zj)
    const TS ry = TS(r.x) - (ye - R.tau * rz);
    const TS chi2 = R.si00 * ry * ry + TS(2) * R.si01 * ry * rz + R.si11 * rz * rz;
    pass = fabs(ddy) <= R.gdy && fabs(rz) <= R.Rz && fabs(ry) <= R.Ry && chi2 <= chi2_max;
    return chi2;
}

// The road as record ranges: one per (stack, dy bin, y bin), each holding the
// road's pad rows of that stack (rows are innermost in the cell key).
struct RangeGrid {
    int s0, nd, ny, n;  // first stack, dy bins, y bins, number of ranges
};

template <typename TS>
__device__ __forceinline__ RangeGrid range_grid(const Road<TS> &R, int nr)
{
    RangeGrid q;
    q.s0 = R.glo / nr;
    q.nd = R.db1 - R.db0 + 1;
    q.ny = R.yb1 - R.yb0 + 1;
    q.n = (R.glo <= R.ghi) ? (R.ghi / nr - q.s0 + 1) * q.nd * q.ny : 0;
    return q;
}

// cell-offset bounds of range (is, id, iy): [*a, *b)
template <typename TS>
__device__ __forceinline__ void range_bounds(const Road<TS> &R, const DevCfg<TS> &g, const MatchIO &io,
                                             int st, int id, int iy, uint32_t *a, uint32_t *b)
{
    const int nr = g.bin.n_rows;
    int r0 = R.glo - st * nr, r1 = R.ghi - st * nr;
    r0 = r0 < 0 ? 0 : r0;
    r1 = r1 > nr - 1 ? nr - 1 : r1;
    const uint32_t base = ((((uint32_t)(R.gdet0 + st * kLayers)) * (uint32_t)g.bin.n_db +
                           (uint32_t)(R.db0 + id)) * (uint32_t)g.bin.n_yb + (uint32_t)(R.yb0 + iy)) *
                          (uint32_t)nr;
    *a = io.offsets[base + r0];
    *b = io.offsets[base + r1 + 1];
}

// Gate and keep the best of the records [a, b) of one stack's chamber.
template <typename TS>
__device__ __forceinline__ void scan_range(const Road<TS> &R, const DevCfg<TS> &g, const MatchIO &io,
                                           uint32_t a, uint32_t b, int st, Best<TS> &B)
{
    constexpr int kUnroll = 2;
    TS ye = R.y, ze = R.z;
    if (g.dx_max != TS(0)) {
        const TS dxd = g.dx[R.sdet0 + st * kLayers];
        ye = R.y + dxd * R.tphi;
        ze = R.z + dxd * R.tz;
    }
    for (uint32_t k0 = a; k0 < b; k0 += kUnroll) {
        float4 rec[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; u++)
            if (k0 + u < b) rec[u] = io.sorted[k0 + u];
#pragma unroll
        for (int u = 0; u < kUnroll; u++) {
            const uint32_t k = k0 + (uint32_t)u;
            if (k < b) {
                bool pass;
                const TS c = cand_chi2(R, ye, ze, rec[u], g.chi2_max, pass);
                const int oj = __float_as_int(rec[u].w);
                const bool take = pass && better(c, oj, B);
                B.chi2 = take ? c : B.chi2;
                B.idx = take ? oj : B.idx;
                B.stack = take ? st : B.stack;
                B.y = take ? rec[u].x : B.y;
                B.z = take ? rec[u].z : B.z;
            }
        }
    }
}

// One lane walks a whole road: the bounds of up to kBatch ranges are fetched
// in one memory round trip, then their records are gated.
template <typename TS>
__device__ __forceinline__ void scan_road_lane(const Road<TS> &R, const DevCfg<TS> &g, const MatchIO &io,
                                               Best<TS> &B)
{
    constexpr int kBatch = 4;
    const RangeGrid q = range_grid(R, g.bin.n_rows);
    int is = 0, id = 0, iy = 0;
    for (int j0 = 0; j0 < q.n; j0 += kBatch) {
        uint32_t a[kBatch], b[kBatch];
        int st[kBatch];
#pragma unroll
        for (int u = 0; u < kBatch; u++) {
            a[u] = 0;
            b[u] = 0;
            st[u] = q.s0 + is;
            if (j0 + u < q.n) {
                range_bounds(R, g, io, st[u], id, iy, &a[u], &b[u]);
                if (++iy == q.ny) {
                    iy = 0;
                    if (++id == q.nd) {
                        id = 0;
                        ++is;
                    }
                }
            }
        }
#pragma unroll
        for (int u = 0; u < kBatch; u++)
            if (a[u] < b[u]) scan_range(R, g, io, a[u], b[u], st[u], B);
    }
}

// Gate one record of stack st (its chamber shifted by dxd in x) and offer it
// to the accumulator unless `in` is false.
template <typename TS, typename A>
__device__ __forceinline__ void gate_record(const Road<TS> &R, const DevCfg<TS> &g, const float4 &rec,
                                            int st, TS dxd, bool in, A &acc)
{
    const TS ye = R.y + dxd * R.tphi, ze = R.z + dxd * R.tz;
    bool pass;
    const TS c = cand_chi2(R, ye, ze, rec, g.chi2_max, pass);
    acc.offer(c, __float_as_int(rec.w), rec.x, rec.z, st, pass & in);
}

// One lane walks a whole road with its records flattened: the bounds of up
// to kBatch ranges come in one memory round trip, then their records are
// taken kU at a time across range boundaries, so a round trip fetches kU
// records however the road's candidates fall into cells.  (One walk for
// shifted and unshifted chambers: a second copy specialised for chambers
// without shifts made the kernel 3-7 % slower.)
template <typename TS, typename A>
__device__ __forceinline__ void scan_road_flat(const Road<TS> &R, const DevCfg<TS> &g, const MatchIO &io,
                                               A &B)
{
    constexpr int kBatch = 4, kU = 4;
    const int nr = g.bin.n_rows;
    const RangeGrid q = range_grid(R, nr);
    const bool shifted = g.dx_max != TS(0);
    // Cell index of the first pad row of range (is, id, iy), kept as a running
    // sum: one y bin further adds sy, the next dy bin (y back to the first)
    // adds sy + wy, the next stack (dy and y back to the first) adds ws on top
    // (additions only: no integer multiplies per range).
    const uint32_t sy = (uint32_t)nr, sd = (uint32_t)g.bin.n_yb * sy, ss = (uint32_t)(kLayers * g.bin.n_db) * sd;
    const uint32_t wy = sd - (uint32_t)q.ny * sy, ws = ss - (uint32_t)q.nd * sd;
    uint32_t cur = ((((uint32_t)(R.gdet0 + q.s0 * kLayers)) * (uint32_t)g.bin.n_db + (uint32_t)R.db0) *
                        (uint32_t)g.bin.n_yb + (uint32_t)R.yb0) * sy;
    int is = 0, id = 0, iy = 0, so = q.s0 * nr;
    for (int j0 = 0; j0 < q.n; j0 += kBatch) {
        uint32_t a[kBatch], e[kBatch];
        int st[kBatch];
#pragma unroll
        for (int u = 0; u < kBatch; u++) {
            a[u] = 0;
            e[u] = 0;
            st[u] = q.s0 + is;
            if (j0 + u < q.n) {
                // the road's pad rows within this stack
                const int r0 = max(R.glo - so, 0), r1 = min(R.ghi - so, nr - 1);
                a[u] = io.offsets[cur + (uint32_t)r0];
                e[u] = io.offsets[cur + (uint32_t)r1 + 1u];
                cur += sy;
                if (++iy == q.ny) {
                    iy = 0;
                    cur += wy;
                    if (++id == q.nd) {
                        id = 0;
                        cur += ws;
                        ++is;
                        so += nr;
                    }
                }
            }
        }
        // running record counts at the range starts
        uint32_t pre[kBatch + 1];
        pre[0] = 0;
#pragma unroll
        for (int u = 0; u < kBatch; u++) pre[u + 1] = pre[u] + (e[u] > a[u] ? e[u] - a[u] : 0u);
        const uint32_t tot = pre[kBatch];
        for (uint32_t f0 = 0; f0 < tot; f0 += kU) {
            float4 rec[kU];
            int su[kU];
            bool in[kU];
            TS dxd[kU];
#pragma unroll
            for (int u = 0; u < kU; u++) {
                // past the end: the batch's last record again, offered as failing
                in[u] = f0 + (uint32_t)u < tot;
                const uint32_t f = in[u] ? f0 + (uint32_t)u : tot - 1u;
                // the range holding flat position f: the last one starting at or before it
                uint32_t k = a[0] + f;
                su[u] = st[0];
#pragma unroll
                for (int q = 1; q < kBatch; q++) {
                    const bool past = f >= pre[q];
                    k = past ? a[q] + (f - pre[q]) : k;
                    su[u] = past ? st[q] : su[u];
                }
                rec[u] = io.sorted[k];
                dxd[u] = TS(0);
                if (shifted) dxd[u] = g.dx[R.sdet0 + su[u] * kLayers];
            }
#pragma unroll
            for (int u = 0; u < kU; u++) gate_record(R, g, rec[u], su[u], dxd[u], in[u], B);
        }
    }
}

// G lanes share a road: lane `sub` takes every G-th range.
template <int G, typename TS>
__device__ __forceinline__ void scan_road_group(const Road<TS> &R, int sub, const DevCfg<TS> &g,
                                                const MatchIO &io, Best<TS> &B)
{
    const RangeGrid q = range_grid(R, g.bin.n_rows);
    const int per_stack = q.nd * q.ny;
    for (int j = sub; j < q.n; j += G) {
        const int is = j / per_stack, rem = j - is * per_stack;
        const int id = rem / q.ny, iy = rem - id * q.ny;
        uint32_t a, b;
        range_bounds(R, g, io, q.s0 + is, id, iy, &a, &b);
        scan_range(R, g, io, a, b, q.s0 + is, B);
    }
}

// Per-track results accumulated over the layers (the per-layer index and
// chi2 go straight to the output arrays).
template <typename TS>
struct Acc {
    int nmatch;
    TS chi2sum;
    int lidx;   // this layer's match, -1 if none
    TS lchi;    // its chi2
};

// Precise propagation to the winner's radius and the Kalman update.
// 0: matched, 1: the track stopped, 2: covariance lost positive definiteness
// (the update is kept and NOT_PD set unless the caller re-runs the track).
template <typename TS, typename TC>
__device__ __forceinline__ int apply_best(Trk<TS, TC> &T, int l, const Road<TS> &R, const Best<TS> &B,
                                          const DevCfg<TS> &g, const MatchIO &io, uint32_t &status,
                                          Acc<TS> &acc)
{
    const TS yj = TS(B.y), zj = TS(B.z);
    const TS bdx = g.dx[R.sdet0 + B.stack * kLayers];
    if (bdx != TS(0)) {
        if (!propagate(T, g.x_layer[l] + bdx, g)) {
            status |= kStopSnp;
            return 1;
        }
    }
    const TS ry = yj - (T.y + R.tau * (T.z - zj));
    const TS rz = zj - T.z;
    const TS syu = poly2(g.sigma_y, T.s);
    int rc = 0;
    if (!kalman_update(T, ry, rz, R.tau, TC(syu) * TC(syu), TC(g.vz))) {
        status |= kNotPD;
        rc = 2;
    }
    acc.lidx = B.idx;
    acc.nmatch++;
    acc.chi2sum += B.chi2;
    acc.lchi = B.chi2;
    if (!(fabs(T.s) < g.snp_max)) {
        status |= kStopSnp;
        return rc == 2 ? 2 : 1;
    }
    return rc;
}

template <typename TS>
__device__ __forceinline__ void write_layer(const MatchIO &io, int64_t i, int l, const Acc<TS> &acc)
{
    if (io.rows_out) {
        TS *r = reinterpret_cast<TS *>(io.rows_out) + i * io.row_out;
        r[25 + l] = as_row(acc.lidx, TS());
        if (io.ochi2l) r[kRowChi2 + l] = acc.lchi;
        return;
    }
    io.oidx[l * io.n + i] = acc.lidx;
    if (io.ochi2l) reinterpret_cast<TS *>(io.ochi2l)[l * io.n + i] = acc.lchi;
}

template <typename TS, typename TC>
__device__ __forceinline__ void write_track(const MatchIO &io, int64_t i, const Trk<TS, TC> &T,
                                            const Acc<TS> &acc, uint32_t status)
{
    if (io.rows_out) {
        TS *r = reinterpret_cast<TS *>(io.rows_out) + i * io.row_out;
        r[0] = T.y;
        r[1] = T.z;
        r[2] = T.s;
        r[3] = T.t;
        r[4] = T.c;
#pragma unroll
        for (int k = 0; k < 15; k++) r[5 + k] = TS(T.C[k]);
        r[20] = T.x;
        r[21] = acc.chi2sum;
        r[22] = as_row(T.sec, TS());
        r[23] = as_row(acc.nmatch, TS());
        r[24] = as_row((int)status, TS());
        return;
    }
    const int64_t n = io.n;
    TS *op = reinterpret_cast<TS *>(io.op);
    TS *oc = reinterpret_cast<TS *>(io.oc);
    TS *ox = reinterpret_cast<TS *>(io.ox);
    TS *och = reinterpret_cast<TS *>(io.ochi2);
    op[i] = T.y;
    op[n + i] = T.z;
    op[2 * n + i] = T.s;
    op[3 * n + i] = T.t;
    op[4 * n + i] = T.c;
#pragma unroll
    for (int k = 0; k < 15; k++) oc[k * n + i] = TS(T.C[k]);
    ox[i] = T.x;
    io.osec[i] = T.sec;
    och[i] = acc.chi2sum;
    io.onm[i] = acc.nmatch;
    io.ost[i] = status;
}

template <typename TS> __device__ __forceinline__ void acc_init(Acc<TS> &acc)
{
    acc.nmatch = 0;
    acc.chi2sum = TS(0);
    acc.lidx = -1;
    acc.lchi = TS(0);
}

// One track, one lane, start to end.  Returns false if the track must be
// re-run with a double covariance (kQueueNotPD only).
template <typename TS, typename TC, bool kQueueNotPD>
__device__ __forceinline__ bool match_lane(const DevCfg<TS> &g, const MatchIO &io, int64_t i,
                                           uint32_t status)
{
    Trk<TS, TC> T;
    int grp;
    const int ld = load_track<TS, TC, kQueueNotPD>(g, io, i, T, grp);
    if (ld == 2) return false;
    Acc<TS> acc;
    acc_init(acc);
    bool live = ld == 0;
    if (ld == 1) status |= kBadInput;
    for (int l = 0; l < kLayers; l++) {
        acc.lidx = -1;
        acc.lchi = TS(0);
        Road<TS> R;
        if (live && !predict(T, l, g, status)) live = false;
        if (live && open_road(T, l, grp, g, status, R)) {
            Best<TS> B = no_best<TS>();
            scan_road_flat(R, g, io, B);
            if (B.idx != 0x7fffffff) {
                const int rc = apply_best(T, l, R, B, g, io, status, acc);
                if (rc == 2 && kQueueNotPD) return false;
                if (rc != 0 && (status & kStopSnp)) live = false;
            }
        } else if (kQueueNotPD && (status & kNotPD)) {
            return false;  // the float innovation covariance is not positive definite
        }
        write_layer(io, i, l, acc);
    }
    write_track(io, i, T, acc, status);
    return true;
}

// Workgroups are dispatched round-robin over the 8 XCDs (workgroup b to XCD
// b mod 8), each with its own L2.  Renumbering them so that XCD x runs the
// x-th contiguous eighth of the tracks keeps neighbouring tracks (in the
// spatial order: neighbouring cells) on one L2.  A bijection on
// [0, gridDim.x) for any grid size.
__device__ __forceinline__ unsigned xcd_block()
{
    const unsigned nb = gridDim.x, b = blockIdx.x, q = nb / 8, r = nb % 8, x = b % 8, k = b / 8;
    return (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + k;
}

// Waves per SIMD the one-lane kernels are compiled for.  Float state and
// covariance: four (at most 128 registers; the road scan is latency bound, so
// the extra waves in flight are worth a few spilled registers; the
// several-hypotheses kernel takes four too: 2.06 -> 1.40 ms on the 450k
// batch with four hypotheses).  Float state with a double covariance: three
// (0.56 -> 0.49 ms).  Double state: two (256 registers and a few spilled;
// left to itself the compiler takes 256 plus accumulation registers for one
// wave, 1.05 ms instead of 0.79 ms; three or four spill and lose 10-20 %).
template <typename TS, typename TC>
constexpr int kMinWaves = sizeof(TC) == 4 ? 4 : (sizeof(TS) == 4 ? 3 : 2);

// One lane per track (the plain kernel; double precision runs here).
template <typename TS, typename TC, bool kFloatCov>
__global__ void __launch_bounds__(256, (kMinWaves<TS, TC>)) k_match(DevCfg<TS> g, MatchIO io)
{
    const int64_t i = (int64_t)xcd_block() * blockDim.x + threadIdx.x;
    if (i >= io.n) return;
    if (!match_lane<TS, TC, kFloatCov>(g, io, i, 0u))
        io.fb_list[atomicAdd(io.fb_count, 1u)] = (int32_t)i;
}

// Persistent variant: a grid sized to the resident capacity of the device
// pulls blocks of tracks from a work counter until every block is taken
// (each workgroup exits once the counter passes the last block).  The last
// workgroup to finish clears the counter for the next launch.
template <typename TS, typename TC, bool kFloatCov>
__global__ void __launch_bounds__(256, (kMinWaves<TS, TC>)) k_match_persistent(DevCfg<TS> g, MatchIO io)
{
    __shared__ uint32_t blk;
    const uint32_t nblk = (uint32_t)((io.n + blockDim.x - 1) / blockDim.x);
    for (;;) {
        if (threadIdx.x == 0) blk = atomicAdd(io.work_next, 1u);
        __syncthreads();
        const uint32_t b = blk;
        __syncthreads();
        if (b >= nblk) break;
        const int64_t i = (int64_t)b * blockDim.x + threadIdx.x;
        if (i < io.n && !match_lane<TS, TC, kFloatCov>(g, io, i, 0u))
            io.fb_list[atomicAdd(io.fb_count, 1u)] = (int32_t)i;
    }
    if (threadIdx.x == 0) {
        __threadfence();
        if (atomicAdd(io.work_done, 1u) == gridDim.x - 1) {
            atomicExch(io.work_next, 0u);
            atomicExch(io.work_done, 0u);
        }
    }
}

// Re-run of the queued tracks with a double covariance.  The last
// workgroup to finish clears the queue for the next call.
__global__ void __launch_bounds__(256) k_match_fallback(DevCfg<float> g, MatchIO io)
{
    const uint32_t cnt = *io.fb_count;
    for (uint32_t j = blockIdx.x * blockDim.x + threadIdx.x; j < cnt; j += gridDim.x * blockDim.x)
        match_lane<float, double, false>(g, io, io.fb_list[j], kFallback);
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        if (atomicAdd(io.fb_done, 1u) == gridDim.x - 1) {
            atomicExch(io.fb_count, 0u);
            atomicExch(io.fb_done, 0u);
        }
    }
}

// orders LDS traffic between the lanes of one wavefront
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Float state; the road scan of each track is shared by G lanes.  The
// per-lane phases (propagation, scattering, road, update) stay one track per
// lane; roads and winners pass through wave-private LDS slots.
template <typename TC, int G, bool kFloatCov>
__global__ void __launch_bounds__(256) k_match_coop(DevCfg<float> g, MatchIO io)
{
    __shared__ Road<float> roads[256];
    __shared__ Best<float> bests[256];
    const int tid = threadIdx.x, lane = tid & 63, wbase = tid & ~63;
    const int sub = lane % G, gid = lane / G;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + tid;
    Trk<float, TC> T;
    int grp = 0;
    uint32_t status = 0;
    bool live = false, queued = false;
    Acc<float> acc;
    acc_init(acc);
    if (i < io.n) {
        const int ld = load_track<float, TC, kFloatCov>(g, io, i, T, grp);
        live = ld == 0;
        queued = ld == 2;
        if (ld == 1) status |= kBadInput;
    }
    for (int l = 0; l < kLayers; l++) {
        acc.lidx = -1;
        acc.lchi = 0.0f;
        bool search = false;
        {
            Road<float> R;
            R.glo = 1;
            R.ghi = 0;
            if (live) {
                if (!predict(T, l, g, status)) {
                    live = false;
                } else {
                    search = open_road(T, l, grp, g, status, R);
                    if (!search && kFloatCov && (status & kNotPD)) {
                        queued = true;  // float innovation covariance not positive definite
                        live = false;
                    }
                }
            }
            roads[tid] = R;
        }
        wave_sync();
#pragma unroll 1
        for (int rnd = 0; rnd < G; rnd++) {
            const int slot = wbase + rnd * (64 / G) + gid;
            const Road<float> Q = roads[slot];
            Best<float> B = no_best<float>();
            if (Q.glo <= Q.ghi) scan_road_group<G>(Q, sub, g, io, B);
#pragma unroll
            for (int off = G / 2; off >= 1; off >>= 1) {
                const float oc = __shfl_xor(B.chi2, off, 64);
                const int oi = __shfl_xor(B.idx, off, 64);
                const int os = __shfl_xor(B.stack, off, 64);
                const float oy = __shfl_xor(B.y, off, 64);
                const float oz = __shfl_xor(B.z, off, 64);
                const bool take = better(oc, oi, B);
                B.chi2 = take ? oc : B.chi2;
                B.idx = take ? oi : B.idx;
                B.stack = take ? os : B.stack;
                B.y = take ? oy : B.y;
                B.z = take ? oz : B.z;
            }
            if (sub == 0) bests[slot] = B;
        }
        wave_sync();
        if (search) {
            const Best<float> B = bests[tid];
            if (B.idx != 0x7fffffff) {
                const Road<float> Rs = roads[tid];  // reloaded: not kept live across the scan
                const int rc = apply_best(T, l, Rs, B, g, io, status, acc);
                if (rc == 2 && kFloatCov) {
                    queued = true;
                    live = false;
                } else if (rc != 0 && (status & kStopSnp)) {
                    live = false;
                }
            }
        }
        if (i < io.n) write_layer(io, i, l, acc);
    }
    if (i < io.n) {
        if (queued)
            io.fb_list[atomicAdd(io.fb_count, 1u)] = (int32_t)i;
        else
            write_track(io, i, T, acc, status);
    }
}

template <typename TC, bool kFloatCov>
void launch_coop(int lanes, const DevCfg<float> &gf, const MatchIO &io, unsigned grid, int block,
                 hipStream_t s)
{
    switch (lanes) {
    case 4: launch_timed(io, k_match_coop<TC, 4, kFloatCov>, dim3(grid), dim3(block), s, gf, io); break;
    case 16: launch_timed(io, k_match_coop<TC, 16, kFloatCov>, dim3(grid), dim3(block), s, gf, io); break;
    case 32: launch_timed(io, k_match_coop<TC, 32, kFloatCov>, dim3(grid), dim3(block), s, gf, io); break;
    case 64: launch_timed(io, k_match_coop<TC, 64, kFloatCov>, dim3(grid), dim3(block), s, gf, io); break;
    default: launch_timed(io, k_match_coop<TC, 8, kFloatCov>, dim3(grid), dim3(block), s, gf, io); break;
    }
}

// ---- several hypotheses per track ------------------------------------------
// A group of N lanes (aligned inside the wavefront) holds one track; lane h
// holds the hypothesis of rank h.  Per layer every lane predicts its own
// hypothesis and keeps the N cheapest of its children in registers; N rounds
// of a group-wide minimum over the children's keys (cost, with-tracklet
// first, parent rank, tracklet index) then pick the survivors, and lane r
// takes the state of the r-th survivor's parent by cross-lane reads.

// the N cheapest passing candidates of one hypothesis, ascending (cost, index)
template <typename TS, int N>
struct TopN {
    TS base;  // the hypothesis' cost so far
    TS cost[N], chi2[N];
    int idx[N], stack[N];
    float y[N], z[N];

    __device__ __forceinline__ void init(TS b)
    {
        base = b;
#pragma unroll
        for (int k = 0; k < N; k++) {
            cost[k] = TS(INFINITY);
            chi2[k] = TS(0);
            idx[k] = 0x7fffffff;
            stack[k] = 0;
            y[k] = 0.f;
            z[k] = 0.f;
        }
    }

    __device__ __forceinline__ void offer(TS c, int oj, float yy, float zz, int st, bool pass)
    {
        const TS cc = base + c;
        if (!pass) return;
        // before[k]: the new entry sorts before entry k (monotone in k)
        bool before[N];
#pragma unroll
        for (int k = 0; k < N; k++) before[k] = cc < cost[k] || (cc == cost[k] && oj < idx[k]);
#pragma unroll
        for (int k = N - 1; k >= 1; k--) {
            const bool sh = before[k - 1], put = before[k] && !before[k - 1];
            cost[k] = sh ? cost[k - 1] : (put ? cc : cost[k]);
            chi2[k] = sh ? chi2[k - 1] : (put ? c : chi2[k]);
            idx[k] = sh ? idx[k - 1] : (put ? oj : idx[k]);
            stack[k] = sh ? stack[k - 1] : (put ? st : stack[k]);
            y[k] = sh ? y[k - 1] : (put ? yy : y[k]);
            z[k] = sh ? z[k - 1] : (put ? zz : z[k]);
        }
        cost[0] = before[0] ? cc : cost[0];
        chi2[0] = before[0] ? c : chi2[0];
        idx[0] = before[0] ? oj : idx[0];
        stack[0] = before[0] ? st : stack[0];
        y[0] = before[0] ? yy : y[0];
        z[0] = before[0] ? zz : z[0];
    }

    __device__ __forceinline__ void pop()
    {
#pragma unroll
        for (int k = 0; k < N - 1; k++) {
            cost[k] = cost[k + 1];
            chi2[k] = chi2[k + 1];
            idx[k] = idx[k + 1];
            stack[k] = stack[k + 1];
            y[k] = y[k + 1];
            z[k] = z[k + 1];
        }
        cost[N - 1] = TS(INFINITY);
        idx[N - 1] = 0x7fffffff;
    }
};

template <typename TS, typename TC>
struct Hyp {
    Trk<TS, TC> T;
    TS cost, chi2sum;
    int nmatch, live, valid;
    uint32_t status;
    int idx[kLayers];
    TS chi2l[kLayers];
};

// lane src's hypothesis (every lane of the group takes part)
template <typename TS, typename TC>
__device__ __forceinline__ void pull(Hyp<TS, TC> &H, int src)
{
    H.T.y = __shfl(H.T.y, src, 64);
    H.T.z = __shfl(H.T.z, src, 64);
    H.T.s = __shfl(H.T.s, src, 64);
    H.T.t = __shfl(H.T.t, src, 64);
    H.T.c = __shfl(H.T.c, src, 64);
    H.T.x = __shfl(H.T.x, src, 64);
#pragma unroll
    for (int k = 0; k < 15; k++) H.T.C[k] = __shfl(H.T.C[k], src, 64);
    H.T.sec = __shfl(H.T.sec, src, 64);
    H.cost = __shfl(H.cost, src, 64);
    H.chi2sum = __shfl(H.chi2sum, src, 64);
    H.nmatch = __shfl(H.nmatch, src, 64);
    H.live = __shfl(H.live, src, 64);
    H.valid = __shfl(H.valid, src, 64);
    H.status = (uint32_t)__shfl((int)H.status, src, 64);
#pragma unroll
    for (int k = 0; k < kLayers; k++) {
        H.idx[k] = __shfl(H.idx[k], src, 64);
        H.chi2l[k] = __shfl(H.chi2l[k], src, 64);
    }
}

// Precise propagation to the chosen tracklet and the Kalman update, as for
// the single best candidate.  False: the covariance lost positive
// definiteness (NOT_PD set).
template <typename TS, typename TC>
__device__ __forceinline__ bool beam_apply(Hyp<TS, TC> &H, int l, int j, TS c2, float yj, float zj, int st,
                                           const DevCfg<TS> &g)
{
    Trk<TS, TC> &T = H.T;
    const TS tau = g.tilt[l];
    const TS bdx = g.dx[T.sec * (kStacks * kLayers) + st * kLayers + l];
    if (bdx != TS(0) && !propagate(T, g.x_layer[l] + bdx, g)) {
        H.status |= kStopSnp;
        H.live = 0;
        return true;
    }
    const TS ry = TS(yj) - (T.y + tau * (T.z - TS(zj)));
    const TS rz = TS(zj) - T.z;
    const TS syu = poly2(g.sigma_y, T.s);
    bool pd = true;
    if (!kalman_update(T, ry, rz, tau, TC(syu) * TC(syu), TC(g.vz))) {
        H.status |= kNotPD;
        pd = false;
    }
#pragma unroll
    for (int k = 0; k < kLayers; k++) {
        H.idx[k] = k == l ? j : H.idx[k];
        H.chi2l[k] = k == l ? c2 : H.chi2l[k];
    }
    H.nmatch++;
    H.chi2sum += c2;
    if (!(fabs(T.s) < g.snp_max)) {
        H.status |= kStopSnp;
        H.live = 0;
    }
    return pd;
}

// One track on the N lanes of a group (h = rank, base = first lane of the
// group).  False: re-run with a double covariance (kQueueNotPD only); the
// answer is group-uniform.
template <typename TS, typename TC, int N, bool kQueueNotPD>
__device__ __forceinline__ bool beam_track(const DevCfg<TS> &g, const MatchIO &io, int64_t i, int h, int base,
                                           uint32_t status0)
{
    Hyp<TS, TC> H;
    H.T.y = H.T.z = H.T.s = H.T.t = H.T.c = H.T.x = TS(0);
#pragma unroll
    for (int k = 0; k < 15; k++) H.T.C[k] = TC(0);
    H.T.sec = 0;
    H.cost = H.chi2sum = TS(0);
    H.nmatch = 0;
    H.live = H.valid = 0;
    H.status = status0;
#pragma unroll
    for (int k = 0; k < kLayers; k++) {
        H.idx[k] = -1;
        H.chi2l[k] = TS(0);
    }
    int grp = 0, ld = 1;
    if (h == 0) {
        ld = load_track<TS, TC, kQueueNotPD>(g, io, i, H.T, grp);
        H.valid = 1;
        H.live = ld == 0;
        if (ld == 1) H.status |= kBadInput;
    }
    ld = __shfl(ld, base, 64);
    grp = __shfl(grp, base, 64);
    if (ld == 2) return false;
    for (int l = 0; l < kLayers; l++) {
        TopN<TS, N> L;
        L.init(H.cost);
        bool no_chamber = false;
        if (H.valid && H.live) {
            if (!predict(H.T, l, g, H.status)) {
                H.live = 0;
            } else {
                no_chamber = absent_at(g, H.T.sec, l, H.T.z);
                Road<TS> R;
                if (open_road(H.T, l, grp, g, H.status, R)) scan_road_flat(R, g, io, L);
            }
        }
        if (kQueueNotPD) {
            // a float innovation covariance that is not positive definite
            // sends the whole track to the double re-run
            int lost = (H.status & kNotPD) ? 1 : 0;
#pragma unroll
            for (int off = N / 2; off >= 1; off >>= 1) lost |= __shfl_xor(lost, off, 64);
            if (lost) return false;
        }
        // survivors: N rounds of a group-wide minimum; a layer whose
        // predicted point lies in an empty chamber slot costs no penalty
        const TS skip_cost = H.cost + (no_chamber ? TS(0) : g.chi2_penalty);
        bool skip = H.valid != 0;
        int s_ok = 0, s_par = h, s_j = -1, s_st = 0;
        TS s_cost = TS(0), s_c2 = TS(0);
        float s_y = 0.f, s_z = 0.f;
#pragma unroll 1
        for (int r = 0; r < N; r++) {
            const bool trk = L.idx[0] != 0x7fffffff;
            const bool use_trk = trk && (!skip || !(skip_cost < L.cost[0]));
            TS mc = use_trk ? L.cost[0] : (skip ? skip_cost : TS(INFINITY));
            int ms = use_trk ? 0 : (skip ? 1 : 2);
            int mj = use_trk ? L.idx[0] : (skip ? -1 : 0x7fffffff);
            int mh = h;
#pragma unroll
            for (int off = N / 2; off >= 1; off >>= 1) {
                const TS oc = __shfl_xor(mc, off, 64);
                const int os = __shfl_xor(ms, off, 64);
                const int oh = __shfl_xor(mh, off, 64);
                const int oj = __shfl_xor(mj, off, 64);
                const bool take =
                    oc < mc ||
                    (oc == mc && (os < ms || (os == ms && (oh < mh || (oh == mh && oj < mj)))));
                mc = take ? oc : mc;
                ms = take ? os : ms;
                mh = take ? oh : mh;
                mj = take ? oj : mj;
            }
            const int src = base + mh;
            const TS pc2 = __shfl(L.chi2[0], src, 64);
            const float py = __shfl(L.y[0], src, 64);
            const float pz = __shfl(L.z[0], src, 64);
            const int pst = __shfl(L.stack[0], src, 64);
            if (h == r) {
                s_ok = ms != 2;
                s_par = ms != 2 ? mh : h;
                s_j = ms == 0 ? mj : -1;
                s_cost = mc;
                s_c2 = pc2;
                s_y = py;
                s_z = pz;
                s_st = pst;
            }
            if (h == mh && ms == 0) L.pop();
            if (h == mh && ms == 1) skip = false;
        }
        pull(H, base + s_par);
        int lost_pd = 0;
        if (!s_ok) {
            H.valid = 0;
        } else {
            H.cost = s_cost;
            if (s_j >= 0 && H.live && !beam_apply(H, l, s_j, s_c2, s_y, s_z, s_st, g)) lost_pd = 1;
        }
        if (kQueueNotPD) {
#pragma unroll
            for (int off = N / 2; off >= 1; off >>= 1) lost_pd |= __shfl_xor(lost_pd, off, 64);
            if (lost_pd) return false;
        }
    }
    if (h == 0) {
        Acc<TS> lay;
        acc_init(lay);
#pragma unroll
        for (int k = 0; k < kLayers; k++) {
            lay.lidx = H.idx[k];
            lay.lchi = H.chi2l[k];
            write_layer(io, i, k, lay);
        }
        Acc<TS> acc;
        acc.nmatch = H.nmatch;
        acc.chi2sum = H.chi2sum;
        acc.lidx = -1;
        acc.lchi = TS(0);
        write_track(io, i, H.T, acc, H.status);
    }
    return true;
}

template <typename TS, typename TC, int N, bool kFloatCov>
__global__ void __launch_bounds__(256, sizeof(TC) == 4 ? 4 : 1) k_match_beam(DevCfg<TS> g, MatchIO io)
{
    const int lane = threadIdx.x & 63, h = lane & (N - 1), base = lane & ~(N - 1);
    const int64_t i = ((int64_t)xcd_block() * blockDim.x + threadIdx.x) / N;
    if (i >= io.n) return;  // uniform over the group
    if (!beam_track<TS, TC, N, kFloatCov>(g, io, i, h, base, 0u) && h == 0)
        io.fb_list[atomicAdd(io.fb_count, 1u)] = (int32_t)i;
}

// Re-run of queued tracks with a double covariance, N lanes per track.
template <int N>
__global__ void __launch_bounds__(256) k_beam_fallback(DevCfg<float> g, MatchIO io)
{
    const uint32_t cnt = *io.fb_count;
    const int lane = threadIdx.x & 63, h = lane & (N - 1), base = lane & ~(N - 1);
    const uint32_t per_block = blockDim.x / N;
    for (uint32_t j = blockIdx.x * per_block + threadIdx.x / N; j < cnt; j += gridDim.x * per_block)
        beam_track<float, double, N, false>(g, io, io.fb_list[j], h, base, kFallback);
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        if (atomicAdd(io.fb_done, 1u) == gridDim.x - 1) {
            atomicExch(io.fb_count, 0u);
            atomicExch(io.fb_done, 0u);
        }
    }
}

template <typename TS, typename TC, bool kFloatCov>
void launch_beam_t(const DevCfg<TS> &g, const MatchIO &io, int n_hyp, hipStream_t s)
{
    const unsigned grid = (unsigned)((io.n * n_hyp + 255) / 256);
    switch (n_hyp) {
    case 1: launch_timed(io, k_match_beam<TS, TC, 1, kFloatCov>, dim3(grid), dim3(256), s, g, io); break;
    case 2: launch_timed(io, k_match_beam<TS, TC, 2, kFloatCov>, dim3(grid), dim3(256), s, g, io); break;
    case 4: launch_timed(io, k_match_beam<TS, TC, 4, kFloatCov>, dim3(grid), dim3(256), s, g, io); break;
    default: launch_timed(io, k_match_beam<TS, TC, 8, kFloatCov>, dim3(grid), dim3(256), s, g, io); break;
    }
}

}  // namespace

void launch_beam(int precision, const DevCfg<double> &gd, const DevCfg<float> &gf, const MatchIO &io,
                 int n_hyp, hipStream_t s)
{
    if (io.n <= 0) return;
    if (precision == 0) {
        launch_beam_t<double, double, false>(gd, io, n_hyp, s);
    } else if (precision == 2) {
        launch_beam_t<float, double, false>(gf, io, n_hyp, s);
    } else {
        launch_beam_t<float, float, true>(gf, io, n_hyp, s);
    }
    if (precision == 1) {
        switch (n_hyp) {
        case 1: hipLaunchKernelGGL(k_beam_fallback<1>, dim3(64), dim3(256), 0, s, gf, io); break;
        case 2: hipLaunchKernelGGL(k_beam_fallback<2>, dim3(64), dim3(256), 0, s, gf, io); break;
        case 4: hipLaunchKernelGGL(k_beam_fallback<4>, dim3(64), dim3(256), 0, s, gf, io); break;
        default: hipLaunchKernelGGL(k_beam_fallback<8>, dim3(64), dim3(256), 0, s, gf, io); break;
        }
    }
}

namespace {

// ---- TRD-only refit --------------------------------------------------------
// One lane per track, inward over the layers: the matched track's state with
// the covariance reset, propagation to each layer plane, a turn into the
// tracklet's sector when it is a neighbour, the precise step and the update,
// then the layer's scattering (none below layer 0).  Covariance in double.
// (Float state: compiled for three waves per SIMD, 3 % faster than two; four
// spill.)
template <typename TS>
__global__ void __launch_bounds__(256, sizeof(TS) == 4 ? 3 : 1) k_refit(DevCfg<TS> g, RefitIO io)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= io.n) return;
    const int64_t n = io.n;
    const TS *ip = reinterpret_cast<const TS *>(io.ip);
    Trk<TS, double> T;
    T.y = ip[i];
    T.z = ip[n + i];
    T.s = ip[2 * n + i];
    T.t = ip[3 * n + i];
    T.c = ip[4 * n + i];
    T.x = reinterpret_cast<const TS *>(io.ix)[i];
    T.sec = io.isec[i];
#pragma unroll
    for (int k = 0; k < 15; k++) T.C[k] = 0.0;
    T.C[YY] = io.cov0[0];
    T.C[ZZ] = io.cov0[1];
    T.C[SS] = io.cov0[2];
    T.C[TT] = io.cov0[3];
    T.C[CC] = io.cov0[4];
    // a usable index names a tracklet of that layer's chamber: in [0, n_tkl),
    // with a chamber below 540 whose layer is l; any other counts as absent
    // (so dx[det] is never read out of its table)
    int idx[kLayers], nm = 0;
#pragma unroll
    for (int l = 0; l < kLayers; l++) {
        int j = io.idx[l * n + i];
        if (j >= 0 && j < io.n_tkl) {
            const uint32_t det = io.det_row[j] >> 5;
            if (!(det < (uint32_t)kDet && det % kLayers == (uint32_t)l)) j = -1;
        } else {
            j = -1;
        }
        idx[l] = j;
        nm += j >= 0 ? 1 : 0;
    }
    uint32_t status = 0;
    int nused = 0;
    double chi2 = 0.0;
    bool bad = !(__builtin_isfinite(T.x) && T.sec >= 0 && T.sec < kSectors && __builtin_isfinite(T.y) &&
                 __builtin_isfinite(T.z) && __builtin_isfinite(T.s) && __builtin_isfinite(T.t) &&
                 __builtin_isfinite(T.c));
    if (!bad) bad = !(fabs(T.s) < g.snp_max);
    if (bad) {
        status = kBadInput;
    } else if (nm < io.min_tracklets) {
        status = kRefitFew;
    } else {
        const double vz = double(g.pad_len) * double(g.pad_len) / 12.0;
        for (int l = kLayers - 1; l >= 0; l--) {
            if (!reach_plane(T, l, g, status)) break;
            const int j = idx[l];
            if (j >= 0) {
                const int det = (int)(io.det_row[j] >> 5), st = det / (kStacks * kLayers);
                bool use = true;
                if (st != T.sec) {
                    const int d = (st - T.sec + kSectors) % kSectors;
                    if (d == 1 || d == kSectors - 1) {
                        if (!rotate(T, d == 1, g)) {
                            status |= kRotFail;
                            break;
                        }
                        T.sec = st;
                        if (!propagate(T, g.x_layer[l], g)) {
                            status |= kStopSnp;
                            break;
                        }
                    } else {
                        status |= kRefitSkip;
                        use = false;
                    }
                }
                if (use) {
                    const TS dxj = g.dx[det];
                    if (dxj != TS(0) && !propagate(T, g.x_layer[l] + dxj, g)) {
                        status |= kStopSnp;
                        break;
                    }
                    const TS tau = g.tilt[l];
                    const TS yj = TS(io.y[j]), zj = TS(io.z[j]);
                    const TS ry = yj - (T.y + tau * (T.z - zj));
                    const TS rz = zj - T.z;
                    const double sy = double(poly2(g.sigma_y, T.s)), tc = double(tau);
                    const double Syy = T.C[YY] + 2.0 * tc * T.C[YZ] + tc * tc * T.C[ZZ] + sy * sy;
                    const double Syz = T.C[YZ] + tc * T.C[ZZ];
                    const double Szz = T.C[ZZ] + vz;
                    const double dry = double(ry), drz = double(rz);
                    chi2 += (Szz * dry * dry - 2.0 * Syz * dry * drz + Syy * drz * drz) / (Syy * Szz - Syz * Syz);
                    if (!kalman_update(T, ry, rz, tau, sy * sy, vz)) status |= kNotPD;
                    nused++;
                    if (!(fabs(T.s) < g.snp_max)) {
                        status |= kStopSnp;
                        break;
                    }
                }
            }
            if (l > 0) {
                add_ms(T, g);
                eloss(T, g, false);
            }
        }
    }
    TS *op = reinterpret_cast<TS *>(io.op);
    TS *oc = reinterpret_cast<TS *>(io.oc);
    op[i] = T.y;
    op[n + i] = T.z;
    op[2 * n + i] = T.s;
    op[3 * n + i] = T.t;
    op[4 * n + i] = T.c;
#pragma unroll
    for (int k = 0; k < 15; k++) oc[k * n + i] = TS(T.C[k]);
    reinterpret_cast<TS *>(io.ox)[i] = T.x;
    io.osec[i] = T.sec;
    reinterpret_cast<TS *>(io.ochi2)[i] = TS(chi2);
    io.onused[i] = nused;
    io.ost[i] = status;
}

// ---- residual maps of TPC clusters ---------------------------------------
// Position-only forms of the helix step and the frame turn (same arithmetic
// as propagate and rotate, without the covariance).
template <typename TS>
__device__ __forceinline__ bool step_state(TS &x, TS &y, TS &z, TS &s, TS t, TS c, TS x2, const DevCfg<TS> &g)
{
    const TS dx = x2 - x;
    const TS cu = g.k_curv * c;
    const TS s1 = s;
    const TS s2 = s1 + cu * dx;
    if (!(fabs(s2) < g.snp_max)) return false;
    const TS f1 = sqrt(TS(1) - s1 * s1);
    const TS f2 = sqrt(TS(1) - s2 * s2);
    const TS dy = div_(dx * (s1 + s2), f1 + f2);
    const TS chord = sqrt(dx * dx + dy * dy);
    const TS h = TS(0.5) * fabs(cu) * chord;
    const TS aoh = asin_over(h);
    const TS arc = (dx >= TS(0) ? chord : -chord) * aoh;
    y += dy;
    z += t * arc;
    s = s2;
    x = x2;
    return true;
}

template <typename TS>
__device__ __forceinline__ bool turn_state(TS &x, TS &y, TS &s, bool up, const DevCfg<TS> &g)
{
    const TS ca = g.cos_sector, sa = up ? g.sin_sector : -g.sin_sector;
    const TS f = sqrt(TS(1) - s * s);
    const TS s1 = s * ca - f * sa;
    const TS f1 = f * ca + s * sa;
    if (!(f1 > TS(0))) return false;
    const TS x1 = x * ca + y * sa;
    const TS y1 = -x * sa + y * ca;
    x = x1;
    y = y1;
    s = s1;
    return true;
}

// One lane per reference track, walking its clusters inward.  The 8 sums of
// every voxel are kept per workgroup in LDS, in the state type (float, or
// double for the double path: 64 B per voxel, at most 128 KB), and added to
// the global double sums at the end; a lane keeps the sums of the voxel it is in in
// registers and adds them to LDS only when the walk leaves that voxel (a
// track stays in one voxel for several pad rows), which cuts the LDS atomics
// several-fold.  The clusters of a track are fetched kPre at a time ahead of
// the walk (they do not depend on it).  Grid-stride over the tracks.
template <typename TS, int kThreads>
__global__ void __launch_bounds__(kThreads) k_residual_sums(DevCfg<TS> g, ResidualIO io)
{
    constexpr int kPre = 8;
    extern __shared__ __align__(8) unsigned char lds_raw[];
    TS *ls = reinterpret_cast<TS *>(lds_raw);
    const int nsum = io.nvox * kVoxelSums;
    for (int k = threadIdx.x; k < nsum; k += blockDim.x) ls[k] = TS(0);
    __syncthreads();
    const TS *rp = reinterpret_cast<const TS *>(io.rp);
    const TS *rx = reinterpret_cast<const TS *>(io.rx);
    const TS step = TS(io.x_out - io.x_in) / TS(io.n_rows - 1);
    const TS fxs = TS(io.nx) / TS(io.x_out - io.x_in);
    int vox = -1;  // voxel whose sums the lane holds
    TS acc[kVoxelSums];
#pragma unroll
    for (int q = 0; q < kVoxelSums; q++) acc[q] = TS(0);
    auto flush = [&]() {
        if (vox >= 0) {
            TS *S = ls + kVoxelSums * vox;
#pragma unroll
            for (int q = 0; q < kVoxelSums; q++) {
                atomicAdd(&S[q], acc[q]);
                acc[q] = TS(0);
            }
        }
    };
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < io.n;
         i += (int64_t)gridDim.x * blockDim.x) {
        if (io.rstatus[i] != 0) continue;
        TS y = rp[i], z = rp[io.n + i], sn = rp[2 * io.n + i], t = rp[3 * io.n + i], c = rp[4 * io.n + i];
        TS x = rx[i];
        int sec = io.rsec[i];
        if (sec < 0 || sec >= kSectors) continue;
        const int64_t kend = io.first[i + 1];
        bool live = true;
        for (int64_t k0 = io.first[i]; live && k0 < kend; k0 += kPre) {
            uint32_t rsv[kPre];
            float cyv[kPre], czv[kPre];
#pragma unroll
            for (int u = 0; u < kPre; u++) {
                rsv[u] = 0xffffffffu;
                cyv[u] = czv[u] = 0.f;
                if (k0 + u < kend) {
                    rsv[u] = io.row_sec[k0 + u];
                    cyv[u] = io.cy[k0 + u];
                    czv[u] = io.cz[k0 + u];
                }
            }
#pragma unroll
            for (int u = 0; u < kPre; u++) {
                if (!live) continue;
                const uint32_t rs = rsv[u];
                const int csec = (int)(rs >> 16), row = (int)(rs & 0xffffu);
                if (csec >= kSectors || row >= io.n_rows) continue;
                const TS xr = TS(io.x_out) - TS(row) * step;
                if (csec != sec) {
                    const int d = (csec - sec + kSectors) % kSectors;
                    if (d != 1 && d != kSectors - 1) continue;
                    if (!turn_state(x, y, sn, d == 1, g)) {
                        live = false;
                        continue;
                    }
                    sec = csec;
                }
                if (!step_state(x, y, z, sn, t, c, xr, g)) {
                    live = false;
                    continue;
                }
                const TS f = sqrt(TS(1) - sn * sn);
                const TS ty = div_(sn, f), tz = div_(t, f);
                const TS ry = TS(cyv[u]) - y, rz = TS(czv[u]) - z;
                const TS fx = (xr - TS(io.x_in)) * fxs;
                const TS fy = (div_(div_(y, xr), g.tan_half_sector) + TS(1)) * TS(0.5) * TS(io.ny);
                const TS fz = (div_(z, xr) + TS(1)) * TS(0.5) * TS(io.nz);
                const int ix = fx < TS(0) ? 0 : (fx >= TS(io.nx) ? io.nx - 1 : (int)fx);
                const int iy = fy < TS(0) ? 0 : (fy >= TS(io.ny) ? io.ny - 1 : (int)fy);
                const int iz = fz < TS(0) ? 0 : (fz >= TS(io.nz) ? io.nz - 1 : (int)fz);
                const int v = ((sec * io.nx + ix) * io.ny + iy) * io.nz + iz;
                if (v != vox) {
                    flush();
                    vox = v;
                }
                acc[0] += TS(1);
                acc[1] += ty;
                acc[2] += tz;
                acc[3] += ty * ty + tz * tz;
                acc[4] += ry;
                acc[5] += rz;
                acc[6] += ty * ry + tz * rz;
                acc[7] += ry * ry + rz * rz;
            }
        }
    }
    flush();
    __syncthreads();
    for (int k = threadIdx.x; k < nsum; k += blockDim.x) {
        const TS v = ls[k];
        if (v != TS(0)) atomicAdd(&io.sums[k], (double)v);
    }
}

// Per voxel (dX, dY, dZ, n): the least-squares solution of
// r_y = dY - dX tan(phi), r_z = dZ - dX tan(lambda)/cos(phi) from its sums.
__global__ void __launch_bounds__(256) k_voxel_solve(const double *sums, int nvox, int min_count, float *dist)
{
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= nvox) return;
    const double *S = sums + kVoxelSums * v;
    float4 o = make_float4(__builtin_nanf(""), __builtin_nanf(""), __builtin_nanf(""), float(S[0]));
    const double nn = S[0], st = S[1], sz = S[2], stt = S[3];
    if (nn >= min_count) {
        const double a = stt - (st * st + sz * sz) / nn;
        const double b = -S[6] + (st * S[4] + sz * S[5]) / nn;
        if (a > 1e-12 * stt) {
            const double dX = b / a;
            o.x = float(dX);
            o.y = float((S[4] + st * dX) / nn);
            o.z = float((S[5] + sz * dX) / nn);
        }
    }
    reinterpret_cast<float4 *>(dist)[v] = o;
}

// input track i -> state row rank[i] (coalesced reads, one row per lane;
// kGrouped: groups read from io.igrp, else 0, so that no load is behind a
// branch)
template <typename TS, bool kGrouped>
__global__ void __launch_bounds__(256) k_track_pack(MatchIO io, const uint32_t *rank, TS *rows)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= io.n) return;
    const int64_t n = io.n;
    const TS *ip = reinterpret_cast<const TS *>(io.ip);
    const TS *ic = reinterpret_cast<const TS *>(io.ic);
    const TS *ix = reinterpret_cast<const TS *>(io.ix);
    TS v[kRowIn];
#pragma unroll
    for (int k = 0; k < 5; k++) v[k] = ip[k * n + i];
#pragma unroll
    for (int k = 0; k < 15; k++) v[5 + k] = ic[k * n + i];
    v[20] = ix[i];
    v[21] = as_row(io.isec[i], TS());
    v[22] = as_row(kGrouped ? io.igrp[i] : 0, TS());
    v[23] = TS(0);
    TS *r = rows + (int64_t)rank[i] * kRowIn;
#pragma unroll
    for (int k = 0; k < kRowIn; k++) r[k] = v[k];
}

// result row rank[i] -> the caller's arrays at input position i
template <typename TS, int kRow>
__global__ void __launch_bounds__(256) k_track_unpack(MatchIO io, const uint32_t *rank, const TS *rows)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= io.n) return;
    const int64_t n = io.n;
    const TS *r = rows + (int64_t)rank[i] * kRow;
    TS v[kRow];
#pragma unroll
    for (int k = 0; k < kRow; k++) v[k] = r[k];
    TS *op = reinterpret_cast<TS *>(io.op);
    TS *oc = reinterpret_cast<TS *>(io.oc);
    TS *ox = reinterpret_cast<TS *>(io.ox);
    TS *och = reinterpret_cast<TS *>(io.ochi2);
#pragma unroll
    for (int k = 0; k < 5; k++) op[k * n + i] = v[k];
#pragma unroll
    for (int k = 0; k < 15; k++) oc[k * n + i] = v[5 + k];
    ox[i] = v[20];
    och[i] = v[21];
    io.osec[i] = int_of(v[22]);
    io.onm[i] = int_of(v[23]);
    io.ost[i] = (uint32_t)int_of(v[24]);
#pragma unroll
    for (int l = 0; l < kLayers; l++) io.oidx[l * n + i] = int_of(v[25 + l]);
    if constexpr (kRow > kRowChi2) {
        TS *ochl = reinterpret_cast<TS *>(io.ochi2l);
#pragma unroll
        for (int l = 0; l < kLayers; l++) ochl[l * n + i] = v[kRowChi2 + l];
    }
}

inline unsigned blocks_for(int64_t n) { return (unsigned)((n + 255) / 256); }

template <typename TS>
void order_in(MatchIO &io, int32_t n_groups, const TrackOrder &o, hipStream_t s)
{
    const int64_t n = io.n;
    launch_track_sort(sizeof(TS) == 8 ? 0 : 1, io.ip, io.isec, io.igrp, n, n_groups, o, s);
    if (io.igrp)
        hipLaunchKernelGGL((k_track_pack<TS, true>), dim3(blocks_for(n)), dim3(256), 0, s, io,
                           (const uint32_t *)o.rank, reinterpret_cast<TS *>(o.rows_in));
    else
        hipLaunchKernelGGL((k_track_pack<TS, false>), dim3(blocks_for(n)), dim3(256), 0, s, io,
                           (const uint32_t *)o.rank, reinterpret_cast<TS *>(o.rows_in));
    io.rows_in = o.rows_in;
    io.rows_out = o.rows_out;
    io.row_out = io.ochi2l ? kRowOut : kRowOutShort;
}

template <typename TS>
void order_out(const MatchIO &io, const TrackOrder &o, hipStream_t s)
{
    if (io.row_out == kRowOut)
        hipLaunchKernelGGL((k_track_unpack<TS, kRowOut>), dim3(blocks_for(io.n)), dim3(256), 0, s, io,
                           (const uint32_t *)o.rank, reinterpret_cast<const TS *>(o.rows_out));
    else
        hipLaunchKernelGGL((k_track_unpack<TS, kRowOutShort>), dim3(blocks_for(io.n)), dim3(256), 0, s, io,
                           (const uint32_t *)o.rank, reinterpret_cast<const TS *>(o.rows_out));
}

}  // namespace

void launch_order_in(int precision, MatchIO &io, int32_t n_groups, const TrackOrder &o, hipStream_t s)
{
    if (io.n <= 0) return;
    if (precision == 0)
        order_in<double>(io, n_groups, o, s);
    else
        order_in<float>(io, n_groups, o, s);
}

void launch_refit(int precision, const DevCfg<double> &gd, const DevCfg<float> &gf, const RefitIO &io,
                  hipStream_t s)
{
    if (io.n <= 0) return;
    const unsigned grid = (unsigned)((io.n + 255) / 256);
    if (precision == 0)
        hipLaunchKernelGGL(k_refit<double>, dim3(grid), dim3(256), 0, s, gd, io);
    else
        hipLaunchKernelGGL(k_refit<float>, dim3(grid), dim3(256), 0, s, gf, io);
}

void launch_residual_sums(int precision, const DevCfg<double> &gd, const DevCfg<float> &gf,
                          const ResidualIO &io, int n_cu, hipStream_t s)
{
    if (io.n <= 0) return;
    constexpr int kThreads = 1024;
    const size_t lds = (precision == 0 ? sizeof(double) : sizeof(float)) * (size_t)io.nvox * kVoxelSums;
    int64_t blocks = (io.n + kThreads - 1) / kThreads;
    // two workgroups per CU (one with the double sums: up to 128 KB of LDS)
    const int64_t cap = (precision == 0 ? 1 : 2) * (int64_t)(n_cu > 0 ? n_cu : 1);
    if (blocks > cap) blocks = cap;
    if (precision == 0) {
        (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&k_residual_sums<double, kThreads>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        hipLaunchKernelGGL((k_residual_sums<double, kThreads>), dim3((unsigned)blocks), dim3(kThreads), lds, s, gd,
                           io);
    } else
        hipLaunchKernelGGL((k_residual_sums<float, kThreads>), dim3((unsigned)blocks), dim3(kThreads), lds, s, gf,
                           io);
}

void launch_voxel_solve(const double *sums, int nvox, int min_count, float *dist, hipStream_t s)
{
    if (nvox <= 0) return;
    hipLaunchKernelGGL(k_voxel_solve, dim3((unsigned)((nvox + 255) / 256)), dim3(256), 0, s, sums, nvox,
                       min_count, dist);
}

void launch_order_out(int precision, const MatchIO &io, const TrackOrder &o, hipStream_t s)
{
    if (io.n <= 0) return;
    if (precision == 0)
        order_out<double>(io, o, s);
    else
        order_out<float>(io, o, s);
}

template <typename TS, typename TC, bool kFloatCov>
unsigned persistent_grid(int block, int n_cu, unsigned grid)
{
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_match_persistent<TS, TC, kFloatCov>,
                                                     block, 0) != hipSuccess || per_cu < 1)
        per_cu = 1;
    const unsigned cap = (unsigned)(per_cu * (n_cu > 0 ? n_cu : 1));
    return grid < cap ? grid : cap;
}

template <typename TS, typename TC, bool kFloatCov>
void launch_lane(const DevCfg<TS> &g, const MatchIO &io, unsigned grid, int block, bool persistent,
                 int n_cu, hipStream_t s)
{
    if (persistent) {
        const unsigned pg = persistent_grid<TS, TC, kFloatCov>(block, n_cu, grid);
        launch_timed(io, k_match_persistent<TS, TC, kFloatCov>, dim3(pg), dim3(block), s, g, io);
    } else {
        launch_timed(io, k_match<TS, TC, kFloatCov>, dim3(grid), dim3(block), s, g, io);
    }
}

void launch_match(int precision, const DevCfg<double> &gd, const DevCfg<float> &gf,
                  const MatchIO &io, int block, int lanes, bool persistent, int n_cu, hipStream_t s)
{
    if (io.n <= 0) return;
    const unsigned grid = (unsigned)((io.n + block - 1) / block);
    if (precision == 0) {
        launch_lane<double, double, false>(gd, io, grid, block, persistent, n_cu, s);
    } else if (precision == 2) {
        if (lanes == 1)
            launch_lane<float, double, false>(gf, io, grid, block, persistent, n_cu, s);
        else
            launch_coop<double, false>(lanes, gf, io, grid, block, s);
    } else {
        if (lanes == 1)
            launch_lane<float, float, true>(gf, io, grid, block, persistent, n_cu, s);
        else
            launch_coop<float, true>(lanes, gf, io, grid, block, s);
    }
    if (precision == 1) hipLaunchKernelGGL(k_match_fallback, dim3(64), dim3(256), 0, s, gf, io);
}

}  // namespace trd
