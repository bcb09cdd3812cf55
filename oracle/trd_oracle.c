/*
 * FP64 CPU oracle of TRD tracklet-to-track matching.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may call, link or
 * load this file: only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark use it.  It shares no source with the HIP library.
 *
 * What it computes, following Sect. 3 of the paper ("TRD tracking
 * algorithm") step by step and in plain double precision:
 *
 *   for every seed track (independently; the paper parallelises over tracks)
 *     for layer l = 0..5
 *       propagate the helix state and covariance to the layer radius
 *       (the most precise extrapolation step of Sect. 3, here a uniform field);
 *       rotate into the neighbouring sector if the point left the sector;
 *       add multiple scattering of the layer;
 *       open a search road sized from the covariances (Sect. 3);
 *       for every tracklet in the road: linear extrapolation to the
 *       tracklet radius, pad-tilt corrected y residual (Sect. 3, last
 *       paragraph), dy exclusion beyond 4 sigma, chi2 from y and z only;
 *       keep the best hypothesis (N_candidates = 1), propagate precisely to
 *       its radius and apply the Kalman update.
 *
 * Readings where the paper is silent (all shared with the HIP path by
 * specification, not by code):
 *   - propagation is the exact helix map in (y, z, sin phi, tan lambda, q/pT)
 *     with its exact Jacobian; curvature C = -kappa * Bz * q/pT so that
 *     sin phi grows by C per cm of x;
 *   - one thin scatterer per layer, Highland width, pion mass;
 *   - tracklet resolutions are second-order polynomials in sin phi, the dy
 *     gate width adds the track slope error: sqrt(s_dy^2 + L^2 C_ss / f^6);
 *   - road half widths n_road * sqrt(S_yy), n_road * sqrt(S_zz) around the
 *     prediction; chi2 <= chi2_max; winner = lexicographic min (chi2, index);
 *   - tracklet cells: key = (((group*540 + det)*n_db + dbin)*n_yb + ybin)*n_rows
 *     + row, ybin = clamp(floor((y - y_min) * (1/w)), 0, n_yb-1) and dbin the
 *     same on dy with its own width, both in double; a road is searched over
 *     the deflection bins x y bins x pad rows that overlap it;
 *   - optional realistic detector model: after the scattering, the layer's
 *     mean energy loss (Bethe formula) lowers the momentum; chamber slots
 *     marked absent hold no tracklets (their tracklets are dropped), and in
 *     the hypothesis mode a layer whose predicted point lies in an absent
 *     chamber costs no penalty.
 *
 * Decision-margin flags mark tracks where a gate, tie or geometric decision
 * lies within a margin, so that a correct implementation in a different
 * precision may legitimately decide differently there.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define NLAY 6
#define NSEC 18
#define NSTK 5
#define NDET 540

/* status bits */
#define ST_STOP_SNP 1u
#define ST_ROT_FAIL 2u
#define ST_OUT_OF_Z 4u
#define ST_BAD_INPUT 32u
#define ST_REFIT_FEW 64u   /* refit: fewer tracklets than refit_min, copied */
#define ST_REFIT_SKIP 128u /* refit: a tracklet more than one sector away was skipped */
#define ST_STOPPED 256u    /* the layer's energy loss left no kinetic energy */
/* decision-margin flags */
#define FL_P1 1u /* winner near one of its gates */
#define FL_P2 2u /* a loser fails exactly one gate by a margin and would win */
#define FL_P3 4u /* near tie between winner and runner-up */
#define FL_P4 8u /* sector edge, z acceptance or sin(phi) limit near */
/* which gate a P1 or P2 decision concerned (both can be set) */
#define FL_KCUT 16u  /* the chi2 cut */
#define FL_KGATE 32u /* a road edge or the dy gate */

typedef struct {
    double x_layer[NLAY];
    double tilt[NLAY];          /* tan of the pad tilt angle per layer */
    double z_min, pad_len;
    double y_bin_w;             /* power of two, cm */
    double dy_bin_w;            /* power of two, cm (deflection bins) */
    double drift_len;
    double dx_chamber[NDET];
    double bz, x_over_x0, mass;
    double sigma_y[3], sigma_dy[3], tan_psi;
    double chi2_max, n_sigma_dy, n_sigma_road, snp_max;
    double m_rel, m_len, m_dy, m_chi2, m_snp; /* decision margins */
    int32_t n_rows, n_yb, n_db;
    int32_t n_hyp;              /* 0: single best candidate; >= 1: hypotheses kept per layer */
    double chi2_penalty;        /* cost of a layer without a tracklet (hypothesis mode) */
    double refit_cov[5];        /* TRD-only refit: starting covariance (diagonal) */
    int32_t refit_min, pad_;    /* TRD-only refit: fewest tracklets refitted */
    /* realistic detector model (Sect. 3: propagation with energy loss; the
     * detector has 522 of its 540 chamber slots equipped) */
    double eloss_xrho;          /* layer material crossed at normal incidence, g/cm^2 (0: no loss) */
    double eloss_za;            /* its Z/A */
    double eloss_i;             /* its mean excitation energy, GeV */
    uint8_t absent[NDET];       /* nonzero: no chamber in this slot */
    uint8_t pad2_[4];
    double m_ke;                /* decision margin: kinetic energy left after a layer's
                                   loss within this fraction of the energy before it */
    double m_state;             /* decision margin: relative tolerance of the compared
                                   path's predicted y and z (floor 10 cm), carried into
                                   each road's chi2 (0: none) */
    /* field inhomogeneity (Sect. 3: the precise extrapolation accounts for the
     * field): Bz(r, z) = bz (1 + field_br (r / 370 cm)^2 + field_bz (z / 360 cm)^2);
     * both 0 = uniform field, stepped in closed form */
    double field_br, field_bz;
    double field_step;          /* largest x step of the integration in a field map, cm */
} ocfg;

static const double KAPPA = 2.99792458e-3;

/* ---------------------------------------------------------------------- */
/* small dense helpers                                                     */
/* ---------------------------------------------------------------------- */

static void unpack(const double *pk, double C[5][5])
{
    int k = 0;
    for (int i = 0; i < 5; i++)
        for (int j = i; j < 5; j++) {
            C[i][j] = pk[k];
            C[j][i] = pk[k];
            k++;
        }
}

static void pack(double C[5][5], double *pk)
{
    int k = 0;
    for (int i = 0; i < 5; i++)
        for (int j = i; j < 5; j++)
            pk[k++] = C[i][j];
}

/* C <- J C J^T, with full 5x5 products */
static void transport(double J[5][5], double C[5][5])
{
    double T[5][5], R[5][5];
    for (int i = 0; i < 5; i++)
        for (int j = 0; j < 5; j++) {
            double a = 0;
            for (int k = 0; k < 5; k++) a += J[i][k] * C[k][j];
            T[i][j] = a;
        }
    for (int i = 0; i < 5; i++)
        for (int j = 0; j < 5; j++) {
            double a = 0;
            for (int k = 0; k < 5; k++) a += T[i][k] * J[j][k];
            R[i][j] = a;
        }
    /* symmetrise exactly: the two halves differ only by rounding order */
    for (int i = 0; i < 5; i++)
        for (int j = i; j < 5; j++) {
            double v = 0.5 * (R[i][j] + R[j][i]);
            C[i][j] = v;
            C[j][i] = v;
        }
}

static void identity(double J[5][5])
{
    memset(J, 0, sizeof(double) * 25);
    for (int i = 0; i < 5; i++) J[i][i] = 1.0;
}

static double sinc(double u) { return u == 0.0 ? 1.0 : sin(u) / u; }

/* (sin d - d) / d^2, by its Taylor series where the direct form cancels */
static double g_of(double d)
{
    if (fabs(d) < 0.5) {
        double d2 = d * d, term = -d / 6.0, sum = 0.0;
        for (int k = 1; k <= 8; k++) {
            sum += term;
            term *= -d2 / ((2.0 * k + 2.0) * (2.0 * k + 3.0));
        }
        return sum;
    }
    return (sin(d) - d) / (d * d);
}

static int near_lim(double a, double lim, double rel, double abs_)
{
    return fabs(a - lim) <= rel * fabs(lim) + abs_;
}

/* ---------------------------------------------------------------------- */
/* helix propagation in the sector frame                                  */
/* ---------------------------------------------------------------------- */

/* Moves the state from *x to x2 along the helix.  Returns 0 (state
 * untouched) if |sin phi| would reach snp_max.  J (optional) receives the
 * Jacobian d p(x2) / d p(x). */
/* Bz (T) at a point of the sector frame: the field depends on the radius
 * r = sqrt(x^2 + y^2) (any frame) and on z. */
#define FIELD_RREF 370.0
#define FIELD_ZREF 360.0
static int field_map(const ocfg *g) { return g->field_br != 0.0 || g->field_bz != 0.0; }
static double field_at(const ocfg *g, double x, double y, double z)
{
    const double r2 = x * x + y * y;
    return g->bz * (1.0 + g->field_br * r2 / (FIELD_RREF * FIELD_RREF) + g->field_bz * z * z / (FIELD_ZREF * FIELD_ZREF));
}

/* Exact Jacobian (M2) of the helix step dx from sin(phi) = s1 with tan(lambda)
 * = t, q/pT = c in a uniform field with curvature coefficient k = -kappa Bz
 * (C = k c).  Also gives the step's dy and arc.  0 if |s2| >= 1. */
static int helix_jacobian(double s1, double t, double c, double dx, double k, double J[5][5], double *dyo,
                          double *arco)
{
    double cu = k * c;
    double s2 = s1 + cu * dx;
    if (!(fabs(s2) < 1.0)) return 0;
    double f1 = sqrt(1.0 - s1 * s1);
    double f2 = sqrt(1.0 - s2 * s2);
    /* transverse displacement: integral of tan(phi) dx, written without 1/C */
    double dy = dx * (s1 + s2) / (f1 + f2);
    /* arc length from the chord */
    double chord = sqrt(dx * dx + dy * dy);
    double h = 0.5 * fabs(cu) * chord;
    double arc = (dx >= 0 ? chord : -chord) * (h > 0 ? asin(h) / h : 1.0);
    double delta = cu * arc;              /* turning angle */
    identity(J);
    J[0][2] = arc * sinc(delta) / (f1 * f2);
    J[0][4] = k * dx * dx / (f1 + f2) * (1.0 + s2 * (s1 + s2) / (f2 * (f1 + f2)));
    J[1][2] = t * dy / (f1 * f2);
    J[1][3] = arc;
    {
        double sh = sinc(0.5 * delta);
        J[1][4] = k * t * arc * arc * ((s2 / f2) * sh * sh * 0.5 + g_of(delta));
    }
    J[2][4] = k * dx;
    *dyo = dy;
    *arco = arc;
    return 1;
}

/* derivative of (y, z, sin phi) with respect to x along the track, and the
 * field there */
static int rk_deriv(const ocfg *g, double x, const double v[3], double t, double c, double d[3], double *bz)
{
    if (!(fabs(v[2]) < 1.0)) return 0;
    double f = sqrt(1.0 - v[2] * v[2]);
    *bz = field_at(g, x, v[0], v[1]);
    d[0] = v[2] / f;
    d[1] = t / f;
    d[2] = -KAPPA * *bz * c;
    return 1;
}

/* Helix step in the sector frame from *x to x2 with its Jacobian applied to
 * C (if given).  Uniform field: the closed form (M1, M2).  Field map: the
 * most precise extrapolation step of Sect. 3 as a classical 4th-order Runge-Kutta
 * integration of y' = tan(phi), z' = tan(lambda)/cos(phi), sin(phi)' =
 * -kappa Bz(r, z) q/pT over equal x steps of at most field_step; the
 * covariance is transported with the exact helix Jacobian over the whole
 * step in the field the integration saw (the mean over the steps of the
 * Runge-Kutta weighted field samples, (B1 + 2 B2 + 2 B3 + B4) / 6).
 * Returns 0 (state untouched) if |sin phi| reaches snp_max. */
static int propagate(double p[5], double C[5][5], double *x, double x2,
                     const ocfg *g, unsigned *flags, double Jout[5][5])
{
    double dx = x2 - *x;
    double k = -KAPPA * g->bz;            /* d curvature / d (q/pT) */
    double J[5][5], dy, arc;
    if (!field_map(g)) {
        double s2 = p[2] + k * p[4] * dx;
        if (flags && near_lim(fabs(s2), g->snp_max, g->m_rel, g->m_snp)) *flags |= FL_P4;
        if (!(fabs(s2) < g->snp_max)) return 0;
        if (!helix_jacobian(p[2], p[3], p[4], dx, k, J, &dy, &arc)) return 0;
        p[0] += dy;
        p[1] += p[3] * arc;
        p[2] = s2;
        *x = x2;
        if (C) transport(J, C);
        if (Jout) memcpy(Jout, J, sizeof(J));
        return 1;
    }
    const int ns = (int)ceil(fabs(dx) / g->field_step);
    const double h = ns > 0 ? dx / ns : 0.0, x1 = *x, t = p[3], c = p[4], s1 = p[2];
    double bsum = 0.0, q[3] = {p[0], p[1], p[2]};
    for (int i = 0; i < ns; i++) {
        const double xa = x1 + i * h, xb = (i == ns - 1) ? x2 : x1 + (i + 1) * h;
        const double hs = xb - xa;
        double v[3] = {q[0], q[1], q[2]}, k1[3], k2[3], k3[3], k4[3], w[3], b1, b2, b3, b4;
        if (!rk_deriv(g, xa, v, t, c, k1, &b1)) return 0;
        for (int j = 0; j < 3; j++) w[j] = v[j] + 0.5 * hs * k1[j];
        if (!rk_deriv(g, xa + 0.5 * hs, w, t, c, k2, &b2)) return 0;
        for (int j = 0; j < 3; j++) w[j] = v[j] + 0.5 * hs * k2[j];
        if (!rk_deriv(g, xa + 0.5 * hs, w, t, c, k3, &b3)) return 0;
        for (int j = 0; j < 3; j++) w[j] = v[j] + hs * k3[j];
        if (!rk_deriv(g, xb, w, t, c, k4, &b4)) return 0;
        for (int j = 0; j < 3; j++) q[j] = v[j] + hs / 6.0 * (k1[j] + 2.0 * k2[j] + 2.0 * k3[j] + k4[j]);
        bsum += (b1 + 2.0 * b2 + 2.0 * b3 + b4) / 6.0;
        if (flags && near_lim(fabs(q[2]), g->snp_max, g->m_rel, g->m_snp)) *flags |= FL_P4;
        if (!(fabs(q[2]) < g->snp_max)) return 0;
    }
    if (ns > 0) k = -KAPPA * bsum / ns;
    if (!helix_jacobian(s1, t, c, dx, k, J, &dy, &arc)) return 0;
    for (int j = 0; j < 3; j++) p[j] = q[j];
    *x = x2;
    if (C) transport(J, C);
    if (Jout) memcpy(Jout, J, sizeof(J));
    return 1;
}

/* Rotates the frame by da (alpha' = alpha + da) at the current point.
 * Returns 0 if the track would move inwards in the new frame. */
static int rotate(double p[5], double C[5][5], double *x, double da,
                  const ocfg *g, double Jout[5][5])
{
    double ca = cos(da), sa = sin(da);
    double s = p[2], f = sqrt(1.0 - s * s);
    double s1 = s * ca - f * sa;
    double f1 = f * ca + s * sa;
    if (!(f1 > 0.0)) return 0;
    double x1 = *x * ca + p[0] * sa;
    double y1 = -*x * sa + p[0] * ca;
    double cu = -KAPPA * (field_map(g) ? field_at(g, *x, p[0], p[1]) : g->bz) * p[4];
    double J[5][5];
    identity(J);
    J[0][0] = f / f1;
    J[1][0] = -sa * p[3] / f1;
    J[2][0] = -cu * sa;
    J[2][2] = f1 / f;
    p[0] = y1;
    p[2] = s1;
    *x = x1;
    if (C) transport(J, C);
    if (Jout) memcpy(Jout, J, sizeof(J));
    return 1;
}

/* Thin scatterer of thickness x_over_x0 crossed at the current point. */
static void add_ms(const double p[5], double C[5][5], const ocfg *g)
{
    double s = p[2], t = p[3], c = p[4];
    if (c == 0.0 || g->x_over_x0 <= 0.0) return;
    double f = sqrt(1.0 - s * s);
    double tt = 1.0 + t * t;
    double pp = sqrt(tt) / fabs(c);
    double beta = pp / sqrt(pp * pp + g->mass * g->mass);
    double xi = g->x_over_x0 * sqrt(tt) / f;
    double th0 = 0.0136 / (beta * pp) * sqrt(xi) * (1.0 + 0.038 * log(xi));
    double th2 = th0 * th0;
    C[2][2] += th2 * f * f * tt;
    C[3][3] += th2 * tt * tt;
    C[4][4] += th2 * c * c * t * t;
    C[3][4] += th2 * tt * c * t;
    C[4][3] = C[3][4];
}

/* Mean energy loss rate of a unit-charge particle of momentum p and mass m
 * in the layer material: the Bethe formula without density-effect or shell
 * corrections, with the kinematic maximum energy transfer to one electron;
 * GeV cm^2/g, never below zero. */
static double bethe(double p, double m, const ocfg *g)
{
    const double K = 0.307075e-3, me = 0.51099895e-3;
    double E = sqrt(p * p + m * m);
    double bg = p / m, gam = E / m, b2 = (p * p) / (E * E), r = me / m;
    double tmax = 2.0 * me * bg * bg / (1.0 + 2.0 * gam * r + r * r);
    double v = K * g->eloss_za / b2 * (0.5 * log(2.0 * me * bg * bg * tmax / (g->eloss_i * g->eloss_i)) - b2);
    return v > 0.0 ? v : 0.0;
}

/* The layer's mean energy loss at the current point, along the path
 * x_rho sqrt(1 + tan^2 lambda) / cos(phi).  Outward (dir = +1) the energy
 * falls by it, inward (dir = -1) it is given back; the rate is taken at the
 * momentum before the step.  q/pT scales by p/p'.  Its covariance row and
 * column scale by d(q/pT')/d(q/pT) with the loss held fixed, (p/p')^3 E'/E,
 * and the diagonal element by the square.  Returns 0 (state untouched) if
 * the energy would not exceed the mass.  Outward, a kinetic energy left
 * within the margin m_ke of what it was raises FL_P4 in *lf: there the stop
 * decision and the new momentum hinge on the last digits of the loss. */
static int eloss(double p[5], double C[5][5], const ocfg *g, int dir, unsigned *lf)
{
    double s = p[2], t = p[3], c = p[4];
    if (c == 0.0 || !(g->eloss_xrho > 0.0)) return 1;
    double f = sqrt(1.0 - s * s), tt = 1.0 + t * t;
    double pp = sqrt(tt) / fabs(c), m = g->mass;
    double E = sqrt(pp * pp + m * m);
    double dE = bethe(pp, m, g) * g->eloss_xrho * sqrt(tt) / f;
    double E2 = dir > 0 ? E - dE : E + dE;
    if (lf && dir > 0 && fabs(E2 - m) <= g->m_ke * (E - m)) *lf |= FL_P4;
    if (!(E2 > m)) return 0;
    double p2 = sqrt(E2 * E2 - m * m);
    double k = pp / p2;
    double j = k * k * k * E2 / E;
    p[4] = c * k;
    for (int a = 0; a < 4; a++) {
        C[4][a] *= j;
        C[a][4] *= j;
    }
    C[4][4] *= j * j;
    return 1;
}

/* Chamber slot holding the point (sector, z) of layer l: -1 outside the
 * stacks in z. */
static int chamber_at(const ocfg *g, int sec, int l, double z)
{
    double row = floor((z - g->z_min) / g->pad_len);
    if (!(row >= 0.0) || row >= (double)(NSTK * g->n_rows)) return -1;
    return sec * (NSTK * NLAY) + ((int)row / g->n_rows) * NLAY + l;
}

/* Kalman update with the measurement m = (y_tkl, z_tkl) of the model
 * h(p) = (y + tau (z - z_tkl), z); r = m - h(p).  Joseph form. */
static void kalman_update(double p[5], double C[5][5], double ry, double rz,
                          double tau, double vy, double vz)
{
    double H[2][5] = {{1, tau, 0, 0, 0}, {0, 1, 0, 0, 0}};
    double V[2][2] = {{vy, 0}, {0, vz}};
    double CHt[5][2], S[2][2], Si[2][2], K[5][2];
    for (int i = 0; i < 5; i++)
        for (int a = 0; a < 2; a++) {
            double v = 0;
            for (int k = 0; k < 5; k++) v += C[i][k] * H[a][k];
            CHt[i][a] = v;
        }
    for (int a = 0; a < 2; a++)
        for (int b = 0; b < 2; b++) {
            double v = V[a][b];
            for (int k = 0; k < 5; k++) v += H[a][k] * CHt[k][b];
            S[a][b] = v;
        }
    double det = S[0][0] * S[1][1] - S[0][1] * S[1][0];
    Si[0][0] = S[1][1] / det;
    Si[1][1] = S[0][0] / det;
    Si[0][1] = -S[0][1] / det;
    Si[1][0] = -S[1][0] / det;
    for (int i = 0; i < 5; i++)
        for (int b = 0; b < 2; b++)
            K[i][b] = CHt[i][0] * Si[0][b] + CHt[i][1] * Si[1][b];
    for (int i = 0; i < 5; i++) p[i] += K[i][0] * ry + K[i][1] * rz;

    double A[5][5], T[5][5], R[5][5];
    for (int i = 0; i < 5; i++)
        for (int j = 0; j < 5; j++)
            A[i][j] = (i == j ? 1.0 : 0.0) - (K[i][0] * H[0][j] + K[i][1] * H[1][j]);
    for (int i = 0; i < 5; i++)
        for (int j = 0; j < 5; j++) {
            double v = 0;
            for (int k = 0; k < 5; k++) v += A[i][k] * C[k][j];
            T[i][j] = v;
        }
    for (int i = 0; i < 5; i++)
        for (int j = 0; j < 5; j++) {
            double v = 0;
            for (int k = 0; k < 5; k++) v += T[i][k] * A[j][k];
            for (int a = 0; a < 2; a++)
                for (int b = 0; b < 2; b++) v += K[i][a] * V[a][b] * K[j][b];
            R[i][j] = v;
        }
    for (int i = 0; i < 5; i++)
        for (int j = i; j < 5; j++) {
            double v = 0.5 * (R[i][j] + R[j][i]);
            C[i][j] = v;
            C[j][i] = v;
        }
}

/* Positive definiteness by an LDL^T factorisation. */
static int ldl_pd(double C[5][5])
{
    double L[5][5] = {{0}}, d[5];
    for (int j = 0; j < 5; j++) {
        double v = C[j][j];
        for (int k = 0; k < j; k++) v -= L[j][k] * L[j][k] * d[k];
        if (!(v > 0.0)) return 0;
        d[j] = v;
        L[j][j] = 1.0;
        for (int i = j + 1; i < 5; i++) {
            double w = C[i][j];
            for (int k = 0; k < j; k++) w -= L[i][k] * L[j][k] * d[k];
            L[i][j] = w / v;
        }
    }
    return 1;
}

static double poly2(const double a[3], double s) { return a[0] + a[1] * s + a[2] * s * s; }

/* ---------------------------------------------------------------------- */
/* tracklet cells                                                          */
/* ---------------------------------------------------------------------- */

static int64_t n_cells_of(const ocfg *g, int32_t n_groups)
{
    return (int64_t)n_groups * NDET * g->n_rows * g->n_db * g->n_yb;
}

/* bin of v among n bins of width w centred on 0, outer bins open */
static int bin_of(double v, double w, int n)
{
    double lo = -w * n / 2.0;
    double u = floor((v - lo) * (1.0 / w));
    if (!(u >= 0)) return 0;
    if (u > n - 1) return n - 1;
    return (int)u;
}

static int ybin_of(const ocfg *g, double y) { return bin_of(y, g->y_bin_w, g->n_yb); }
static int dbin_of(const ocfg *g, double dy) { return bin_of(dy, g->dy_bin_w, g->n_db); }

/* Cell key of one tracklet; the invalid ones get n_cells (placed last). */
static int64_t tkl_key(const ocfg *g, double y, double z, double dy, uint32_t det_row,
                       int32_t grp, int32_t n_groups)
{
    uint32_t det = det_row >> 5, row = det_row & 31u;
    if (det >= NDET || (int32_t)row >= g->n_rows || grp < 0 || grp >= n_groups ||
        !isfinite(y) || !isfinite(z) || !isfinite(dy) || g->absent[det])
        return n_cells_of(g, n_groups);
    return ((((int64_t)grp * NDET + det) * g->n_db + dbin_of(g, dy)) * g->n_yb + ybin_of(g, y)) *
               g->n_rows + row;
}

typedef struct { int64_t key; int64_t idx; } keyidx;

static int cmp_keyidx(const void *a, const void *b)
{
    const keyidx *u = (const keyidx *)a, *v = (const keyidx *)b;
    if (u->key != v->key) return u->key < v->key ? -1 : 1;
    if (u->idx != v->idx) return u->idx < v->idx ? -1 : 1;
    return 0;
}

/* Stable counting sort by cell: perm[] lists input indices in (key, index)
 * order; offsets[c] is the first sorted position of cell c and
 * offsets[n_cells] the number of valid tracklets. */
int oracle_bin(const ocfg *g, int64_t n, const double *y, const double *z, const double *dy,
               const uint32_t *det_row, const int32_t *grp, int32_t n_groups,
               int32_t *perm, uint32_t *offsets)
{
    int64_t nc = n_cells_of(g, n_groups);
    keyidx *ki = (keyidx *)malloc(sizeof(keyidx) * (size_t)(n > 0 ? n : 1));
    if (!ki) return -2;
    for (int64_t i = 0; i < n; i++) {
        ki[i].key = tkl_key(g, y[i], z[i], dy[i], det_row[i], grp ? grp[i] : 0, n_groups);
        ki[i].idx = i;
    }
    qsort(ki, (size_t)n, sizeof(keyidx), cmp_keyidx);
    for (int64_t c = 0; c <= nc; c++) offsets[c] = 0;
    for (int64_t i = 0; i < n; i++) {
        perm[i] = (int32_t)ki[i].idx;
        if (ki[i].key < nc) offsets[ki[i].key + 1]++;
    }
    for (int64_t c = 0; c < nc; c++) offsets[c + 1] += offsets[c];
    free(ki);
    return 0;
}

/* ---------------------------------------------------------------------- */
/* per-track matching                                                      */
/* ---------------------------------------------------------------------- */

typedef struct {
    const double *y, *z, *dy;
    const uint32_t *det_row;
    const int32_t *grp;
    int64_t n;
    const int32_t *perm;     /* binned mode */
    const uint32_t *offsets; /* binned mode */
    int32_t n_groups;
    int brute;
} otkl;

typedef struct {
    int32_t *idx;          /* [6][n] */
    double *p, *c, *x;     /* [5][n], [15][n], [n] */
    int32_t *sec;
    double *chi2, *chi2_layer;   /* [n], [6][n] (optional) */
    int32_t *n_match;
    uint32_t *status, *flags;
    int32_t *flag_layer;   /* optional: first layer holding a flag, 6 if none */
    int64_t *n_cand;       /* optional: candidates looked at */
    double *lp, *lc, *lx;  /* optional per-layer state: [6][5][n], [6][15][n], [6][n] */
    int32_t *lsec;         /* optional [6][n] */
    double *cost;          /* optional [n]: cost of the answer (hypothesis mode; NaN otherwise) */
} oout;

/* prediction-side quantities of one layer's road */
typedef struct {
    double y, z, s, t, f, tphi, tz, tau;
    double Ry, Rz, gdy, dytrk;
    double Si[2][2];
    double kchi;   /* chi2 error scale of this road, see road_chi2_scale */
} road_t;

/* A predicted state whose y, z carry errors up to m_state max(|.|, 10 cm) and
 * whose sin(phi), tan(lambda) carry errors up to m_state max(|.|, 0.1) moves
 * the residual r = (r_y, r_z) of a candidate at most dxmax away in x by at
 * most e = (e_y + |tau| e_z, e_z), with e_y, e_z the errors of the linearly
 * extrapolated point; a candidate's chi2 = r' S^-1 r then moves by at most
 * 2 |S^-1/2 r| |S^-1/2 e| + |S^-1/2 e|^2 <= kchi sqrt(chi2) + kchi^2 / 4 with
 * kchi = 2 |e| / sqrt(lambda_min(S)). */
static void road_chi2_scale(const ocfg *g, road_t *r, double Syy, double Syz, double Szz, double dxmax)
{
    r->kchi = 0.0;
    if (!(g->m_state > 0.0)) return;
    const double ds = g->m_state * fmax(fabs(r->s), 0.1), dt = g->m_state * fmax(fabs(r->t), 0.1);
    const double f3 = r->f * r->f * r->f;
    const double ez = g->m_state * fmax(fabs(r->z), 10.0) + dxmax * (dt / r->f + fabs(r->t * r->s) * ds / f3);
    const double ey = g->m_state * fmax(fabs(r->y), 10.0) + dxmax * ds / f3 + fabs(r->tau) * ez;
    const double h = 0.5 * (Syy - Szz);
    const double lmin = 0.5 * (Syy + Szz) - sqrt(h * h + Syz * Syz);
    r->kchi = lmin > 0.0 ? 2.0 * sqrt(ey * ey + ez * ez) / sqrt(lmin) : INFINITY;
}

static double chi2_err(const road_t *r, double c2)
{
    return r->kchi * sqrt(fmax(c2, 0.0)) + 0.25 * r->kchi * r->kchi;
}

/* Evaluates one candidate.  fail: bit0 y road, bit1 z road, bit2 dy gate,
 * bit3 chi2 cut; nearm: same bits when the value lies within the margin of
 * its limit. */
static void eval_cand(const ocfg *g, const road_t *r, double yj, double zj, double dyj, double dxj,
                      double *chi2, unsigned *fail, unsigned *nearm)
{
    double ye = r->y + dxj * r->tphi;
    double ze = r->z + dxj * r->tz;
    double ry = yj - (ye + r->tau * (ze - zj));
    double rz = zj - ze;
    double ddy = dyj - r->dytrk;
    double c2 = r->Si[0][0] * ry * ry + 2.0 * r->Si[0][1] * ry * rz + r->Si[1][1] * rz * rz;
    unsigned f = 0, nm = 0;
    if (!(fabs(ry) <= r->Ry)) f |= 1u;
    if (!(fabs(rz) <= r->Rz)) f |= 2u;
    if (!(fabs(ddy) <= r->gdy)) f |= 4u;
    if (!(c2 <= g->chi2_max)) f |= 8u;
    if (near_lim(fabs(ry), r->Ry, g->m_rel, g->m_len)) nm |= 1u;
    if (near_lim(fabs(rz), r->Rz, g->m_rel, g->m_len)) nm |= 2u;
    if (near_lim(fabs(ddy), r->gdy, g->m_rel, g->m_dy)) nm |= 4u;
    if (near_lim(c2, g->chi2_max, g->m_rel, g->m_chi2 + chi2_err(r, g->chi2_max))) nm |= 8u;
    *chi2 = c2;
    *fail = f;
    *nearm = nm;
}

static int popcount4(unsigned v) { return (v & 1) + ((v >> 1) & 1) + ((v >> 2) & 1) + ((v >> 3) & 1); }

/* candidate list of one layer (indices into the input tracklet arrays) */
typedef struct { int64_t *v; int64_t n, cap; } ilist;

static void ilist_push(ilist *L, int64_t j)
{
    if (L->n == L->cap) {
        L->cap = L->cap ? 2 * L->cap : 256;
        L->v = (int64_t *)realloc(L->v, sizeof(int64_t) * (size_t)L->cap);
    }
    L->v[L->n++] = j;
}

static void gather_candidates(const ocfg *g, const otkl *T, const road_t *r, int grp, int sec, int l,
                              double dxmax, ilist *L)
{
    L->n = 0;
    if (T->brute) {
        for (int64_t j = 0; j < T->n; j++) {
            uint32_t det = T->det_row[j] >> 5, row = T->det_row[j] & 31u;
            int32_t gj = T->grp ? T->grp[j] : 0;
            if (det >= NDET || (int32_t)row >= g->n_rows || gj != grp || g->absent[det]) continue;
            if (!isfinite(T->y[j]) || !isfinite(T->z[j]) || !isfinite(T->dy[j])) continue;
            if ((int)(det / (NSTK * NLAY)) != sec || (int)(det % NLAY) != l) continue;
            ilist_push(L, j);
        }
        return;
    }
    /* cells whose pad rows and y bins overlap the road (plus margins that
     * cover misalignment, tilt and the decision margins) */
    double slack_y = 2.0 * (g->m_rel * r->Ry + g->m_len) + 1e-3;
    double slack_z = 2.0 * (g->m_rel * r->Rz + g->m_len) + 1e-3;
    double slack_d = 2.0 * (g->m_rel * r->gdy + g->m_dy) + 1e-4;
    double mz = dxmax * fabs(r->tz);
    double my = fabs(r->tau) * (r->Rz + mz + slack_z) + dxmax * fabs(r->tphi);
    double zlo = r->z - r->Rz - mz - slack_z, zhi = r->z + r->Rz + mz + slack_z;
    double ylo = r->y - r->Ry - my - slack_y, yhi = r->y + r->Ry + my + slack_y;
    int nrt = NSTK * g->n_rows;
    double glo = floor((zlo - g->z_min) / g->pad_len), ghi = floor((zhi - g->z_min) / g->pad_len);
    if (glo < 0) glo = 0;
    if (ghi > nrt - 1) ghi = nrt - 1;
    int yb0 = ybin_of(g, ylo), yb1 = ybin_of(g, yhi);
    int db0 = dbin_of(g, r->dytrk - r->gdy - slack_d), db1 = dbin_of(g, r->dytrk + r->gdy + slack_d);
    for (int stack = (int)glo / g->n_rows; stack <= (int)ghi / g->n_rows; stack++) {
        int r0 = (int)glo - stack * g->n_rows, r1 = (int)ghi - stack * g->n_rows;
        if (r0 < 0) r0 = 0;
        if (r1 > g->n_rows - 1) r1 = g->n_rows - 1;
        int det = sec * (NSTK * NLAY) + stack * NLAY + l;
        if (g->absent[det]) continue;
        for (int db = db0; db <= db1; db++)
            for (int yb = yb0; yb <= yb1; yb++) {
                int64_t base = ((((int64_t)grp * NDET + det) * g->n_db + db) * g->n_yb + yb) * g->n_rows;
                uint32_t a = T->offsets[base + r0], b = T->offsets[base + r1 + 1];
                for (uint32_t k = a; k < b; k++) ilist_push(L, T->perm[k]);
            }
    }
}

static void match_one(const ocfg *g, int64_t i, int64_t n, const double *ip, const double *ic,
                      const double *ix, const int32_t *isec, const int32_t *igrp, const otkl *T,
                      double dxmax, const oout *o, ilist *L)
{
    double p[5], C[5][5], pk[15], x = ix[i];
    for (int k = 0; k < 5; k++) p[k] = ip[k * n + i];
    for (int k = 0; k < 15; k++) pk[k] = ic[k * n + i];
    unpack(pk, C);
    int sec = isec[i], grp = igrp ? igrp[i] : 0;
    unsigned status = 0, flags = 0;
    int flag_layer = NLAY, nmatch = 0;
    double chi2sum = 0.0;
    int64_t ncand = 0;
    const double tan10 = tan(M_PI / NSEC), dphi = 2.0 * M_PI / NSEC;
    for (int l = 0; l < NLAY; l++) {
        o->idx[l * n + i] = -1;
        if (o->chi2_layer) o->chi2_layer[l * n + i] = 0.0;
        if (o->lx) o->lx[l * n + i] = NAN;
        if (o->lsec) o->lsec[l * n + i] = -1;
    }

    int bad = !(isfinite(x) && sec >= 0 && sec < NSEC && grp >= 0 && grp < T->n_groups);
    for (int k = 0; k < 5; k++) bad |= !isfinite(p[k]);
    for (int k = 0; k < 15; k++) bad |= !isfinite(pk[k]);
    if (!bad) bad = !(fabs(p[2]) < g->snp_max) || !ldl_pd(C);
    if (bad) {
        status = ST_BAD_INPUT;
        goto done;
    }

    for (int l = 0; l < NLAY; l++) {
        unsigned lf = 0;
        double xl = g->x_layer[l];
        if (!propagate(p, C, &x, xl, g, &lf, NULL)) {
            status |= ST_STOP_SNP;
            flags |= lf;
            if (lf && flag_layer == NLAY) flag_layer = l;
            break;
        }
        /* sector containing the point (at most two hops) */
        int stop = 0;
        for (int nrot = 0;; nrot++) {
            double ylim = xl * tan10;
            if (near_lim(fabs(p[0]), ylim, g->m_rel, g->m_len)) lf |= FL_P4;
            if (fabs(p[0]) <= ylim) break;
            if (nrot == 2) { status |= ST_ROT_FAIL; stop = 1; break; }
            int up = p[0] > 0;
            if (!rotate(p, C, &x, up ? dphi : -dphi, g, NULL)) { status |= ST_ROT_FAIL; stop = 1; break; }
            sec = (sec + (up ? 1 : NSEC - 1)) % NSEC;
            if (!propagate(p, C, &x, xl, g, &lf, NULL)) { status |= ST_STOP_SNP; stop = 1; break; }
        }
        if (!stop) {
            add_ms(p, C, g);
            if (!eloss(p, C, g, 1, &lf)) {
                status |= ST_STOPPED;
                stop = 1;
            }
        }
        if (stop) {
            flags |= lf;
            if (lf && flag_layer == NLAY) flag_layer = l;
            break;
        }

        /* road from the covariance */
        road_t r;
        r.y = p[0]; r.z = p[1]; r.s = p[2]; r.t = p[3];
        r.f = sqrt(1.0 - r.s * r.s);
        r.tphi = r.s / r.f;
        r.tz = r.t / r.f;
        r.tau = g->tilt[l];
        double sy = poly2(g->sigma_y, r.s);
        double vy = sy * sy, vz = g->pad_len * g->pad_len / 12.0;
        double Syy = C[0][0] + 2.0 * r.tau * C[0][1] + r.tau * r.tau * C[1][1] + vy;
        double Syz = C[0][1] + r.tau * C[1][1];
        double Szz = C[1][1] + vz;
        double det = Syy * Szz - Syz * Syz;
        r.Si[0][0] = Szz / det;
        r.Si[1][1] = Syy / det;
        r.Si[0][1] = r.Si[1][0] = -Syz / det;
        r.Ry = g->n_sigma_road * sqrt(Syy);
        r.Rz = g->n_sigma_road * sqrt(Szz);
        r.dytrk = g->drift_len * (r.tphi - g->tan_psi);
        road_chi2_scale(g, &r, Syy, Syz, Szz, dxmax);
        {
            double sdy = poly2(g->sigma_dy, r.s);
            double f3 = r.f * r.f * r.f;
            r.gdy = g->n_sigma_dy * sqrt(sdy * sdy + g->drift_len * g->drift_len * C[2][2] / (f3 * f3));
        }

        /* z acceptance of the whole search window */
        double mz = dxmax * fabs(r.tz);
        double wlo = r.z - r.Rz - mz, whi = r.z + r.Rz + mz, zmax = -g->z_min;
        if (near_lim(whi, g->z_min, g->m_rel, g->m_len) || near_lim(wlo, zmax, g->m_rel, g->m_len)) lf |= FL_P4;
        if (whi < g->z_min || wlo > zmax) {
            status |= ST_OUT_OF_Z;
        } else {
            gather_candidates(g, T, &r, grp, sec, l, dxmax, L);
            ncand += L->n;
            int64_t best = -1, best_orig = -1;
            double bchi = 0.0, second = INFINITY;
            unsigned bnear = 0;
            for (int64_t a = 0; a < L->n; a++) {
                int64_t j = L->v[a];
                double c2;
                unsigned fail, nm;
                eval_cand(g, &r, T->y[j], T->z[j], T->dy[j], g->dx_chamber[T->det_row[j] >> 5], &c2, &fail, &nm);
                if (fail) continue;
                if (best < 0 || c2 < bchi || (c2 == bchi && j < best_orig)) {
                    if (best >= 0) second = bchi < second ? bchi : second;
                    best = a; best_orig = j; bchi = c2; bnear = nm;
                } else if (c2 < second) {
                    second = c2;
                }
            }
            if (best >= 0) {
                if (bnear) lf |= FL_P1;
                if (bnear & 8u) lf |= FL_KCUT;
                if (bnear & 7u) lf |= FL_KGATE;
                if (isfinite(second) &&
                    second - bchi <= g->m_rel * bchi + g->m_chi2 + chi2_err(&r, bchi) + chi2_err(&r, second))
                    lf |= FL_P3;
            }
            /* a rejected candidate one marginal gate away from winning */
            for (int64_t a = 0; a < L->n; a++) {
                int64_t j = L->v[a];
                double c2;
                unsigned fail, nm;
                eval_cand(g, &r, T->y[j], T->z[j], T->dy[j], g->dx_chamber[T->det_row[j] >> 5], &c2, &fail, &nm);
                if (!fail || popcount4(fail) != 1 || !(fail & nm)) continue;
                if (best < 0 || c2 <= bchi + g->m_rel * bchi + g->m_chi2 + chi2_err(&r, bchi) + chi2_err(&r, c2))
                    lf |= FL_P2 | ((fail & 8u) ? FL_KCUT : FL_KGATE);
            }
            if (best >= 0) {
                int64_t j = best_orig;
                double dxj = g->dx_chamber[T->det_row[j] >> 5];
                if (dxj != 0.0) {
                    if (!propagate(p, C, &x, xl + dxj, g, &lf, NULL)) {
                        status |= ST_STOP_SNP;
                        flags |= lf;
                        if (lf && flag_layer == NLAY) flag_layer = l;
                        break;
                    }
                }
                double ry = T->y[j] - (p[0] + r.tau * (p[1] - T->z[j]));
                double rz = T->z[j] - p[1];
                double syu = poly2(g->sigma_y, p[2]);
                kalman_update(p, C, ry, rz, r.tau, syu * syu, vz);
                o->idx[l * n + i] = (int32_t)j;
                nmatch++;
                chi2sum += bchi;
                if (o->chi2_layer) o->chi2_layer[l * n + i] = bchi;
                if (near_lim(fabs(p[2]), g->snp_max, g->m_rel, g->m_snp)) lf |= FL_P4;
                if (!(fabs(p[2]) < g->snp_max)) {
                    status |= ST_STOP_SNP;
                    flags |= lf;
                    if (lf && flag_layer == NLAY) flag_layer = l;
                    break;
                }
            }
        }
        flags |= lf;
        if (lf && flag_layer == NLAY) flag_layer = l;
        if (o->lp) {
            double q[15];
            pack(C, q);
            for (int k = 0; k < 5; k++) o->lp[(l * 5 + k) * n + i] = p[k];
            for (int k = 0; k < 15; k++) o->lc[(l * 15 + k) * n + i] = q[k];
            o->lx[l * n + i] = x;
            o->lsec[l * n + i] = sec;
        }
    }
done:
    pack(C, pk);
    for (int k = 0; k < 5; k++) o->p[k * n + i] = p[k];
    for (int k = 0; k < 15; k++) o->c[k * n + i] = pk[k];
    o->x[i] = x;
    o->sec[i] = sec;
    o->chi2[i] = chi2sum;
    o->n_match[i] = nmatch;
    o->status[i] = status;
    o->flags[i] = flags;
    if (o->flag_layer) o->flag_layer[i] = flag_layer;
    if (o->n_cand) o->n_cand[i] = ncand;
    if (o->cost) o->cost[i] = NAN;
}

/* ---------------------------------------------------------------------- */
/* several hypotheses per track (Sect. 3 and Fig. 2: the best N_candidates */
/* hypotheses of a layer are the seeds of the next one)                    */
/* ---------------------------------------------------------------------- */

/* Readings where the paper is silent:
 *   - a hypothesis is one path through the layers; its cost is the sum of
 *     the chi2 of its tracklets plus chi2_penalty for every layer where it
 *     takes none;
 *   - every hypothesis has, at every layer, one child per candidate passing
 *     all gates of its own road and one child without a tracklet (also when
 *     it is outside the chambers or has stopped: it then only carries its
 *     cost forward);
 *   - the children of all hypotheses are ordered by (cost, with-tracklet
 *     before without, parent rank, tracklet index) and the first n_hyp
 *     survive; a child with a tracklet is then propagated precisely to it and
 *     updated exactly as in the single-hypothesis matcher;
 *   - the answer is the first hypothesis after the last layer.
 * With n_hyp = 1 and chi2_penalty >= chi2_max this is the single best
 * candidate rule. */

#define MAX_HYP 16

typedef struct {
    double p[5], C[5][5], x;
    int sec, live, nmatch;
    unsigned status;
    double cost, chi2sum;
    int32_t idx[NLAY];
    double chi2l[NLAY];
} hyp_t;

typedef struct {
    double cost, chi2;
    int parent;   /* rank of the parent hypothesis */
    int64_t j;    /* tracklet, -1: none at this layer */
} child_t;

typedef struct { child_t *v; int64_t n, cap; } clist;

static void clist_push(clist *L, double cost, double chi2, int parent, int64_t j)
{
    if (L->n == L->cap) {
        L->cap = L->cap ? 2 * L->cap : 64;
        L->v = (child_t *)realloc(L->v, sizeof(child_t) * (size_t)L->cap);
    }
    child_t c = {cost, chi2, parent, j};
    L->v[L->n++] = c;
}

static int cmp_child(const void *a, const void *b)
{
    const child_t *u = (const child_t *)a, *v = (const child_t *)b;
    if (u->cost != v->cost) return u->cost < v->cost ? -1 : 1;
    int nu = u->j < 0, nv = v->j < 0;
    if (nu != nv) return nu - nv;
    if (u->parent != v->parent) return u->parent < v->parent ? -1 : 1;
    if (u->j != v->j) return u->j < v->j ? -1 : 1;
    return 0;
}

/* Propagation to layer l, sector hops and the layer's scattering. */
static int hyp_predict(const ocfg *g, hyp_t *h, int l, unsigned *lf)
{
    const double tan10 = tan(M_PI / NSEC), dphi = 2.0 * M_PI / NSEC;
    double xl = g->x_layer[l];
    if (!propagate(h->p, h->C, &h->x, xl, g, lf, NULL)) {
        h->status |= ST_STOP_SNP;
        return 0;
    }
    for (int nrot = 0;; nrot++) {
        double ylim = xl * tan10;
        if (near_lim(fabs(h->p[0]), ylim, g->m_rel, g->m_len)) *lf |= FL_P4;
        if (fabs(h->p[0]) <= ylim) break;
        if (nrot == 2) { h->status |= ST_ROT_FAIL; return 0; }
        int up = h->p[0] > 0;
        if (!rotate(h->p, h->C, &h->x, up ? dphi : -dphi, g, NULL)) { h->status |= ST_ROT_FAIL; return 0; }
        h->sec = (h->sec + (up ? 1 : NSEC - 1)) % NSEC;
        if (!propagate(h->p, h->C, &h->x, xl, g, lf, NULL)) { h->status |= ST_STOP_SNP; return 0; }
    }
    add_ms(h->p, h->C, g);
    if (!eloss(h->p, h->C, g, 1, lf)) {
        h->status |= ST_STOPPED;
        return 0;
    }
    return 1;
}

/* Road of a predicted hypothesis (same quantities as the single matcher). */
static void hyp_road(const ocfg *g, const hyp_t *h, int l, double dxmax, road_t *r)
{
    r->y = h->p[0]; r->z = h->p[1]; r->s = h->p[2]; r->t = h->p[3];
    r->f = sqrt(1.0 - r->s * r->s);
    r->tphi = r->s / r->f;
    r->tz = r->t / r->f;
    r->tau = g->tilt[l];
    double sy = poly2(g->sigma_y, r->s);
    double vz = g->pad_len * g->pad_len / 12.0;
    double Syy = h->C[0][0] + 2.0 * r->tau * h->C[0][1] + r->tau * r->tau * h->C[1][1] + sy * sy;
    double Syz = h->C[0][1] + r->tau * h->C[1][1];
    double Szz = h->C[1][1] + vz;
    double det = Syy * Szz - Syz * Syz;
    r->Si[0][0] = Szz / det;
    r->Si[1][1] = Syy / det;
    r->Si[0][1] = r->Si[1][0] = -Syz / det;
    r->Ry = g->n_sigma_road * sqrt(Syy);
    r->Rz = g->n_sigma_road * sqrt(Szz);
    r->dytrk = g->drift_len * (r->tphi - g->tan_psi);
    road_chi2_scale(g, r, Syy, Syz, Szz, dxmax);
    double sdy = poly2(g->sigma_dy, r->s);
    double f3 = r->f * r->f * r->f;
    r->gdy = g->n_sigma_dy * sqrt(sdy * sdy + g->drift_len * g->drift_len * h->C[2][2] / (f3 * f3));
}

/* A candidate near the edge of the kept set: its cost, and whether a gate
 * decision on it lies within the margins. */
typedef struct { double cost; int passed; } edge_t;

static void match_one_beam(const ocfg *g, int64_t i, int64_t n, const double *ip, const double *ic,
                           const double *ix, const int32_t *isec, const int32_t *igrp, const otkl *T,
                           double dxmax, const oout *o, ilist *L, clist *K, clist *E)
{
    const int N = g->n_hyp < MAX_HYP ? g->n_hyp : MAX_HYP;
    hyp_t H[MAX_HYP], Hn[MAX_HYP];
    int nh = 1;
    unsigned flags = 0;
    int64_t ncand = 0;
    const double vz = g->pad_len * g->pad_len / 12.0;
    hyp_t *h0 = &H[0];
    memset(h0, 0, sizeof(*h0));
    double pk[15];
    for (int k = 0; k < 5; k++) h0->p[k] = ip[k * n + i];
    for (int k = 0; k < 15; k++) pk[k] = ic[k * n + i];
    unpack(pk, h0->C);
    h0->x = ix[i];
    h0->sec = isec[i];
    int grp = igrp ? igrp[i] : 0;
    for (int l = 0; l < NLAY; l++) { h0->idx[l] = -1; h0->chi2l[l] = 0.0; }
    int bad = !(isfinite(h0->x) && h0->sec >= 0 && h0->sec < NSEC && grp >= 0 && grp < T->n_groups);
    for (int k = 0; k < 5; k++) bad |= !isfinite(h0->p[k]);
    for (int k = 0; k < 15; k++) bad |= !isfinite(pk[k]);
    if (!bad) bad = !(fabs(h0->p[2]) < g->snp_max) || !ldl_pd(h0->C);
    if (bad) {
        h0->status = ST_BAD_INPUT;
        goto done;
    }
    h0->live = 1;

    for (int l = 0; l < NLAY; l++) {
        K->n = 0;
        E->n = 0;
        for (int h = 0; h < nh; h++) {
            hyp_t *Hh = &H[h];
            if (Hh->live) Hh->live = hyp_predict(g, Hh, l, &flags);
            if (Hh->live) {
                road_t r;
                hyp_road(g, Hh, l, dxmax, &r);
                double mz = dxmax * fabs(r.tz);
                double wlo = r.z - r.Rz - mz, whi = r.z + r.Rz + mz, zmax = -g->z_min;
                if (near_lim(whi, g->z_min, g->m_rel, g->m_len) || near_lim(wlo, zmax, g->m_rel, g->m_len))
                    flags |= FL_P4;
                if (whi < g->z_min || wlo > zmax) {
                    Hh->status |= ST_OUT_OF_Z;
                } else {
                    gather_candidates(g, T, &r, grp, Hh->sec, l, dxmax, L);
                    ncand += L->n;
                    for (int64_t a = 0; a < L->n; a++) {
                        int64_t j = L->v[a];
                        double c2;
                        unsigned fail, nm;
                        eval_cand(g, &r, T->y[j], T->z[j], T->dy[j], g->dx_chamber[T->det_row[j] >> 5],
                                  &c2, &fail, &nm);
                        if (!fail) clist_push(K, Hh->cost + c2, c2, h, j);
                        /* a gate decision within the margins: passing near a
                         * limit, or failing exactly one gate by a margin */
                        if ((!fail && nm) || (fail && popcount4(fail) == 1 && (fail & nm))) {
                            unsigned near = fail ? (fail & nm) : nm;
                            clist_push(E, Hh->cost + c2, c2, h,
                                       (fail ? 1 : 0) | ((near & 8u) ? 2 : 0) | ((near & 7u) ? 4 : 0));
                        }
                    }
                }
            }
            /* no chamber in this slot: nothing to miss, no penalty */
            double pen = g->chi2_penalty;
            if (Hh->live) {
                double mzs = g->m_rel * fabs(Hh->p[1]) + g->m_len;
                int d0 = chamber_at(g, Hh->sec, l, Hh->p[1]);
                int dlo = chamber_at(g, Hh->sec, l, Hh->p[1] - mzs), dhi = chamber_at(g, Hh->sec, l, Hh->p[1] + mzs);
                int a0 = d0 >= 0 && g->absent[d0], alo = dlo >= 0 && g->absent[dlo], ahi = dhi >= 0 && g->absent[dhi];
                if (a0 != alo || a0 != ahi) flags |= FL_P4;
                if (a0) pen = 0.0;
            }
            clist_push(K, Hh->cost + pen, 0.0, h, -1);
        }
        qsort(K->v, (size_t)K->n, sizeof(child_t), cmp_child);
        int nk = K->n < N ? (int)K->n : N;
        /* decisions within the margins: the edge of the kept set, the final
         * winner, and gate decisions on children that would be kept */
        double edge = K->v[nk - 1].cost;
        /* (path costs are sums over the layers: compared with the fixed
         * absolute margin m_chi2, not the per-road state tolerance) */
        if (K->n > nk && K->v[nk].cost - edge <= g->m_rel * fabs(edge) + g->m_chi2) flags |= FL_P3;
        if (l == NLAY - 1 && nk > 1 && K->v[1].cost - K->v[0].cost <= g->m_rel * fabs(K->v[0].cost) + g->m_chi2)
            flags |= FL_P3;
        for (int64_t a = 0; a < E->n; a++)
            if (E->v[a].cost <= edge + g->m_rel * fabs(edge) + g->m_chi2)
                flags |= ((E->v[a].j & 1) ? FL_P2 : FL_P1) | ((E->v[a].j & 2) ? FL_KCUT : 0u) |
                         ((E->v[a].j & 4) ? FL_KGATE : 0u);
        for (int k = 0; k < nk; k++) {
            const child_t *c = &K->v[k];
            hyp_t *d = &Hn[k];
            *d = H[c->parent];
            d->cost = c->cost;
            if (c->j < 0 || !d->live) continue;
            int64_t j = c->j;
            double dxj = g->dx_chamber[T->det_row[j] >> 5];
            if (dxj != 0.0 && !propagate(d->p, d->C, &d->x, g->x_layer[l] + dxj, g, &flags, NULL)) {
                d->status |= ST_STOP_SNP;
                d->live = 0;
                continue;
            }
            double ry = T->y[j] - (d->p[0] + g->tilt[l] * (d->p[1] - T->z[j]));
            double rz = T->z[j] - d->p[1];
            double syu = poly2(g->sigma_y, d->p[2]);
            kalman_update(d->p, d->C, ry, rz, g->tilt[l], syu * syu, vz);
            d->idx[l] = (int32_t)j;
            d->chi2l[l] = c->chi2;
            d->nmatch++;
            d->chi2sum += c->chi2;
            if (near_lim(fabs(d->p[2]), g->snp_max, g->m_rel, g->m_snp)) flags |= FL_P4;
            if (!(fabs(d->p[2]) < g->snp_max)) {
                d->status |= ST_STOP_SNP;
                d->live = 0;
            }
        }
        memcpy(H, Hn, sizeof(hyp_t) * (size_t)nk);
        nh = nk;
    }
done:
    {
        hyp_t *b = &H[0];
        pack(b->C, pk);
        for (int k = 0; k < 5; k++) o->p[k * n + i] = b->p[k];
        for (int k = 0; k < 15; k++) o->c[k * n + i] = pk[k];
        for (int l = 0; l < NLAY; l++) {
            o->idx[l * n + i] = b->idx[l];
            if (o->chi2_layer) o->chi2_layer[l * n + i] = b->chi2l[l];
            if (o->lx) o->lx[l * n + i] = NAN;
            if (o->lsec) o->lsec[l * n + i] = -1;
        }
        o->x[i] = b->x;
        o->sec[i] = b->sec;
        o->chi2[i] = b->chi2sum;
        o->n_match[i] = b->nmatch;
        o->status[i] = b->status;
        o->flags[i] = flags;
        /* the answer depends on every layer's selection */
        if (o->flag_layer) o->flag_layer[i] = flags ? 0 : NLAY;
        if (o->n_cand) o->n_cand[i] = ncand;
        if (o->cost) o->cost[i] = b->cost;
    }
}

/* Matches every track.  mode 0: binned search over the sorted cells;
 * mode 1: brute force over all tracklets of the same group/sector/layer. */
int oracle_match(const ocfg *g, int64_t n_trk, const double *tp, const double *tc,
                 const double *tx, const int32_t *tsec, const int32_t *tgrp,
                 int64_t n_tkl, const double *ky, const double *kz, const double *kdy,
                 const uint32_t *kdetrow, const int32_t *kgrp, int32_t n_groups,
                 int32_t mode, int32_t n_threads,
                 int32_t *idx, double *op, double *oc, double *ox, int32_t *osec,
                 double *ochi2, double *ochi2_layer, int32_t *on_match, uint32_t *ostatus,
                 uint32_t *oflags, int32_t *oflag_layer, int64_t *on_cand,
                 double *lp, double *lc, double *lx, int32_t *lsec, double *ocost)
{
    otkl T = {ky, kz, kdy, kdetrow, kgrp, n_tkl, NULL, NULL, n_groups, mode == 1};
    int32_t *perm = NULL;
    uint32_t *offsets = NULL;
    if (n_groups < 1) return -1;
    if (!T.brute) {
        int64_t nc = n_cells_of(g, n_groups);
        perm = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n_tkl > 0 ? n_tkl : 1));
        offsets = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(nc + 1));
        if (!perm || !offsets) { free(perm); free(offsets); return -2; }
        oracle_bin(g, n_tkl, ky, kz, kdy, kdetrow, kgrp, n_groups, perm, offsets);
        T.perm = perm;
        T.offsets = offsets;
    }
    double dxmax = 0.0;
    for (int d = 0; d < NDET; d++) dxmax = fabs(g->dx_chamber[d]) > dxmax ? fabs(g->dx_chamber[d]) : dxmax;
    oout o = {idx, op, oc, ox, osec, ochi2, ochi2_layer, on_match, ostatus, oflags, oflag_layer,
              on_cand, lp, lc, lx, lsec, ocost};
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#endif
#pragma omp parallel
    {
        ilist L = {NULL, 0, 0};
        clist K = {NULL, 0, 0}, E = {NULL, 0, 0};
#pragma omp for schedule(dynamic, 256)
        for (int64_t i = 0; i < n_trk; i++) {
            if (g->n_hyp >= 1)
                match_one_beam(g, i, n_trk, tp, tc, tx, tsec, tgrp, &T, dxmax, &o, &L, &K, &E);
            else
                match_one(g, i, n_trk, tp, tc, tx, tsec, tgrp, &T, dxmax, &o, &L);
        }
        free(L.v);
        free(K.v);
        free(E.v);
    }
    free(perm);
    free(offsets);
    return 0;
}

/* ---------------------------------------------------------------------- */
/* TRD-only refit (Sect. 2, step 3: refits from the outer detectors with   */
/* the TPC information ignored)                                            */
/* ---------------------------------------------------------------------- */

/* Readings where the paper is silent:
 *   - the refit starts from the matched track's final state with the
 *     covariance replaced by diag(refit_cov), which drops what the TPC
 *     contributed to it;
 *   - it runs inward over layers 5..0: propagate to the layer plane (sector
 *     hops as in the matching); with a tracklet at that layer, turn into the
 *     tracklet's sector if it is a neighbour (else skip it, REFIT_SKIP), step
 *     to x_l + dx and update; then add the layer's scattering, except at
 *     layer 0;
 *   - the result is the state after layer 0; chi2 is the sum of the
 *     predicted chi2 of the updates;
 *   - fewer than refit_min tracklets: the input state is copied with the
 *     starting covariance and REFIT_FEW. */
/* The matched tracklet of layer l, or -1: an index is one only if it lies in
 * [0, n_tkl) and its chamber exists (det < 540) and belongs to layer l. */
static int32_t refit_index(int32_t j, int l, int64_t n_tkl, const uint32_t *kdr)
{
    if (j < 0 || j >= n_tkl) return -1;
    const uint32_t det = kdr[j] >> 5;
    return (det < NDET && det % NLAY == (uint32_t)l) ? j : -1;
}

static void refit_one(const ocfg *g, int64_t i, int64_t n, const double *ip, const double *ix,
                      const int32_t *isec, const int32_t *idx, int64_t n_tkl, const double *ky,
                      const double *kz, const uint32_t *kdr, double *op, double *oc, double *ox,
                      int32_t *osec, double *ochi2, int32_t *onused, uint32_t *ostatus)
{
    const double tan10 = tan(M_PI / NSEC), dphi = 2.0 * M_PI / NSEC;
    double p[5], C[5][5], x = ix[i], chi2 = 0.0;
    int sec = isec[i], nused = 0, nm = 0;
    unsigned status = 0;
    memset(C, 0, sizeof(C));
    for (int k = 0; k < 5; k++) {
        p[k] = ip[k * n + i];
        C[k][k] = g->refit_cov[k];
    }
    for (int l = 0; l < NLAY; l++)
        if (refit_index(idx[l * n + i], l, n_tkl, kdr) >= 0) nm++;
    int bad = !(isfinite(x) && sec >= 0 && sec < NSEC);
    for (int k = 0; k < 5; k++) bad |= !isfinite(p[k]);
    if (!bad) bad = !(fabs(p[2]) < g->snp_max);
    if (bad) {
        status = ST_BAD_INPUT;
    } else if (nm < g->refit_min) {
        status = ST_REFIT_FEW;
    } else {
        const double vz = g->pad_len * g->pad_len / 12.0;
        for (int l = NLAY - 1; l >= 0 && !(status & (ST_STOP_SNP | ST_ROT_FAIL)); l--) {
            const double xl = g->x_layer[l];
            if (!propagate(p, C, &x, xl, g, NULL, NULL)) { status |= ST_STOP_SNP; break; }
            for (int nrot = 0;; nrot++) {
                if (fabs(p[0]) <= xl * tan10) break;
                if (nrot == 2) { status |= ST_ROT_FAIL; break; }
                int up = p[0] > 0;
                if (!rotate(p, C, &x, up ? dphi : -dphi, g, NULL)) { status |= ST_ROT_FAIL; break; }
                sec = (sec + (up ? 1 : NSEC - 1)) % NSEC;
                if (!propagate(p, C, &x, xl, g, NULL, NULL)) { status |= ST_STOP_SNP; break; }
            }
            if (status & (ST_STOP_SNP | ST_ROT_FAIL)) break;
            int32_t j = refit_index(idx[l * n + i], l, n_tkl, kdr);
            if (j >= 0) {
                const int det = (int)(kdr[j] >> 5), st = det / (NSTK * NLAY);
                int ok = 1;
                if (st != sec) {
                    int d = (st - sec + NSEC) % NSEC;
                    if (d == 1 || d == NSEC - 1) {
                        if (!rotate(p, C, &x, d == 1 ? dphi : -dphi, g, NULL)) { status |= ST_ROT_FAIL; break; }
                        sec = st;
                        if (!propagate(p, C, &x, xl, g, NULL, NULL)) { status |= ST_STOP_SNP; break; }
                    } else {
                        status |= ST_REFIT_SKIP;
                        ok = 0;
                    }
                }
                if (ok) {
                    const double dxj = g->dx_chamber[det];
                    if (dxj != 0.0 && !propagate(p, C, &x, xl + dxj, g, NULL, NULL)) { status |= ST_STOP_SNP; break; }
                    const double tau = g->tilt[l];
                    const double ry = ky[j] - (p[0] + tau * (p[1] - kz[j]));
                    const double rz = kz[j] - p[1];
                    const double sy = poly2(g->sigma_y, p[2]);
                    const double Syy = C[0][0] + 2.0 * tau * C[0][1] + tau * tau * C[1][1] + sy * sy;
                    const double Syz = C[0][1] + tau * C[1][1];
                    const double Szz = C[1][1] + vz;
                    const double det2 = Syy * Szz - Syz * Syz;
                    chi2 += (Szz * ry * ry - 2.0 * Syz * ry * rz + Syy * rz * rz) / det2;
                    kalman_update(p, C, ry, rz, tau, sy * sy, vz);
                    nused++;
                    if (!(fabs(p[2]) < g->snp_max)) { status |= ST_STOP_SNP; break; }
                }
            }
            if (l > 0) {
                add_ms(p, C, g);
                eloss(p, C, g, -1, NULL);
            }
        }
    }
    double pk[15];
    pack(C, pk);
    for (int k = 0; k < 5; k++) op[k * n + i] = p[k];
    for (int k = 0; k < 15; k++) oc[k * n + i] = pk[k];
    ox[i] = x;
    osec[i] = sec;
    ochi2[i] = chi2;
    onused[i] = nused;
    ostatus[i] = status;
}

int oracle_refit(const ocfg *g, int64_t n, const double *tp, const double *tx, const int32_t *tsec,
                 const int32_t *idx, int64_t n_tkl, const double *ky, const double *kz, const uint32_t *kdr,
                 int32_t n_threads, double *op, double *oc, double *ox, int32_t *osec, double *ochi2,
                 int32_t *onused, uint32_t *ostatus)
{
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#endif
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < n; i++)
        refit_one(g, i, n, tp, tx, tsec, idx, n_tkl, ky, kz, kdr, op, oc, ox, osec, ochi2, onused, ostatus);
    return 0;
}

/* ---------------------------------------------------------------------- */
/* Residuals of TPC clusters against the reference tracks, per sub-volume  */
/* (Sect. 2, steps 4 and 5)                                                */
/* ---------------------------------------------------------------------- */

typedef struct {
    double x_in, x_out;         /* pad rows: x_r = x_out - r (x_out - x_in) / (n_rows - 1) */
    int32_t n_rows;
    int32_t nx, ny, nz;         /* voxels per sector: x, y/x over +-tan 10deg, z/x over +-1 */
    int32_t min_count;          /* fewest clusters for a voxel's distortion */
    int32_t pad_;
} otpc;

#define NSUM 8

/* Readings where the paper is silent:
 *   - the reference of a cluster is the reference track (the TRD-only refit
 *     here; the ITS side is out of scope) propagated along its helix to the
 *     cluster's pad row, turned into the cluster's sector when that is a
 *     neighbour (clusters further away are left out);
 *   - a cluster seen at row x was created at x - dX and displaced by
 *     (dY, dZ), so to first order its residuals are
 *     r_y = dY - dX tan(phi), r_z = dZ - dX tan(lambda)/cos(phi);
 *   - a voxel is (sector, x bin, y/x bin, z/x bin) of the reference point;
 *     per voxel (dX, dY, dZ) is the least-squares solution of those equations
 *     over its clusters (unit weights), from 8 sums: n, sum t_y, sum t_z,
 *     sum (t_y^2 + t_z^2), sum r_y, sum r_z, sum (t_y r_y + t_z r_z),
 *     sum (r_y^2 + r_z^2);
 *   - reference tracks with any status bit are left out. */
static int64_t voxel_of(const otpc *t, int sec, double x, double y, double z)
{
    const double tan10 = tan(M_PI / NSEC);
    double fx = (x - t->x_in) / (t->x_out - t->x_in) * t->nx;
    double fy = (y / x / tan10 + 1.0) * 0.5 * t->ny;
    double fz = (z / x + 1.0) * 0.5 * t->nz;
    int ix = fx < 0 ? 0 : (fx >= t->nx ? t->nx - 1 : (int)fx);
    int iy = fy < 0 ? 0 : (fy >= t->ny ? t->ny - 1 : (int)fy);
    int iz = fz < 0 ? 0 : (fz >= t->nz ? t->nz - 1 : (int)fz);
    return (((int64_t)sec * t->nx + ix) * t->ny + iy) * t->nz + iz;
}

int oracle_residuals(const ocfg *g, const otpc *t, int64_t n, const double *rp, const double *rx,
                     const int32_t *rsec, const uint32_t *rstatus, const int64_t *first, const double *cy,
                     const double *cz, const int32_t *crow, const int32_t *csec, double *sums)
{
    const double dphi = 2.0 * M_PI / NSEC;
    const double step = (t->x_out - t->x_in) / (t->n_rows - 1);
    for (int64_t i = 0; i < n; i++) {
        if (rstatus[i] != 0) continue;
        double p[5], x = rx[i];
        int sec = rsec[i];
        for (int k = 0; k < 5; k++) p[k] = rp[k * n + i];
        for (int64_t c = first[i]; c < first[i + 1]; c++) {
            const double xr = t->x_out - crow[c] * step;
            if (csec[c] != sec) {
                int d = (csec[c] - sec + NSEC) % NSEC;
                if (d != 1 && d != NSEC - 1) continue;
                if (!rotate(p, NULL, &x, d == 1 ? dphi : -dphi, g, NULL)) break;
                sec = csec[c];
            }
            if (!propagate(p, NULL, &x, xr, g, NULL, NULL)) break;
            const double f = sqrt(1.0 - p[2] * p[2]);
            const double ty = p[2] / f, tz = p[3] / f;
            const double ry = cy[c] - p[0], rz = cz[c] - p[1];
            double *S = sums + NSUM * voxel_of(t, sec, xr, p[0], p[1]);
            S[0] += 1.0;
            S[1] += ty;
            S[2] += tz;
            S[3] += ty * ty + tz * tz;
            S[4] += ry;
            S[5] += rz;
            S[6] += ty * ry + tz * rz;
            S[7] += ry * ry + rz * rz;
        }
    }
    return 0;
}

/* Per voxel (dX, dY, dZ, n) from the sums: the normal equations
 *   [ n     0    -St ] [dY]   [  Sy ]
 *   [ 0     n    -Sz ] [dZ] = [  Sz_r ]
 *   [-St   -Sz   Stt ] [dX]   [ -Str ]
 * solved by elimination; NaN below min_count or when singular. */
int oracle_voxel_solve(const otpc *t, int64_t nvox, const double *sums, double *dist)
{
    for (int64_t v = 0; v < nvox; v++) {
        const double *S = sums + NSUM * v;
        double *o = dist + 4 * v;
        o[3] = S[0];
        o[0] = o[1] = o[2] = NAN;
        if (S[0] < t->min_count) continue;
        const double nn = S[0], st = S[1], sz = S[2], stt = S[3];
        /* eliminate dY and dZ: dY = (Sy + st dX)/n, dZ = (Sz + sz dX)/n */
        const double a = stt - (st * st + sz * sz) / nn;
        const double b = -S[6] + (st * S[4] + sz * S[5]) / nn;
        if (!(a > 1e-12 * stt)) continue;
        const double dX = b / a;
        o[0] = dX;
        o[1] = (S[4] + st * dX) / nn;
        o[2] = (S[5] + sz * dX) / nn;
    }
    return 0;
}

int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ---------------------------------------------------------------------- */
/* single steps, exported for the unit pins                               */
/* ---------------------------------------------------------------------- */

int oracle_propagate(const ocfg *g, double *p, double *cpk, double *x, double x2, double *J)
{
    double C[5][5], Jm[5][5];
    if (cpk) unpack(cpk, C);
    int ok = propagate(p, cpk ? C : NULL, x, x2, g, NULL, Jm);
    if (ok && cpk) pack(C, cpk);
    if (ok && J) memcpy(J, Jm, sizeof(Jm));
    return ok;
}

int oracle_rotate(const ocfg *g, double *p, double *cpk, double *x, double da, double *J)
{
    double C[5][5], Jm[5][5];
    if (cpk) unpack(cpk, C);
    int ok = rotate(p, cpk ? C : NULL, x, da, g, Jm);
    if (ok && cpk) pack(C, cpk);
    if (ok && J) memcpy(J, Jm, sizeof(Jm));
    return ok;
}

void oracle_add_ms(const ocfg *g, const double *p, double *cpk)
{
    double C[5][5];
    unpack(cpk, C);
    add_ms(p, C, g);
    pack(C, cpk);
}

int oracle_eloss(const ocfg *g, double *p, double *cpk, int dir)
{
    double C[5][5];
    unpack(cpk, C);
    int ok = eloss(p, C, g, dir, NULL);
    pack(C, cpk);
    return ok;
}

double oracle_bethe(const ocfg *g, double p, double m) { return bethe(p, m, g); }

int oracle_chamber_at(const ocfg *g, int sec, int l, double z) { return chamber_at(g, sec, l, z); }

void oracle_update(double *p, double *cpk, double ry, double rz, double tau, double vy, double vz)
{
    double C[5][5];
    unpack(cpk, C);
    kalman_update(p, C, ry, rz, tau, vy, vz);
    pack(C, cpk);
}

int oracle_ldl_pd(const double *cpk)
{
    double C[5][5];
    unpack(cpk, C);
    return ldl_pd(C);
}

int64_t oracle_key(const ocfg *g, double y, double z, double dy, uint32_t det_row, int32_t grp,
                   int32_t n_groups)
{
    return tkl_key(g, y, z, dy, det_row, grp, n_groups);
}

int32_t oracle_cfg_size(void) { return (int32_t)sizeof(ocfg); }
