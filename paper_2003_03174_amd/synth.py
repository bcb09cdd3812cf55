"""Seeded synthetic TRD workloads: ITS-TPC seed tracks and TRD tracklets.

This module is input generation only.  It simulates charged tracks as global
helices from the vertex in a uniform solenoid field (closed-form circle/line and
circle/cylinder crossings in the global frame), applies multiple-scattering kicks
at the six TRD layers, and records one tracklet per crossed chamber plus uniform
fakes.  It implements none of the matching method: no Kalman propagation,
gating, binning or update.  Both the FP64 oracle and the HIP path are fed from
here; the truth it records pins the oracle's propagation.

Geometry follows the paper's description of the TRD (Sect. 3): 18 azimuthal
sectors, 5 stacks along z, 6 radial layers, tracklets that carry a transverse
offset y at the chamber radius, a deflection dy over the 3 cm drift length and
the pad row in z.  The pad tilt correction of Sect. 3 enters the measured y.
Where the paper gives no number the readings are documented with the workload
presets at the bottom of this file.

Units: cm, GeV/c, tesla.  Track state (y, z, sin(phi), tan(lambda), q/pT) is
expressed at local x in the frame of a sector rotated by alpha = (sec+1/2)*20deg.
"""
from __future__ import annotations

import math

import numpy as np

KAPPA = 2.99792458e-3          # cm^-1 GeV T^-1: curvature of a pT=1 GeV track in 1 T
N_SECTORS, N_STACKS, N_LAYERS, N_ROWS = 18, 5, 6, 18
N_DET = N_SECTORS * N_STACKS * N_LAYERS   # 540 chamber slots
SECTOR_DPHI = 2.0 * math.pi / N_SECTORS
PION_MASS = 0.13957

# status-free packed covariance layout: upper triangle, row-major, of the 5x5
# matrix over (y, z, snp, tgl, q/pT)
COV_DIAG = (0, 5, 9, 12, 14)


def default_params(**over):
    """Detector, physics, resolution and cut parameters of one workload.

    Plain values only; both the oracle and the HIP library take their
    configuration from such a dict.
    """
    chi2_max = -2.0 * math.log(1e-3)          # 0.1 % tail of a 2-dof chi2
    p = dict(
        x_layer=[290.0 + 13.0 * l for l in range(N_LAYERS)],
        tilt=[0.0] * N_LAYERS,                 # tan(pad tilt) per layer
        z_min=-360.0,
        pad_len=8.0,
        n_rows=N_ROWS,
        n_yb=16,
        y_bin_w=8.0,
        n_db=1,                                # deflection bins per y bin row
        dy_bin_w=0.0625,
        drift_len=3.0,
        dx_chamber=np.zeros(N_DET),
        bz=0.5,
        x_over_x0=0.03,
        mass=PION_MASS,
        sigma_y=[0.04, 0.0, 0.0],
        sigma_dy=[0.0015, 0.0, 0.0],
        tan_psi=0.0,
        chi2_max=chi2_max,
        n_sigma_dy=4.0,
        n_sigma_road=math.sqrt(chi2_max),
        snp_max=0.95,
        # realistic detector model, off by default: mean energy loss in each
        # layer's material (g/cm^2 at normal incidence, Z/A, mean excitation
        # energy in GeV) and the chamber slots without a chamber
        eloss_xrho=0.0,
        eloss_za=0.5,
        eloss_i=1e-7,
        absent=np.zeros(N_DET, dtype=np.uint8),
        # field inhomogeneity, off by default: Bz(r, z) = bz (1 + field_br
        # (r / 370 cm)^2 + field_bz (z / 360 cm)^2), and the largest x step
        # of the matcher's Runge-Kutta integration in such a field
        field_br=0.0,
        field_bz=0.0,
        field_step=0.25,
    )
    for k, v in over.items():
        if k not in p:
            raise KeyError(f"unknown parameter {k!r}")
        p[k] = v
    p["dx_chamber"] = np.asarray(p["dx_chamber"], dtype=np.float64).reshape(N_DET)
    p["absent"] = (np.asarray(p["absent"]).reshape(N_DET) != 0).astype(np.uint8)
    return p


def absent_522():
    """The installed detector: 522 of the 540 chamber slots, the middle stack
    of sectors 13, 14 and 15 (in front of the photon spectrometer) left
    empty."""
    a = np.zeros(N_DET, dtype=np.uint8)
    for sec in (13, 14, 15):
        for l in range(N_LAYERS):
            a[sec * N_STACKS * N_LAYERS + 2 * N_LAYERS + l] = 1
    return a


def realistic_overrides():
    """Detector model with energy loss and the 522-chamber layout.  The layer
    material is a plastic-like radiator and chamber: 1.2 g/cm^2 (about
    X/X0 = 0.03 at X0 = 40 g/cm^2), Z/A = 0.53, I = 70 eV."""
    return dict(eloss_xrho=1.2, eloss_za=0.53, eloss_i=70e-9, absent=absent_522())


def realistic_params(**over):
    p = realistic_overrides()
    p.update(over)
    return default_params(**p)


def inclined_resolution(psi_deg=8.0):
    """Tracklet resolutions that depend on the track inclination, with the dy
    offset of the Lorentz angle (Sect. 3 and Fig. 3: the widths are
    second-order polynomials in sin(phi), best for tracks at the Lorentz
    angle, about 8 degrees at 0.5 T).  The figure's coefficients are not in
    the text; these curves put the minimum at sin(phi) = sin(psi_L):
    sigma_y = 0.03 cm + 0.5 cm (s - s_L)^2, sigma_dy = 0.0015 cm +
    0.02 cm (s - s_L)^2 (0.5 mrad over the 3 cm drift at the minimum)."""
    sl = math.sin(math.radians(psi_deg))

    def around(w0, k):
        return [w0 + k * sl * sl, -2.0 * k * sl, k]

    return dict(sigma_y=around(0.03, 0.5), sigma_dy=around(0.0015, 0.02),
                tan_psi=math.tan(math.radians(psi_deg)))


def field_map_overrides(br=-0.02, bz=-0.04):
    """A field that falls off towards the ends of the solenoid and outwards:
    2 % lower at the outer TRD radius, 4 % lower at the ends of the chambers
    (the paper names field inhomogeneities in the precise extrapolation and
    gives no map; this one is synthetic)."""
    return dict(field_br=br, field_bz=bz)


FIELD_RREF, FIELD_ZREF = 370.0, 360.0


def field_at(P, X, Y, Z):
    """Bz (T) of the field model at global (X, Y, Z)."""
    r2 = X * X + Y * Y
    return P["bz"] * (1.0 + P["field_br"] * r2 / FIELD_RREF ** 2 + P["field_bz"] * Z * Z / FIELD_ZREF ** 2)


def _field_on(P):
    return P.get("field_br", 0.0) != 0.0 or P.get("field_bz", 0.0) != 0.0


def _rk_global(P, X, Y, Z, Phi, tg, c, ds):
    """One classical Runge-Kutta step of length ds (transverse path, signed)
    of the equation of motion in the global frame: X' = cos Phi, Y' = sin Phi,
    Z' = tan(lambda), Phi' = -kappa Bz(X, Y, Z) q/pT (Bz only: pT and pz are
    constant)."""
    def f(Xa, Ya, Za, Pa):
        return np.cos(Pa), np.sin(Pa), tg, -KAPPA * field_at(P, Xa, Ya, Za) * c
    a = f(X, Y, Z, Phi)
    b = f(X + 0.5 * ds * a[0], Y + 0.5 * ds * a[1], Z + 0.5 * ds * a[2], Phi + 0.5 * ds * a[3])
    cc = f(X + 0.5 * ds * b[0], Y + 0.5 * ds * b[1], Z + 0.5 * ds * b[2], Phi + 0.5 * ds * b[3])
    d = f(X + ds * cc[0], Y + ds * cc[1], Z + ds * cc[2], Phi + ds * cc[3])
    k6 = ds / 6.0
    return (X + k6 * (a[0] + 2 * b[0] + 2 * cc[0] + d[0]), Y + k6 * (a[1] + 2 * b[1] + 2 * cc[1] + d[1]),
            Z + k6 * (a[2] + 2 * b[2] + 2 * cc[2] + d[2]), Phi + k6 * (a[3] + 2 * b[3] + 2 * cc[3] + d[3]))


def _march(P, X, Y, Z, Phi, tg, c, level, dlevel, target, h, max_len):
    """Steps of length h along the track (forward where target > level, else
    backward) while the next one stays short of level == target, then Newton
    on the last partial step.  level(X, Y) is the quantity that must reach
    target, dlevel(X, Y, Phi) its derivative along the path.  Returns
    (ok, X, Y, Z, Phi, s) with s the signed path length."""
    sgn = np.where(level(X, Y) <= target, 1.0, -1.0)
    s = np.zeros_like(X)
    ok = np.ones(X.shape, dtype=bool)
    active = ok.copy()
    nmax = int(np.ceil(max_len / h)) + 2
    for _ in range(nmax):
        if not active.any():
            break
        Xn, Yn, Zn, Pn = _rk_global(P, X, Y, Z, Phi, tg, c, sgn * h)
        passed = sgn * (level(Xn, Yn) - target) >= 0
        step = active & ~passed
        X, Y, Z, Phi = (np.where(step, Xn, X), np.where(step, Yn, Y), np.where(step, Zn, Z),
                        np.where(step, Pn, Phi))
        s = np.where(step, s + sgn * h, s)
        active &= ~passed
        # a track that turns away from the target never reaches it
        away = active & (sgn * dlevel(X, Y, Phi) <= 0)
        ok &= ~away
        active &= ~away
    ok &= ~active
    # the partial step: Newton on its length
    d = np.where(ok, (target - level(X, Y)) / np.where(ok, dlevel(X, Y, Phi), 1.0), 0.0)
    for _ in range(6):
        Xn, Yn, Zn, Pn = _rk_global(P, X, Y, Z, Phi, tg, c, d)
        dl = dlevel(Xn, Yn, Pn)
        ok &= dl * sgn > 0
        d = d - np.where(ok, (level(Xn, Yn) - target) / np.where(ok, dl, 1.0), 0.0)
    Xn, Yn, Zn, Pn = _rk_global(P, X, Y, Z, Phi, tg, c, d)
    return ok, Xn, Yn, Zn, Pn, s + d


def _cross_cylinder_field(P, phi0, tg, c, rho, dt, h=0.25):
    """Crossing of a track from the origin with the cylinder r = rho in the
    field model: (ok, X, Y, Z, Phi)."""
    z0 = np.zeros(phi0.shape, dtype=dt)
    ok, X, Y, Z, Phi, _ = _march(P, z0, z0.copy(), z0.copy(), phi0.astype(dt), tg, c,
                                 lambda X, Y: np.hypot(X, Y),
                                 lambda X, Y, Ph: np.where(np.hypot(X, Y) > 0,
                                                           (X * np.cos(Ph) + Y * np.sin(Ph)) /
                                                           np.maximum(np.hypot(X, Y), 1e-300), 1.0),
                                 dt(rho), h, 4.0 * rho)
    return ok, X, Y, Z, Phi


def _cross_plane_field(P, X, Y, Z, Phi, tg, c, alpha, xl, dt, h=0.25):
    """Crossing of the track through (X, Y, Z) with direction Phi with the
    plane X cos(alpha) + Y sin(alpha) = xl of a sector, forwards or
    backwards, in the field model.  Same outputs as _cross_plane, plus Z."""
    ca, sa = np.cos(alpha), np.sin(alpha)
    x0 = X * ca + Y * sa
    ok, X1, Y1, Z1, Phi1, arc = _march(P, X, Y, Z, Phi, tg, c, lambda Xa, Ya: Xa * ca + Ya * sa,
                                       lambda Xa, Ya, Pa: np.cos(Pa - alpha), xl, h,
                                       4.0 * np.max(np.abs(np.asarray(xl - x0, dtype=np.float64)), initial=1.0) + 10.0)
    y = -X1 * sa + Y1 * ca
    phl = Phi1 - alpha
    snp, csp = np.sin(phl), np.cos(phl)
    ok &= csp > 0
    return ok, y, snp, csp, X1, Y1, arc, Phi1, Z1


def tilt_pm2deg():
    """The paper's +-2 degree pad tilt, alternating sign from layer to layer."""
    t = math.tan(math.radians(2.0))
    return [t if l % 2 == 0 else -t for l in range(N_LAYERS)]


# ---------------------------------------------------------------------------
# closed-form helix geometry (global frame)
# ---------------------------------------------------------------------------

def _sector_of(X, Y):
    ang = np.mod(np.arctan2(Y, X), 2.0 * np.pi)
    sec = np.floor(ang / SECTOR_DPHI).astype(np.int64)
    return np.mod(sec, N_SECTORS)


def _alpha(sec, dt):
    return (np.asarray(sec, dtype=dt) + dt(0.5)) * dt(2.0) * dt(np.pi) / dt(N_SECTORS)


def _cross_cylinder(phi0, cu, rho, dt):
    """First crossing of a helix from the origin with the cylinder r = rho.

    Returns (ok, phi_pos, phi_dir, arc): the azimuth of the crossing point, the
    azimuth of the direction there and the transverse arc length.  A chord of
    length rho subtends the turning angle 2*asin(rho*|C|/2).
    """
    h = rho * np.abs(cu) / dt(2.0)
    ok = h < 1.0
    hs = np.where(ok, h, dt(0.5))
    asin_over_h = np.where(hs > 0, np.arcsin(hs) / np.where(hs > 0, hs, 1), dt(1.0))
    delta = np.sign(cu) * dt(2.0) * np.arcsin(hs)
    arc = rho * asin_over_h
    return ok, phi0 + delta / 2, phi0 + delta, arc


def _cross_plane(X, Y, Phi, cu, alpha, xl, dt):
    """Crossing of a helix through (X, Y) with direction Phi with the plane of a
    sector: X cos(alpha) + Y sin(alpha) = xl.

    Circle/line intersection via the circle centre; the branch taken is the one
    where the track moves towards larger local x.  Works forwards and backwards
    along the helix.  Returns (ok, y_loc, snp, csp, X1, Y1, signed_arc, Phi1).
    """
    ca, sa = np.cos(alpha), np.sin(alpha)
    x0 = X * ca + Y * sa
    straight = cu == 0
    cus = np.where(straight, dt(1.0), cu)
    # circle centre P + (-sin Phi, cos Phi)/C and its local coordinates
    Xc = X - np.sin(Phi) / cus
    Yc = Y + np.cos(Phi) / cus
    xc = Xc * ca + Yc * sa
    yc = -Xc * sa + Yc * ca
    R = dt(1.0) / np.abs(cus)
    d = xl - xc
    disc = R * R - d * d
    ok = disc > 0
    root = np.sqrt(np.where(ok, disc, dt(1.0)))
    y = yc - np.sign(cus) * root
    snp = cus * d
    csp = np.abs(cus) * root
    # straight line: y = y0 + (xl - x0) tan(phi_loc)
    phl = Phi - alpha
    y0 = -X * sa + Y * ca
    y_str = y0 + (xl - x0) * np.sin(phl) / np.cos(phl)
    y = np.where(straight, y_str, y)
    snp = np.where(straight, np.sin(phl), snp)
    csp = np.where(straight, np.cos(phl), csp)
    ok = np.where(straight, np.cos(phl) > 0, ok & (csp > 0))
    X1 = xl * ca - y * sa
    Y1 = xl * sa + y * ca
    chord = np.hypot(X1 - X, Y1 - Y)
    h = chord * np.abs(np.where(straight, dt(0.0), cu)) / dt(2.0)
    hs = np.clip(h, dt(0.0), dt(1.0))
    asin_over_h = np.where(hs > 0, np.arcsin(hs) / np.where(hs > 0, hs, 1), dt(1.0))
    arc = chord * asin_over_h * np.sign(xl - x0)
    Phi1 = alpha + np.arctan2(snp, csp)
    return ok, y, snp, csp, X1, Y1, arc, Phi1


def bethe_rate(p, mass, za, i_exc):
    """Mean energy-loss rate (GeV cm^2/g) of a unit-charge particle: the Bethe
    formula without density-effect or shell terms (PDG review of the passage
    of particles through matter), clipped at zero."""
    me = 0.51099895e-3
    e = np.sqrt(p * p + mass * mass)
    bg2 = (p / mass) ** 2
    b2 = bg2 / (1.0 + bg2)
    gam = e / mass
    wmax = 2.0 * me * bg2 / (1.0 + 2.0 * gam * me / mass + (me / mass) ** 2)
    v = 0.307075e-3 * za / b2 * (0.5 * np.log(2.0 * me * bg2 * wmax / (i_exc * i_exc)) - b2)
    return np.maximum(v, 0.0)


def highland_theta0(p, beta, xi):
    """Highland/PDG width of the projected scattering angle (unit charge)."""
    return 0.0136 / (beta * p) * np.sqrt(xi) * (1.0 + 0.038 * np.log(xi))


# ---------------------------------------------------------------------------
# one group (frame / event) of tracks and tracklets
# ---------------------------------------------------------------------------

def generate_group(rng, params, n_tracks, *, pt_dist="exp", fake_ratio=0.2,
                   ineff_frac=0.0, distortion=None, noise_free=False,
                   ms=True, fp32=True, dtype=np.float64, rho_seed=250.0, seed_sigma_y=0.1,
                   seed_sigma_z=0.1):
    """Simulate one group.

    pt_dist: "exp" (pT = 0.3 + Exp(1)) or "pow3" (pdf ~ pT^-3 above 0.3).
    fake_ratio: fakes per true tracklet, uniform over the detector.
    ineff_frac: fraction of tracks that lose the tracklets of 1 or 2 layers.
    distortion: None or (dmin, dmax): random (y, z) displacement of the seed.
    noise_free: seeds are truth, tracklets are exact (z = true z), no MS kicks,
      no rounding to float32.
    seed_sigma_y, seed_sigma_z: Gaussian errors of the seed's y and z (cm).
    Returns a dict of numpy arrays (see generate()).
    """
    dt = dtype
    P = params
    n = int(n_tracks)
    bz = P["bz"]
    q = np.where(rng.random(n) < 0.5, -1.0, 1.0)
    phi0 = rng.random(n) * 2.0 * np.pi
    eta = rng.uniform(-0.84, 0.84, n)
    if pt_dist == "exp":
        pt = 0.3 + rng.exponential(1.0, n)
    elif pt_dist == "pow3":
        pt = 0.3 / np.sqrt(1.0 - rng.random(n))
    else:
        raise ValueError(pt_dist)
    tgl = np.sinh(eta)
    qpt = q / pt

    # seed point: helix / cylinder r = rho_seed (in a field map: integrated)
    fmap = _field_on(P)
    cu = (-KAPPA * bz * qpt).astype(dt)
    if fmap:
        ok0, X, Y, Z, phi_dir = _cross_cylinder_field(P, phi0.astype(dt), tgl.astype(dt), qpt.astype(dt),
                                                      rho_seed, dt)
    else:
        ok0, phi_pos, phi_dir, arc0 = _cross_cylinder(phi0.astype(dt), cu, dt(rho_seed), dt)
        X = dt(rho_seed) * np.cos(phi_pos)
        Y = dt(rho_seed) * np.sin(phi_pos)
        Z = tgl.astype(dt) * arc0
    sec0 = _sector_of(X, Y)
    a0 = _alpha(sec0, dt)
    seed = np.zeros((5, n), dtype=np.float64)
    seed_x = (X * np.cos(a0) + Y * np.sin(a0)).astype(np.float64)
    seed[0] = (-X * np.sin(a0) + Y * np.cos(a0)).astype(np.float64)
    seed[1] = Z.astype(np.float64)
    seed[2] = np.sin(phi_dir - a0).astype(np.float64)
    seed[3] = tgl
    seed[4] = qpt
    truth_seed = seed.copy()

    cov0 = np.array([seed_sigma_y ** 2, seed_sigma_z ** 2, 1e-3 ** 2, 1e-3 ** 2, 0.01 ** 2])
    if distortion is not None:
        cov0[0] += (distortion[1] / 3.0) ** 2
        cov0[1] += (distortion[1] / 3.0) ** 2
    cov = np.zeros((15, n))
    for k, j in enumerate(COV_DIAG):
        cov[j] = cov0[k]
    inp = seed.copy()
    if not noise_free:
        sig = np.array([seed_sigma_y, seed_sigma_z, 1e-3, 1e-3, 0.01])
        inp += rng.standard_normal((5, n)) * sig[:, None]
        if distortion is not None:
            dd = rng.uniform(distortion[0], distortion[1], n)
            th = rng.random(n) * 2.0 * np.pi
            inp[0] += dd * np.cos(th)
            inp[1] += dd * np.sin(th)
    inp[2] = np.clip(inp[2], -0.999, 0.999)

    # ---- propagate the true helix through the six layers ----
    xl_arr = P["x_layer"]
    tan10 = math.tan(SECTOR_DPHI / 2)
    pad, zmin = P["pad_len"], P["z_min"]
    zmax = -zmin
    n_rows_tot = N_STACKS * P["n_rows"]
    alive = ok0.copy()
    sec = sec0.copy()
    Phi = phi_dir.copy()
    tg = tgl.astype(dt).copy()
    c = qpt.astype(dt).copy()
    pabs = (pt * np.sqrt(1.0 + tgl * tgl)).astype(dt)   # |p| is kept by the kicks
    truth = {k: np.full((N_LAYERS, n), np.nan) for k in ("x", "y", "z", "snp", "tgl", "qpt")}
    truth["sec"] = np.full((N_LAYERS, n), -1, dtype=np.int64)
    tk_rows = []   # per layer: (track ids, y, z, dy, det, row)

    def cross(Xs, Ys, Zs, Phs, tgs, cs, alpha, xplane):
        """(ok, y, snp, csp, X1, Y1, arc, Phi1) of the crossing with a sector plane"""
        if fmap:
            return _cross_plane_field(P, Xs, Ys, Zs, Phs, tgs, cs, alpha, xplane, dt)[:8]
        return _cross_plane(Xs, Ys, Phs, -dt(KAPPA * bz) * cs, alpha, xplane, dt)

    for l in range(N_LAYERS):
        xl = dt(xl_arr[l])
        a = _alpha(sec, dt)
        ok, y, snp, csp, X1, Y1, arc, Phi1 = cross(X, Y, Z, Phi, tg, c, a, xl)
        for _ in range(2):   # switch to the neighbouring sector that holds the point
            out = ok & (np.abs(y) > xl * dt(tan10))
            if not out.any():
                break
            sec = np.where(out, np.mod(sec + np.where(y > 0, 1, -1), N_SECTORS), sec)
            a = _alpha(sec, dt)
            ok2, y2, s2, c2, X2, Y2, arc2, Ph2 = cross(X, Y, Z, Phi, tg, c, a, xl)
            ok = np.where(out, ok2, ok)
            y, snp, csp = np.where(out, y2, y), np.where(out, s2, snp), np.where(out, c2, csp)
            X1, Y1 = np.where(out, X2, X1), np.where(out, Y2, Y1)
            arc, Phi1 = np.where(out, arc2, arc), np.where(out, Ph2, Phi1)
        ok = ok & (np.abs(y) <= xl * dt(tan10)) & (np.abs(snp) < P["snp_max"])
        alive = alive & ok
        Z1 = Z + tg * arc
        X, Y, Z, Phi = (np.where(alive, X1, X), np.where(alive, Y1, Y),
                        np.where(alive, Z1, Z), np.where(alive, Phi1, Phi))
        # multiple-scattering kick (radiator in front of the drift region)
        if ms and not noise_free:
            beta = pabs / np.sqrt(pabs * pabs + dt(P["mass"]) ** 2)
            csp_safe = np.where(alive, csp, dt(1.0))
            xi = dt(P["x_over_x0"]) * np.sqrt(dt(1.0) + tg * tg) / csp_safe
            th0 = highland_theta0(pabs, beta, xi)
            k1 = rng.standard_normal(n).astype(dt) * th0
            k2 = rng.standard_normal(n).astype(dt) * th0
            lam = np.arctan(tg)
            Phi = np.where(alive, Phi + k1 * np.sqrt(dt(1.0) + tg * tg), Phi)
            lam2 = lam + k2
            tg = np.where(alive, np.tan(lam2), tg)
            c = np.where(alive, np.sign(c) / (pabs * np.cos(lam2)), c)
            phl = Phi - a
            alive = alive & (np.cos(phl) > 0) & (np.abs(np.sin(phl)) < P["snp_max"])
        # mean energy loss in the layer: the path through the slab is its
        # thickness over the cosine of the angle to the slab normal (the
        # sector's x axis)
        if P["eloss_xrho"] > 0:
            m = dt(P["mass"])
            cos_inc = np.cos(np.arctan(tg)) * np.cos(Phi - a)
            cos_inc = np.where(alive & (cos_inc > 0), cos_inc, dt(1.0))
            e0 = np.sqrt(pabs * pabs + m * m)
            e1 = e0 - bethe_rate(pabs, m, P["eloss_za"], P["eloss_i"]) * dt(P["eloss_xrho"]) / cos_inc
            alive = alive & (e1 > m)
            p1 = np.sqrt(np.maximum(e1 * e1 - m * m, dt(0.0)))
            c = np.where(alive, c * (pabs / np.where(alive, p1, pabs)), c)
            pabs = np.where(alive, p1, pabs)
        phl = Phi - a
        truth["sec"][l] = np.where(alive, sec, -1)
        truth["x"][l] = np.where(alive, np.float64(xl), np.nan)
        truth["y"][l] = np.where(alive, (-X * np.sin(a) + Y * np.cos(a)).astype(np.float64), np.nan)
        truth["z"][l] = np.where(alive, Z.astype(np.float64), np.nan)
        truth["snp"][l] = np.where(alive, np.sin(phl).astype(np.float64), np.nan)
        truth["tgl"][l] = np.where(alive, tg.astype(np.float64), np.nan)
        truth["qpt"][l] = np.where(alive, c.astype(np.float64), np.nan)

        # tracklet at the chamber radius x_l + dx[det] on the post-kick helix
        ids = np.nonzero(alive)[0]
        if ids.size == 0:
            tk_rows.append(None)
            continue
        Xa, Ya, Za, Pa, ca_ = X[ids], Y[ids], Z[ids], Phi[ids], c[ids]
        seca, aa, tga = sec[ids], a[ids], tg[ids]
        zrow = np.floor((Za.astype(np.float64) - zmin) / pad).astype(np.int64)
        stack = np.clip(zrow // P["n_rows"], 0, N_STACKS - 1)
        det = seca * (N_STACKS * N_LAYERS) + stack * N_LAYERS + l
        dxa = P["dx_chamber"][det].astype(dt)
        okt, yt, st, ct, _, _, arct, _ = cross(Xa, Ya, Za, Pa, tga, ca_, aa, xl + dxa)
        zt = (Za + tga * arct).astype(np.float64)
        yt = yt.astype(np.float64)
        st = st.astype(np.float64)
        ct = ct.astype(np.float64)
        keep = okt & (zt >= zmin) & (zt < zmax)
        ids, yt, zt, st, ct = ids[keep], yt[keep], zt[keep], st[keep], ct[keep]
        seca = seca[keep]
        tau = P["tilt"][l]
        if noise_free:
            zmeas = zt.copy()
        else:
            zmeas = None
        grow = np.floor((zt - zmin) / pad).astype(np.int64)
        grow = np.clip(grow, 0, n_rows_tot - 1)
        # the chamber (stack) is the one whose pad rows hold the tracklet's z
        det = seca * (N_STACKS * N_LAYERS) + (grow // P["n_rows"]) * N_LAYERS + l
        zcen = zmin + (grow + 0.5) * pad
        if not noise_free:
            zmeas = zcen
        sy = np.polyval(P["sigma_y"][::-1], st)
        sdy = np.polyval(P["sigma_dy"][::-1], st)
        ymeas = yt + tau * (zt - zmeas)
        dymeas = P["drift_len"] * (st / ct - P["tan_psi"])
        if not noise_free:
            ymeas = ymeas + rng.standard_normal(ids.size) * sy
            dymeas = dymeas + rng.standard_normal(ids.size) * sdy
        tk_rows.append((ids, ymeas, zmeas, dymeas, det, grow % P["n_rows"], grow))

    # inefficiency: some tracks lose the true tracklets of 1 or 2 layers
    drop = np.zeros((N_LAYERS, n), dtype=bool)
    if ineff_frac > 0:
        sel = np.nonzero(rng.random(n) < ineff_frac)[0]
        two = rng.random(sel.size) < 0.5
        l1 = rng.integers(0, N_LAYERS, sel.size)
        l2 = (l1 + rng.integers(1, N_LAYERS, sel.size)) % N_LAYERS   # a different layer
        drop[l1, sel] = True
        drop[l2[two], sel[two]] = True

    ys, zs, dys, dets, rows, labels, lays = [], [], [], [], [], [], []
    for l, tr in enumerate(tk_rows):
        if tr is None:
            continue
        ids, ym, zm, dym, det, row, _ = tr
        keep = ~drop[l, ids] & (P["absent"][det] == 0)
        ys.append(ym[keep]); zs.append(zm[keep]); dys.append(dym[keep])
        dets.append(det[keep]); rows.append(row[keep]); labels.append(ids[keep])
        lays.append(np.full(int(keep.sum()), l))
    n_true = int(sum(a.size for a in ys))
    n_fake = int(round(fake_ratio * n_true))
    if n_fake:
        fsec = rng.integers(0, N_SECTORS, n_fake)
        fst = rng.integers(0, N_STACKS, n_fake)
        flay = rng.integers(0, N_LAYERS, n_fake)
        frow = rng.integers(0, P["n_rows"], n_fake)
        fxl = np.asarray(P["x_layer"])[flay]
        fy = rng.uniform(-1.0, 1.0, n_fake) * fxl * tan10
        fdy = rng.uniform(-1.0, 1.0, n_fake)
        fdet = fsec * (N_STACKS * N_LAYERS) + fst * N_LAYERS + flay
        fk = P["absent"][fdet] == 0
        ys.append(fy[fk])
        zs.append((zmin + (fst * P["n_rows"] + frow + 0.5) * pad)[fk])
        dys.append(fdy[fk])
        dets.append(fdet[fk])
        rows.append(frow[fk])
        labels.append(np.full(int(fk.sum()), -1))
        lays.append(flay[fk])
    ty = np.concatenate(ys) if ys else np.zeros(0)
    tz = np.concatenate(zs) if zs else np.zeros(0)
    tdy = np.concatenate(dys) if dys else np.zeros(0)
    tdet = np.concatenate(dets).astype(np.int64) if dets else np.zeros(0, np.int64)
    trow = np.concatenate(rows).astype(np.int64) if rows else np.zeros(0, np.int64)
    tlab = np.concatenate(labels).astype(np.int64) if labels else np.zeros(0, np.int64)
    tlay = np.concatenate(lays).astype(np.int64) if lays else np.zeros(0, np.int64)
    perm = rng.permutation(ty.size)
    ty, tz, tdy, tdet, trow, tlab, tlay = (a[perm] for a in (ty, tz, tdy, tdet, trow, tlab, tlay))

    if fp32 and not noise_free:
        inp = inp.astype(np.float32).astype(np.float64)
        cov = cov.astype(np.float32).astype(np.float64)
        seed_x = seed_x.astype(np.float32).astype(np.float64)
        ty = ty.astype(np.float32).astype(np.float64)
        tz = tz.astype(np.float32).astype(np.float64)
        tdy = tdy.astype(np.float32).astype(np.float64)

    # index of each track's true tracklet per layer in the shuffled order
    true_idx = np.full((N_LAYERS, n), -1, dtype=np.int64)
    real = np.nonzero(tlab >= 0)[0]
    true_idx[tlay[real], tlab[real]] = real
    return dict(
        n_tracks=n, p=inp, cov=cov, x=seed_x, sector=sec0.astype(np.int32),
        truth_seed=truth_seed, truth=truth, true_idx=true_idx,
        tkl_y=ty, tkl_z=tz, tkl_dy=tdy, tkl_det=tdet, tkl_row=trow,
        tkl_label=tlab, tkl_layer=tlay, pt=pt, q=q, eta=eta, phi0=phi0.astype(np.float64),
    )


def _concat_groups(groups, params):
    keys_trk = ("p", "cov", "truth_seed")
    out = {}
    ng = len(groups)
    out["n_groups"] = ng
    out["params"] = params
    out["n_tracks"] = int(sum(g["n_tracks"] for g in groups))
    for k in keys_trk:
        out[k] = np.concatenate([g[k] for g in groups], axis=1)
    out["x"] = np.concatenate([g["x"] for g in groups])
    out["sector"] = np.concatenate([g["sector"] for g in groups]).astype(np.int32)
    out["group"] = np.concatenate([np.full(g["n_tracks"], i, np.int32) for i, g in enumerate(groups)])
    out["pt"] = np.concatenate([g["pt"] for g in groups])
    for k in ("q", "eta", "phi0"):
        out[k] = np.concatenate([g[k] for g in groups])
    out["truth"] = {k: np.concatenate([g["truth"][k] for g in groups], axis=1) for k in groups[0]["truth"]}
    tk_off = np.cumsum([0] + [g["tkl_y"].size for g in groups])
    tr_off = np.cumsum([0] + [g["n_tracks"] for g in groups])
    ti = []
    for i, g in enumerate(groups):
        t = g["true_idx"].copy()
        t[t >= 0] += tk_off[i]
        ti.append(t)
    out["true_idx"] = np.concatenate(ti, axis=1)
    for k in ("tkl_y", "tkl_z", "tkl_dy", "tkl_det", "tkl_row", "tkl_layer"):
        out[k] = np.concatenate([g[k] for g in groups])
    labs = []
    for i, g in enumerate(groups):
        lab = g["tkl_label"].copy()
        lab[lab >= 0] += tr_off[i]
        labs.append(lab)
    out["tkl_label"] = np.concatenate(labs)
    out["tkl_group"] = np.concatenate([np.full(g["tkl_y"].size, i, np.int32) for i, g in enumerate(groups)])
    out["group_tracks"] = np.array([g["n_tracks"] for g in groups])
    out["group_tracklets"] = np.array([g["tkl_y"].size for g in groups])
    out["tkl_det_row"] = ((out["tkl_det"].astype(np.uint32) << np.uint32(5)) |
                          out["tkl_row"].astype(np.uint32)).astype(np.uint32)
    out["n_tracklets"] = int(out["tkl_y"].size)
    return out


# ---------------------------------------------------------------------------
# workload presets
# ---------------------------------------------------------------------------
# Readings where the paper gives no number:
#  * layers at x = 290 + 13 l cm, flat planes across the full sector width,
#    5 stacks x 18 pad rows of 8 cm (z in [-360, 360] cm), no dead zones;
#  * seeds on the r = 250 cm cylinder, smeared with sigma = (0.1 cm, 0.1 cm,
#    1e-3, 1e-3, 0.01 c/GeV) and rounded to float32;
#  * one thin scatterer of X/X0 = 0.03 per layer, pion mass, Highland width;
#  * sigma_y = 0.04 cm, sigma_dy = 0.0015 cm (0.5 mrad over 3 cm), no Lorentz
#    offset; chi2_max = 13.8155 (0.1 % tail for 2 dof), 4 sigma dy gate;
#  * fakes uniform over sector/stack/layer/row, y uniform over the chamber,
#    z at the row centre, dy uniform in [-1, 1] cm.

WORKLOADS = {
    "c1_small_fp64": dict(n_tracks=1000, pt_dist="exp", fake_ratio=0.2, ineff_frac=0.0,
                          seed=0, params=dict(y_bin_w=8.0, n_yb=16)),
    "c2_frame_20k": dict(n_tracks=20000, pt_dist="exp", fake_ratio=0.5, ineff_frac=0.1,
                         seed=1, params=dict(y_bin_w=8.0, n_yb=16)),
    # 8 cm y bins x 1/4 cm deflection bins over +-4 cm: the road of a seed
    # with a 5 cm position error is cut down by the 4 sigma dy window
    "c5_distortion_450k": dict(n_tracks=450000, pt_dist="pow3", fake_ratio=0.5, ineff_frac=0.1,
                               distortion=(5.0, 15.0), seed=4,
                               params=dict(y_bin_w=8.0, n_yb=16, dy_bin_w=0.25, n_db=32,
                                           n_sigma_road=3.0)),
}


def generate(name=None, *, seed=None, n_tracks=None, params=None, groups=None, **kw):
    """Build a workload: one or more groups with group ids in the tracklet keys.

    Either a preset name (WORKLOADS) with optional overrides, or explicit
    keywords for generate_group.  `groups` > 1 simulates that many groups with
    independent streams (numpy SeedSequence spawn) of the same size.
    """
    spec = {}
    if name is not None:
        spec = dict(WORKLOADS[name])
    spec.update({k: v for k, v in kw.items()})
    pover = dict(spec.pop("params", {}) or {})
    if params:
        pover.update(params)
    P = default_params(**pover)
    if seed is None:
        seed = spec.pop("seed", 0)
    else:
        spec.pop("seed", None)
    if n_tracks is None:
        n_tracks = spec.pop("n_tracks", 1000)
    else:
        spec.pop("n_tracks", None)
    ng = int(groups or 1)
    if ng == 1:
        gs = [generate_group(np.random.default_rng(seed), P, n_tracks, **spec)]
    else:
        ss = np.random.SeedSequence(seed).spawn(ng)
        sizes = n_tracks if np.ndim(n_tracks) else [n_tracks] * ng
        gs = [generate_group(np.random.default_rng(s), P, int(sz), **spec) for s, sz in zip(ss, sizes)]
    return _concat_groups(gs, P)


def generate_frames(seed, n_frames, sizes, fake_ratios, params_over=None, **kw):
    """Many frames with their own sizes and fake ratios (multi-frame batches).

    Each frame is one group; frame f draws from SeedSequence(seed).spawn()[f].
    """
    P = default_params(**(params_over or {}))
    ss = np.random.SeedSequence(seed).spawn(n_frames)
    gs = [generate_group(np.random.default_rng(ss[f]), P, int(sizes[f]),
                         fake_ratio=float(fake_ratios[f]), **kw) for f in range(n_frames)]
    return _concat_groups(gs, P)


def multiframe_64(seed=2, n_frames=64, lo=2000, hi=40000):
    """64 frames, tracks per frame uniform in [2000, 40000], fake ratio per
    frame uniform in [0.2, 0.8], 10 % inefficiency, one group per frame."""
    rng = np.random.default_rng(seed)
    sizes = rng.integers(lo, hi + 1, n_frames)
    ratios = rng.uniform(0.2, 0.8, n_frames)
    return generate_frames(seed, n_frames, sizes, ratios,
                           params_over=dict(y_bin_w=8.0, n_yb=16), pt_dist="exp",
                           ineff_frac=0.1)


def serving_stream(seed=3, n_frames=100, rate_hz=200.0, median=15000, sigma=0.6):
    """Poisson arrival times and lognormal track counts of a frame stream."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_hz, n_frames)
    sizes = np.maximum(1, np.round(rng.lognormal(math.log(median), sigma, n_frames))).astype(np.int64)
    return np.cumsum(gaps), sizes


# ---------------------------------------------------------------------------
# TPC clusters with space-charge distortions (Sect. 2: the calibration the
# TRD matching serves)
# ---------------------------------------------------------------------------
# Readings: pad rows are planes at x_r in the sector frames, n_rows of them
# evenly over [x_in, x_out]; an electron created at local x - dX reaches pad
# row x and is seen displaced by (dY, dZ), with (dX, dY, dZ) a smooth field of
# the sector-local position; clusters carry y, z at the row, float32-rounded,
# with Gaussian noise sigma_cl.

TPC_DEFAULT = dict(x_in=85.0, x_out=245.0, n_rows=64, sigma_cl=0.05, amp=(0.8, 2.0, 1.5))


def tpc_field(x, y, z, amp=TPC_DEFAULT["amp"], x_in=85.0, x_out=245.0):
    """Distortion (dX, dY, dZ) in cm at sector-local (x, y, z): largest at the
    inner radius, smooth in y/x and z."""
    u = (np.asarray(x) - x_in) / (x_out - x_in)
    v = np.asarray(y) / (np.asarray(x) * math.tan(SECTOR_DPHI / 2))
    w = np.asarray(z) / 250.0
    ax, ay, az = amp
    dX = ax * (1.0 - u) * (1.0 - w * w)
    dY = ay * (1.0 - u) ** 2 * (1.0 + 0.3 * v) * (1.0 - 0.5 * w * w)
    dZ = az * (1.0 - u) * w
    return dX, dY, dZ


def tpc_clusters(w, seed=0, *, tpc=None, field=True, noise_free=False, tracks=None):
    """Clusters of the tracks of workload w (all, or the index array
    `tracks`) on the TPC pad rows, outermost first.  Returns a dict: first
    [n+1] (CSR), y, z (float32-valued), row, sector per cluster, and the field
    and track at the true point (truth)."""
    T = dict(TPC_DEFAULT, **(tpc or {}))
    rng = np.random.default_rng(seed)
    dt = np.float64
    sel = np.arange(w["n_tracks"]) if tracks is None else np.asarray(tracks)
    n = int(sel.size)
    bz = w["params"]["bz"]
    cu = -KAPPA * bz * (w["q"][sel] / w["pt"][sel])
    tgl = np.sinh(w["eta"][sel])
    phi0 = w["phi0"][sel]
    xs = np.linspace(T["x_out"], T["x_in"], T["n_rows"])        # outermost first
    tan10 = math.tan(SECTOR_DPHI / 2)
    per_row = []
    alive = np.ones(n, dtype=bool)
    for r, xr in enumerate(xs):
        # sector holding the crossing: start from the one at the cylinder r = xr
        ok0, phi_pos, _, _ = _cross_cylinder(phi0, cu, dt(xr), dt)
        sec = _sector_of(np.cos(phi_pos), np.sin(phi_pos))
        zero = np.zeros(n)
        ok, y, snp, csp, X1, Y1, arc, _ = _cross_plane(zero, zero, phi0, cu, _alpha(sec, dt), xr, dt)
        for _ in range(2):
            out = ok & (np.abs(y) > xr * tan10)
            if not out.any():
                break
            sec = np.where(out, np.mod(sec + np.where(y > 0, 1, -1), N_SECTORS), sec)
            ok2, y2, s2, c2, _, _, a2, _ = _cross_plane(zero, zero, phi0, cu, _alpha(sec, dt), xr, dt)
            ok, y, snp, arc = np.where(out, ok2, ok), np.where(out, y2, y), np.where(out, s2, snp), \
                np.where(out, a2, arc)
        ok = ok0 & ok & (np.abs(y) <= xr * tan10) & (np.abs(snp) < 0.95)
        z = tgl * arc
        if field:
            dX, dY, dZ = tpc_field(xr, y, z, T["amp"], T["x_in"], T["x_out"])
        else:
            dX = dY = dZ = np.zeros(n)
        # the electron seen at row xr started at xr - dX on the same track
        okd, yd, _, _, _, _, arcd, _ = _cross_plane(zero, zero, phi0, cu, _alpha(sec, dt), xr - dX, dt)
        yc = yd + dY
        zc = tgl * arcd + dZ
        ok &= okd & (np.abs(zc) < 250.0)
        if not noise_free:
            yc = yc + rng.standard_normal(n) * T["sigma_cl"]
            zc = zc + rng.standard_normal(n) * T["sigma_cl"]
            yc = yc.astype(np.float32).astype(np.float64)
            zc = zc.astype(np.float32).astype(np.float64)
        alive &= ok   # a track that left the volume stays out
        f = np.sqrt(np.maximum(1.0 - snp * snp, 1e-12))
        per_row.append((alive.copy(), yc, zc, sec, dX, dY, dZ, y, z, snp / f, tgl / f))
    cnt = np.zeros(n, dtype=np.int64)
    for a, *_ in per_row:
        cnt += a
    first = np.zeros(n + 1, dtype=np.int64)
    first[1:] = np.cumsum(cnt)
    m = int(first[-1])
    out = dict(first=first, y=np.zeros(m), z=np.zeros(m), row=np.zeros(m, np.int32),
               sector=np.zeros(m, np.int32), dX=np.zeros(m), dY=np.zeros(m), dZ=np.zeros(m),
               y_true=np.zeros(m), z_true=np.zeros(m), ty_true=np.zeros(m), tz_true=np.zeros(m),
               x_rows=xs, tpc=T)
    pos = first[:-1].copy()
    for r, (a, yc, zc, sec, dX, dY, dZ, yt, zt, ty, tz) in enumerate(per_row):
        ids = np.nonzero(a)[0]
        k = pos[ids]
        out["y"][k], out["z"][k] = yc[ids], zc[ids]
        out["row"][k], out["sector"][k] = r, sec[ids]
        out["dX"][k], out["dY"][k], out["dZ"][k] = dX[ids], dY[ids], dZ[ids]
        out["y_true"][k], out["z_true"][k] = yt[ids], zt[ids]
        out["ty_true"][k], out["tz_true"][k] = ty[ids], tz[ids]
        pos[ids] += 1
    out["n_clusters"] = m
    return out


DESCRIPTIONS = {
    "c1_small_fp64": "pT = 0.3 + Exp(1) GeV/c, |eta| < 0.84, 20% uniform fakes, 8 cm y bins",
    "c2_frame_20k": "pT = 0.3 + Exp(1) GeV/c, 50% uniform fakes, 10% of tracks miss 1-2 layers, "
                    "8 cm y bins",
    "c5_distortion_450k": "pT^-3 above 0.3 GeV/c, 50% uniform fakes, 10% inefficiency, 5-15 cm "
                          "random (y, z) seed displacement, road 3 sigma, 8 cm y x 1/4 cm dy bins",
    "multiframe_64": "64 frames, U[2000, 40000] tracks each, fakes per true tracklet U[0.2, 0.8], "
                     "10% inefficiency, group = frame, 8 cm y bins",
}


def describe(name):
    return DESCRIPTIONS.get(name, name)


def load_workload(name):
    """A named workload: a preset of WORKLOADS or the 64-frame batch."""
    if name == "multiframe_64":
        return multiframe_64()
    return generate(name)


def to_device_layout(w):
    """Float32 SoA arrays in the layout the C ABI reads (component-major)."""
    n = w["n_tracks"]
    return dict(
        p32=np.ascontiguousarray(w["p"].astype(np.float32)),
        cov32=np.ascontiguousarray(w["cov"].astype(np.float32)),
        x32=np.ascontiguousarray(w["x"].astype(np.float32)),
        sector=np.ascontiguousarray(w["sector"].astype(np.int32)),
        group=np.ascontiguousarray(w["group"].astype(np.int32)),
        y32=np.ascontiguousarray(w["tkl_y"].astype(np.float32)),
        z32=np.ascontiguousarray(w["tkl_z"].astype(np.float32)),
        dy32=np.ascontiguousarray(w["tkl_dy"].astype(np.float32)),
        det_row=np.ascontiguousarray(w["tkl_det_row"].astype(np.uint32)),
        tgroup=np.ascontiguousarray(w["tkl_group"].astype(np.int32)),
        n=n,
    )
