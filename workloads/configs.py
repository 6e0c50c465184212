"""Named workloads: geometry, frequency, leaf size, ACA tolerance and the
plane-wave sweep of each scattering problem.

Angles follow the usual spherical convention: r_hat(theta, phi) =
(sin t cos p, sin t sin p, cos t), theta_hat = (cos t cos p, cos t sin p, -sin t).
A monostatic look from (theta, phi) illuminates the body with a plane wave
travelling along k_hat = -r_hat(theta, phi), polarised along theta_hat (VV).
"""

import math

import numpy as np

from .meshes import icosphere, geodesic_sphere, ellipsoid_mesh, flat_plate

C0_LIGHT = 299792458.0


def r_hat(theta, phi):
    return np.stack([np.sin(theta) * np.cos(phi), np.sin(theta) * np.sin(phi),
                     np.cos(theta)], axis=-1)


def theta_hat(theta, phi):
    return np.stack([np.cos(theta) * np.cos(phi), np.cos(theta) * np.sin(phi),
                     -np.sin(theta)], axis=-1)


def monostatic_angles(theta_deg, phi_deg):
    """(khat, pol) arrays (R, 3) for monostatic looks at the given angles.
    phi is reduced to [0, 360) degrees first, so phi = 360 gives exactly the
    vectors of phi = 0 (a full azimuth sweep lists that look twice)."""
    t = np.deg2rad(np.asarray(theta_deg, dtype=np.float64))
    p = np.deg2rad(np.mod(np.asarray(phi_deg, dtype=np.float64), 360.0))
    t, p = np.broadcast_arrays(t, p)
    return -r_hat(t, p), theta_hat(t, p)


def plane_wave_dirs(kind, **kw):
    if kind == "single_minus_z":
        return np.array([[0.0, 0.0, -1.0]]), np.array([[1.0, 0.0, 0.0]])
    if kind == "theta_sweep":
        th = np.arange(kw.get("start", 0.0), kw.get("stop", 180.0) + 1e-9, kw.get("step", 1.0))
        return monostatic_angles(th, np.zeros_like(th))
    if kind == "phi_sweep":
        ph = np.arange(kw.get("start", 0.0), kw.get("stop", 360.0) + 1e-9, kw.get("step", 0.5))
        return monostatic_angles(np.full_like(ph, 90.0), ph)
    if kind == "phi_list":
        ph = np.asarray(kw["phi"], dtype=np.float64)
        return monostatic_angles(np.full_like(ph, 90.0), ph)
    raise ValueError(kind)


def _thomsen_area(a, b, c, p=1.6075):
    return 4.0 * math.pi * (((a * b) ** p + (a * c) ** p + (b * c) ** p) / 3.0) ** (1.0 / p)


def batch_ellipsoids(count=32, freq_hz=600e6, seed=0, n_lo=2000, n_hi=40000):
    """Seed-drawn axis-aligned ellipsoids for the batched workload: semi-axes
    log-uniform in [0.5, 2] m (drawn x, y, z), aspect <= 4, meshed as geodesic
    spheres of frequency nu sized for lambda/10 edges, mapped affinely."""
    rng = np.random.default_rng(seed)
    lam = C0_LIGHT / freq_hz
    out = []
    while len(out) < count:
        ax = np.exp(rng.uniform(math.log(0.5), math.log(2.0), 3))
        if ax.max() / ax.min() > 4.0:
            continue
        s = _thomsen_area(*ax)
        n_target = 1.5 * s / (math.sqrt(3.0) / 4.0 * (lam / 10.0) ** 2)
        nu = max(1, int(round(math.sqrt(n_target / 30.0))))
        n = 30 * nu * nu
        if not (n_lo <= n <= n_hi):
            continue
        out.append((tuple(float(x) for x in ax), nu))
    return out


WORKLOADS = {
    "sphere_s3_200MHz": dict(
        desc="PEC sphere r=1 m, icosphere subdiv 3 (1,280 tris, 1,920 RWG), EFIE 200 MHz, "
             "leaf<=64, ACA 1e-3, 1 RHS x-pol along -z",
        mesh=("icosphere", 3, 1.0), freq_hz=200e6, leaf_max=64, aca_tol=1e-3,
        rhs=("single_minus_z", {}), precision=0),
    "sphere_s5_790MHz": dict(
        desc="PEC sphere r=1 m, icosphere subdiv 5 (20,480 tris, 30,720 RWG), EFIE 790 MHz, "
             "leaf<=128, ACA 1e-3, 181 monostatic RHS theta=0..180 step 1, phi=0, theta-pol",
        mesh=("icosphere", 5, 1.0), freq_hz=790e6, leaf_max=128, aca_tol=1e-3,
        rhs=("theta_sweep", {"start": 0.0, "stop": 180.0, "step": 1.0}), precision=0),
    "sphere_s5_790MHz_mixed": dict(
        desc="as sphere_s5_790MHz in the precision form: BF16 far factors with per-block "
             "FP32 scale, FP32 D^-1 and scaling blocks, FP64 setup, one FP32 residual pass",
        mesh=("icosphere", 5, 1.0), freq_hz=790e6, leaf_max=128, aca_tol=1e-3,
        rhs=("theta_sweep", {"start": 0.0, "stop": 180.0, "step": 1.0}), precision=1),
    "plate_20lambda_300MHz": dict(
        desc="PEC square plate of 20 wavelengths at 300 MHz in the z=0 plane, 200 x 200 squares of "
             "two triangles (lambda/10, 119,600 RWG), open surface, leaf<=128, ACA 1e-3, 181 RHS "
             "theta=0..180 step 1, phi=0, theta-pol (VV)",
        mesh=("plate", 20.0 * C0_LIGHT / 300e6, 200), open=True, freq_hz=300e6, leaf_max=128, aca_tol=1e-3,
        rhs=("theta_sweep", {"start": 0.0, "stop": 180.0, "step": 1.0}), precision=0),
    "plate_2lambda_300MHz": dict(
        desc="PEC square plate of 2 wavelengths at 300 MHz, 20 x 20 squares (lambda/10, 1,160 RWG), "
             "open surface, leaf<=64, ACA 1e-3, 7 RHS theta=0..180 step 30, phi=0, theta-pol",
        mesh=("plate", 2.0 * C0_LIGHT / 300e6, 20), open=True, freq_hz=300e6, leaf_max=64, aca_tol=1e-3,
        rhs=("theta_sweep", {"start": 0.0, "stop": 180.0, "step": 30.0}), precision=0),
    "ellipsoid_4x2x1_300MHz": dict(
        desc="PEC ellipsoid 4x2x1 m, icosphere subdiv 7 mapped affinely (327,680 tris, "
             "491,520 RWG), 300 MHz, leaf<=256, ACA 1e-3, 721 RHS theta=90, phi=0..360 step 0.5",
        mesh=("ellipsoid", 7, (4.0, 2.0, 1.0)), freq_hz=300e6, leaf_max=256, aca_tol=1e-3,
        rhs=("phi_sweep", {"start": 0.0, "stop": 360.0, "step": 0.5}), precision=1),
}


def workload_mesh(spec):
    kind = spec[0]
    if kind == "icosphere":
        return icosphere(spec[1], spec[2])
    if kind == "geodesic":
        return geodesic_sphere(spec[1], spec[2])
    if kind == "ellipsoid":
        xyz, tri = icosphere(spec[1], 1.0)
        return ellipsoid_mesh(xyz, tri, spec[2])
    if kind == "plate":
        return flat_plate(spec[1], spec[2])
    if kind == "geodesic_ellipsoid":
        xyz, tri = geodesic_sphere(spec[1], 1.0)
        return ellipsoid_mesh(xyz, tri, spec[2])
    raise ValueError(kind)


BATCH_WORKLOADS = {
    "ellipsoids32_600MHz": dict(
        desc="32 seed-drawn PEC ellipsoids (semi-axes log-uniform in [0.5, 2] m, aspect <= 4, "
             "numpy default_rng(0)), geodesic meshes at lambda/10 for 600 MHz (8,670-38,880 RWG each, "
             "735,090 in all), leaf<=128, ACA 1e-3, 64 RHS each: theta=90, phi=k*5.625 deg, theta-pol",
        count=32, freq_hz=600e6, seed=0, leaf_max=128, aca_tol=1e-3,
        rhs=("phi_list", {"phi": [k * 5.625 for k in range(64)]})),
    "ellipsoids3_150MHz_small": dict(
        desc="3 seed-drawn PEC ellipsoids as above at 150 MHz (a few thousand RWG in all), "
             "leaf<=64, ACA 1e-3, 8 RHS: theta=90, phi=k*45 deg (small batching case)",
        count=3, freq_hz=150e6, seed=0, leaf_max=64, aca_tol=1e-3, n_lo=100, n_hi=5000,
        rhs=("phi_list", {"phi": [k * 45.0 for k in range(8)]})),
}


def batch_workload(name):
    """Return dict(meshes=[(xyz, tri), ...], axes, freq_hz, leaf_max, aca_tol, khat, pol, ...)."""
    w = dict(BATCH_WORKLOADS[name])
    draws = batch_ellipsoids(w["count"], w["freq_hz"], w["seed"], w.get("n_lo", 2000), w.get("n_hi", 40000))
    meshes = []
    for axes, nu in draws:
        xyz, tri = geodesic_sphere(nu, 1.0)
        meshes.append(ellipsoid_mesh(xyz, tri, axes))
    kind, kw = w["rhs"]
    khat, pol = plane_wave_dirs(kind, **kw)
    w.update(meshes=meshes, axes=[a for a, _ in draws], nu=[n for _, n in draws], khat=khat, pol=pol, name=name)
    return w


def workload(name):
    """Return dict(xyz, tri, freq_hz, leaf_max, aca_tol, khat, pol, ...)."""
    w = dict(WORKLOADS[name])
    xyz, tri = workload_mesh(w["mesh"])
    kind, kw = w["rhs"]
    khat, pol = plane_wave_dirs(kind, **kw)
    w.update(xyz=xyz, tri=tri, khat=khat, pol=pol, name=name)
    w.setdefault("open", False)
    return w
