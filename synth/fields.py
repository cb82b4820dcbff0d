"""Seeded real-space field generators (x fastest: arrays are shaped (Nz, Ny, Nx)).

Every generator takes an explicit ``numpy.random.Generator`` so that a workload
is reproducible from its configuration id and stream number alone.
"""

from __future__ import annotations

import numpy as np

# Order in which the eleven real arrays of one box travel through the solver:
# E (3), B (3), J at the half step (3), rho at the start and at the end of the step.
FIELD_NAMES = ("ex", "ey", "ez", "bx", "by", "bz", "jx", "jy", "jz", "rho_old", "rho_new")

SEED_BASE = 1812_07357 * 10


def rng_for(config_id: int, stream: int = 0) -> np.random.Generator:
    """PCG64 generator for ``(config_id, stream)``; streams are independent children."""
    children = np.random.SeedSequence(SEED_BASE + int(config_id)).spawn(int(stream) + 1)
    return np.random.Generator(np.random.PCG64(children[int(stream)]))


def random_fields(rng: np.random.Generator, shape, nfields: int = 11, scale: float = 1.0):
    """``nfields`` arrays of i.i.d. N(0, scale^2) values, shape (nfields, *shape), float64."""
    return rng.normal(0.0, scale, size=(nfields,) + tuple(shape))


def _coords(shape, d):
    nz, ny, nx = shape
    dz, dy, dx = (d, d, d) if np.isscalar(d) else d
    z = np.arange(nz, dtype=np.float64)[:, None, None] * dz
    y = np.arange(ny, dtype=np.float64)[None, :, None] * dy
    x = np.arange(nx, dtype=np.float64)[None, None, :] * dx
    return x, y, z


def plane_wave_modes(rng: np.random.Generator, shape, nmodes: int, mmax=None):
    """Draw ``nmodes`` grid modes for a sum of plane waves.

    Returns integer mode numbers ``m`` (nmodes, 3) ordered (mx, my, mz), never the
    zero mode and never a Nyquist index, with ``|m_i| <= mmax_i`` (default: the
    largest index below Nyquist); amplitudes a ~ N(0, 1); phases ~ U[0, 2 pi);
    and a random unit vector per mode from which the caller builds a polarisation.
    """
    nz, ny, nx = shape
    lim = np.array([(nx - 1) // 2, (ny - 1) // 2, (nz - 1) // 2])
    if mmax is not None:
        lim = np.minimum(lim, np.broadcast_to(np.asarray(mmax), (3,)))
    modes = []
    while len(modes) < nmodes:
        m = rng.integers(-lim, lim + 1)
        if np.any(m != 0):
            modes.append(m)
    m = np.array(modes, dtype=np.int64)
    amp = rng.normal(0.0, 1.0, size=nmodes)
    phase = rng.uniform(0.0, 2.0 * np.pi, size=nmodes)
    u = rng.normal(0.0, 1.0, size=(nmodes, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    return {"m": m, "amp": amp, "phase": phase, "u": u}


def transverse_unit(u, kvec):
    """Unit vector along the part of ``u`` orthogonal to ``kvec`` (plain Gram-Schmidt)."""
    u = np.asarray(u, dtype=np.float64)
    k = np.asarray(kvec, dtype=np.float64)
    kk = float(k @ k)
    v = u - (u @ k) / kk * k if kk > 0 else u.copy()
    return v / np.linalg.norm(v)


def plane_wave_sum(shape, d, m, amp, phase, evec, bvec, omega=None, t: float = 0.0):
    """Sum of real plane waves sampled on the grid nodes.

    Wave j has spatial phase k_j . x with k_j = 2 pi m_j / (N d) (the grid mode),
    and time phase -omega_j t + phase_j.  E = sum a_j evec_j cos(...),
    B = sum a_j bvec_j cos(...).  Returns (E, B), each (3, Nz, Ny, Nx).
    """
    nz, ny, nx = shape
    dz, dy, dx = (d, d, d) if np.isscalar(d) else d
    x, y, z = _coords(shape, d)
    E = np.zeros((3,) + tuple(shape))
    B = np.zeros((3,) + tuple(shape))
    for j in range(len(amp)):
        kx = 2.0 * np.pi * m[j][0] / (nx * dx)
        ky = 2.0 * np.pi * m[j][1] / (ny * dy)
        kz = 2.0 * np.pi * m[j][2] / (nz * dz)
        w = 0.0 if omega is None else omega[j]
        arg = kx * x + ky * y + kz * z - w * t + phase[j]
        cs = np.cos(arg)
        for c in range(3):
            E[c] += amp[j] * evec[j][c] * cs
            B[c] += amp[j] * bvec[j][c] * cs
    return E, B


def laser_modes(rng: np.random.Generator, shape, d: float, wavelength: float, width: float, nmodes: int = 16,
                transverse: float = 0.6, c: float = 1.0):
    """A laser-like vacuum wave packet as a sum of grid plane waves, for ``plane_wave_sum``.

    Mode numbers are drawn around the grid mode of the laser wavenumber
    k0 = 2 pi / wavelength along +x: m_x ~ round(N(m0, (width * m0)^2)) with
    m0 = N_x d / wavelength (width = 1 / (k0 L), the relative spectral width),
    m_y, m_z ~ round(N(0, transverse^2)); duplicates, the zero mode and
    Nyquist indices are rejected (at most ``nmodes`` distinct modes are kept).
    Phases -k . x_c put every mode's crest at one random centre x_c, so the
    modes add up to a pulse there.  Polarisation: the part of y-hat orthogonal
    to k; B = k-hat x E / c (forward propagation).  Equal amplitudes
    1 / sqrt(number of modes).
    """
    nz, ny, nx = shape
    lim = np.array([(nx - 1) // 2, (ny - 1) // 2, (nz - 1) // 2])
    m0 = nx * d / wavelength
    sx = max(width * m0, 1e-3)
    seen, modes = set(), []
    for _ in range(50 * nmodes):
        if len(modes) == nmodes:
            break
        m = (int(np.rint(rng.normal(m0, sx))), int(np.rint(rng.normal(0.0, transverse))),
             int(np.rint(rng.normal(0.0, transverse))))
        if m in seen or m[0] <= 0 or abs(m[0]) > lim[0] or abs(m[1]) > lim[1] or abs(m[2]) > lim[2]:
            continue
        seen.add(m)
        modes.append(m)
    m = np.array(modes, dtype=np.int64)
    n = len(modes)
    centre = rng.uniform(0.0, 1.0, size=3) * np.array([nx, ny, nz]) * d
    kvec = 2.0 * np.pi * m / (np.array([nx, ny, nz]) * d)
    phase = -(kvec @ centre)
    evec = np.array([transverse_unit((0.0, 1.0, 0.0), k) for k in kvec])
    khat = kvec / np.linalg.norm(kvec, axis=1, keepdims=True)
    bvec = np.cross(khat, evec) / c
    return {"m": m, "amp": np.full(n, 1.0 / np.sqrt(n)), "phase": phase, "evec": evec, "bvec": bvec,
            "centre": centre}


def gaussian_blob(shape, d, center, sigma: float, amplitude: float, direction):
    """Vector field amplitude * direction * exp(-|x - center|^2 / (2 sigma^2)), (3, Nz, Ny, Nx).

    ``center`` is (cx, cy, cz) in grid units of length; ``sigma`` in cells.
    """
    x, y, z = _coords(shape, d)
    dd = d if np.isscalar(d) else d[0]
    r2 = (x - center[0]) ** 2 + (y - center[1]) ** 2 + (z - center[2]) ** 2
    g = amplitude * np.exp(-r2 / (2.0 * (sigma * dd) ** 2))
    direction = np.asarray(direction, dtype=np.float64)
    direction = direction / np.linalg.norm(direction)
    return np.stack([direction[c] * g for c in range(3)])


def laser_pulse(shape, d, wavelength: float, waist: float, length: float, x_center: float, c: float = 1.0):
    """Gaussian laser pulse polarised along y and moving along +x.

    E_y = exp(-((x-xc)/L)^2) exp(-(r_perp/w0)^2) cos(k0 (x-xc)), B_z = E_y / c,
    with k0 = 2 pi / wavelength and r_perp measured from the transverse centre.
    All lengths are in units of length (not cells).  Returns (E, B), each (3, ...).
    """
    nz, ny, nx = shape
    x, y, z = _coords(shape, d)
    dd = d if np.isscalar(d) else d[0]
    yc = 0.5 * (ny - 1) * dd
    zc = 0.5 * (nz - 1) * dd
    k0 = 2.0 * np.pi / wavelength
    env = np.exp(-(((x - x_center) / length) ** 2)) * np.exp(-((y - yc) ** 2 + (z - zc) ** 2) / waist**2)
    ey = env * np.cos(k0 * (x - x_center))
    E = np.zeros((3,) + tuple(shape))
    B = np.zeros((3,) + tuple(shape))
    E[1] = ey
    B[2] = ey / c
    return E, B


def _cic(shape, pos, weight):
    """Cloud-in-cell deposit of ``weight`` at positions ``pos`` (n, 3) in cell units, periodic."""
    nz, ny, nx = shape
    i0 = np.floor(pos).astype(np.int64)
    f = pos - i0
    idx, wts = [], []
    for cx in (0, 1):
        wx = f[:, 0] if cx else 1.0 - f[:, 0]
        ix = (i0[:, 0] + cx) % nx
        for cy in (0, 1):
            wy = f[:, 1] if cy else 1.0 - f[:, 1]
            iy = (i0[:, 1] + cy) % ny
            for cz in (0, 1):
                wz = f[:, 2] if cz else 1.0 - f[:, 2]
                iz = (i0[:, 2] + cz) % nz
                idx.append((iz * ny + iy) * nx + ix)
                wts.append(weight * wx * wy * wz)
    out = np.bincount(np.concatenate(idx), weights=np.concatenate(wts), minlength=nx * ny * nz)
    return out.reshape(shape)


def macro_particle_deposit(rng: np.random.Generator, shape, d: float, dt: float, npart: int, q: float = 0.1):
    """Current and charge of ``npart`` macro-particles making one random-walk step.

    Start positions are uniform on the periodic grid, the displacement is
    U[-1/2, 1/2]^3 cells.  rho_old / rho_new are the CIC charge densities at the
    start / end positions; J = q v is CIC-deposited at the midpoint with
    v = displacement / dt.  Returns (J (3, ...), rho_old, rho_new).
    """
    nz, ny, nx = shape
    box = np.array([nx, ny, nz], dtype=np.float64)
    x0 = rng.uniform(0.0, 1.0, size=(npart, 3)) * box
    step = rng.uniform(-0.5, 0.5, size=(npart, 3))
    x1 = np.mod(x0 + step, box)
    xm = np.mod(x0 + 0.5 * step, box)
    vol = d**3
    rho_old = _cic(shape, x0, np.full(npart, q / vol))
    rho_new = _cic(shape, x1, np.full(npart, q / vol))
    J = np.stack([_cic(shape, xm, q * step[:, c] * d / dt / vol) for c in range(3)])
    return J, rho_old, rho_new


def uneven_decomposition(rng: np.random.Generator, per_axis: int = 4, smin: int = 32, smax: int = 96,
                         guards=(8, 16, 32, 64), orders=(16, 32, 64)):
    """Rectilinear split of a periodic grid into per_axis^3 uneven sub-domains.

    Widths along each axis are drawn U{smin..smax} (one draw per slab, shared by
    the boxes of that slab); every box draws its guard width and stencil order.
    Returns (global_dims (nx, ny, nz), list of dicts with origin, interior, nguard, order).
    """
    widths = [rng.integers(smin, smax + 1, size=per_axis) for _ in range(3)]
    starts = [np.concatenate([[0], np.cumsum(w)[:-1]]) for w in widths]
    gdims = tuple(int(w.sum()) for w in widths)
    boxes = []
    for kz in range(per_axis):
        for ky in range(per_axis):
            for kx in range(per_axis):
                boxes.append({
                    "origin": (int(starts[0][kx]), int(starts[1][ky]), int(starts[2][kz])),
                    "interior": (int(widths[0][kx]), int(widths[1][ky]), int(widths[2][kz])),
                    "nguard": int(rng.choice(guards)),
                    "order": int(rng.choice(orders)),
                })
    return gdims, boxes


def plane_waves_and_blob(rng: np.random.Generator, shape, d: float, nmodes: int, mmax=None, sigma: float = 3.0,
                         amplitude: float = 0.1, c: float = 1.0):
    """(11, Nz, Ny, Nx) float64 arrays: ``nmodes`` vacuum plane waves in E, B plus a Gaussian current blob.

    Modes as ``plane_wave_modes`` (amplitudes N(0, 1), random phases); the
    polarisation is the part of a random unit vector orthogonal to the grid
    wave vector k, and B = k-hat x E / c (forward propagation).  J is a centred
    Gaussian blob of width ``sigma`` cells and peak ``amplitude`` along a seeded
    unit direction, held constant in time; rho_old and rho_new are left zero
    (whoever needs a charge consistent with J computes it).
    """
    nz, ny, nx = shape
    pw = plane_wave_modes(rng, shape, nmodes, mmax=mmax)
    dims = np.array([nx, ny, nz], dtype=np.float64)
    ev, bv = [], []
    for j in range(nmodes):
        kvec = pw["m"][j] / dims
        e = transverse_unit(pw["u"][j], kvec)
        ev.append(e)
        bv.append(np.cross(kvec / np.linalg.norm(kvec), e) / c)
    out = np.zeros((11,) + tuple(shape))
    out[0:3], out[3:6] = plane_wave_sum(shape, d, pw["m"], pw["amp"], pw["phase"], ev, bv)
    direction = rng.normal(0.0, 1.0, size=3)
    centre = tuple(0.5 * n * d for n in (nx, ny, nz))
    out[6:9] = gaussian_blob(shape, d, centre, sigma, amplitude, direction)
    return out
