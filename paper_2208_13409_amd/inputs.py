"""Seeded synthetic workloads (shared by the GPU path, the oracle and the tests).

This module holds only input preparation: initial volume fractions, densities,
specific energies and nodal velocities on the grid.  It does none of the
scheme's arithmetic.  Every random draw uses numpy's PCG64 with the seed
given (problem b of a batch uses ``seed + b``), in the order written below.

A problem is a dict with keys ``nx, ny, gammas, domain, k, rho, e, ux, uy,
t_end, name``; per-material arrays are ``[nmat][ny][nx]``, nodal arrays
``[ny+1][nx+1]``.
"""
import math

import numpy as np

BASE_SEED = 2014


def _cell_centres(nx, ny, domain):
    x0, x1, y0, y1 = domain
    dx, dy = (x1 - x0) / nx, (y1 - y0) / ny
    xc = x0 + (np.arange(nx) + 0.5) * dx
    yc = y0 + (np.arange(ny) + 0.5) * dy
    return np.meshgrid(xc, yc), dx, dy


def _energy(p, rho, gamma):
    return p / ((gamma - 1.0) * rho)


def nodal_velocity(mass, ucell, vcell):
    """Nodal velocity as the mass-weighted mean of the adjacent cells'
    velocities (cells outside the grid are skipped); mass [ny][nx]."""
    ny, nx = mass.shape
    num_u = np.zeros((ny + 1, nx + 1))
    num_v = np.zeros((ny + 1, nx + 1))
    den = np.zeros((ny + 1, nx + 1))
    for dj in (0, 1):
        for di in (0, 1):
            num_u[dj:dj + ny, di:di + nx] += mass * ucell
            num_v[dj:dj + ny, di:di + nx] += mass * vcell
            den[dj:dj + ny, di:di + nx] += mass
    return num_u / den, num_v / den


def sod(nx=400, ny=4):
    """Two-gamma Sod tube on [0,1]x[0,0.01]: x<0.5 rho=1, p=1, gamma 1.4;
    x>=0.5 rho=0.125, p=0.1, gamma 1.6; at rest; t_end 0.2."""
    domain = (0.0, 1.0, 0.0, 0.01 * ny / 4.0)
    (X, Y), dx, dy = _cell_centres(nx, ny, domain)
    left = X < 0.5
    gam = [1.4, 1.6]
    k = np.stack([left, ~left]).astype(float)
    rho = np.stack([np.where(left, 1.0, 0.0), np.where(left, 0.0, 0.125)])
    p = np.stack([np.where(left, 1.0, 0.0), np.where(left, 0.0, 0.1)])
    e = np.zeros_like(rho)
    for a in range(2):
        m = k[a] > 0
        e[a][m] = _energy(p[a][m], rho[a][m], gam[a])
    z = np.zeros((ny + 1, nx + 1))
    return dict(name=f"sod_{nx}x{ny}", nx=nx, ny=ny, gammas=gam, domain=domain, k=k,
                rho=rho, e=e, ux=z, uy=z.copy(), t_end=0.2)


def triple_point(scale=1):
    """Triple-point problem on [0,7]x[0,3] with 448s x 192s cells: material 0
    (x<1: rho 1, p 1, gamma 1.5), material 1 (x>1, y>1.5: rho 1, p 0.1,
    gamma 1.4), material 2 (x>1, y<1.5: rho 0.125, p 0.1, gamma 1.5); at rest,
    t_end 3.5.  The material boundaries lie on cell faces."""
    nx, ny = 448 * scale, 192 * scale
    domain = (0.0, 7.0, 0.0, 3.0)
    (X, Y), dx, dy = _cell_centres(nx, ny, domain)
    m0 = X < 1.0
    m1 = (~m0) & (Y > 1.5)
    m2 = (~m0) & (Y < 1.5)
    gam = [1.5, 1.4, 1.5]
    k = np.stack([m0, m1, m2]).astype(float)
    rho = np.stack([np.where(m0, 1.0, 0.0), np.where(m1, 1.0, 0.0), np.where(m2, 0.125, 0.0)])
    p = np.stack([np.where(m0, 1.0, 0.0), np.where(m1, 0.1, 0.0), np.where(m2, 0.1, 0.0)])
    e = np.zeros_like(rho)
    for a in range(3):
        m = k[a] > 0
        e[a][m] = _energy(p[a][m], rho[a][m], gam[a])
    z = np.zeros((ny + 1, nx + 1))
    return dict(name=f"triple_point_{nx}x{ny}", nx=nx, ny=ny, gammas=gam, domain=domain,
                k=k, rho=rho, e=e, ux=z, uy=z.copy(), t_end=3.5)


def _subsampled_fraction(inside, nx, ny, domain, cells, sub):
    """Fraction of each listed cell (i, j) for which inside(x, y) holds, from
    sub x sub point samples at the sub-cell centres."""
    x0, x1, y0, y1 = domain
    dx, dy = (x1 - x0) / nx, (y1 - y0) / ny
    off = (np.arange(sub) + 0.5) / sub
    ox, oy = np.meshgrid(off, off)
    out = np.empty(len(cells))
    for n, (i, j) in enumerate(cells):
        xs = x0 + (i + ox) * dx
        ys = y0 + (j + oy) * dy
        out[n] = inside(xs, ys).mean()
    return out


def circle_fraction(nx, ny, domain, cx, cy, r, sub=64):
    """Volume fraction of the disc (cx, cy, r) in each cell, exact 0/1 away
    from the circle and sub x sub point sampling on cells it crosses."""
    (X, Y), dx, dy = _cell_centres(nx, ny, domain)
    dist = np.hypot(X - cx, Y - cy)
    half_diag = 0.5 * math.hypot(dx, dy)
    k = (dist < r).astype(float)
    cut = np.argwhere(np.abs(dist - r) <= half_diag)
    if len(cut):
        cells = [(int(i), int(j)) for j, i in cut]
        frac = _subsampled_fraction(lambda x, y: np.hypot(x - cx, y - cy) < r,
                                    nx, ny, domain, cells, sub)
        for (i, j), f in zip(cells, frac):
            k[j, i] = f
    return k


GRID_LADDER = [(64, 64), (128, 64), (128, 128), (256, 128), (256, 256), (512, 256)]


def shock_bubble(seed, grid=None):
    """One shock–bubble problem: ambient gas (gamma 1.4, rho 1, p 1) with a
    light bubble (gamma 1.67, rho 0.14, p 1) of radius r ~ U[0.1, 0.3] centred
    at (0.15 + r, 0.5), hit by a planar shock of Mach M ~ U[1.2, 3] whose front
    is at x = 0.1 (post-shock state from the Rankine–Hugoniot relations).
    Domain [0, nx/ny] x [0, 1], square cells; grid drawn from GRID_LADDER
    unless given.  Draw order: grid index, M, r."""
    rng = np.random.Generator(np.random.PCG64(seed))
    gi = int(rng.integers(len(GRID_LADDER)))
    mach = float(rng.uniform(1.2, 3.0))
    r = float(rng.uniform(0.1, 0.3))
    nx, ny = grid if grid is not None else GRID_LADDER[gi]
    domain = (0.0, nx / ny, 0.0, 1.0)
    g0, g1 = 1.4, 1.67
    rho1, p1 = 1.0, 1.0
    c1 = math.sqrt(g0 * p1 / rho1)
    p2 = p1 * (1.0 + 2.0 * g0 / (g0 + 1.0) * (mach * mach - 1.0))
    rho2 = rho1 * (g0 + 1.0) * mach * mach / ((g0 - 1.0) * mach * mach + 2.0)
    u2 = c1 * 2.0 / (g0 + 1.0) * (mach - 1.0 / mach)
    (X, Y), dx, dy = _cell_centres(nx, ny, domain)
    kb = circle_fraction(nx, ny, domain, 0.15 + r, 0.5, r)
    post = X < 0.1
    k = np.stack([1.0 - kb, kb])
    rho = np.stack([np.where(post, rho2, rho1), np.full((ny, nx), 0.14)])
    p = np.stack([np.where(post, p2, p1), np.full((ny, nx), 1.0)])
    e = np.stack([_energy(p[0], rho[0], g0), _energy(p[1], rho[1], g1)])
    rho = np.where(k > 0, rho, 0.0)
    e = np.where(k > 0, e, 0.0)
    ucell = np.where(post, u2, 0.0)
    mass = (k * rho).sum(0)
    ux, uy = nodal_velocity(mass, ucell, np.zeros_like(ucell))
    return dict(name=f"shock_bubble_{seed}_{nx}x{ny}", nx=nx, ny=ny, gammas=[g0, g1],
                domain=domain, k=k, rho=rho, e=e, ux=ux, uy=uy, t_end=0.25,
                mach=mach, radius=r)


def _stiff_energy(p, rho, gamma, pinf):
    """specific internal energy of the stiffened gas p = (gamma-1) rho e - pi"""
    return (p + pinf) / ((gamma - 1.0) * rho)


def water_air_tube(nx=400, ny=4):
    """Water-air shock tube of §5.2's kind on [0,1] m x [0, ny/nx]: compressed
    water (rho 1000 kg/m^3, p 1e9 Pa, stiffened gas gamma 7, pi 2.1e9 Pa) for
    x < 0.5 against air (rho 50, p 1e5, perfect gas gamma 1.4), at rest;
    t_end 1.2e-4 s (the rarefaction has not reached the wall)."""
    domain = (0.0, 1.0, 0.0, ny / nx)
    (X, Y), dx, dy = _cell_centres(nx, ny, domain)
    left = X < 0.5
    gam, pinfs = [7.0, 1.4], [2.1e9, 0.0]
    k = np.stack([left, ~left]).astype(float)
    rho = np.stack([np.where(left, 1000.0, 0.0), np.where(left, 0.0, 50.0)])
    e = np.stack([np.where(left, _stiff_energy(1e9, 1000.0, 7.0, 2.1e9), 0.0),
                  np.where(left, 0.0, _energy(1e5, 50.0, 1.4))])
    z = np.zeros((ny + 1, nx + 1))
    return dict(name=f"water_air_tube_{nx}x{ny}", nx=nx, ny=ny, gammas=gam, pinfs=pinfs, domain=domain,
                k=k, rho=rho, e=e, ux=z, uy=z.copy(), t_end=1.2e-4)


def water_impact(scale=1):
    """Water-drop impact of §5.2 (air perfect gas, water stiffened gas) on
    the paper's mesh of 320 x 160 cells (times `scale`) over [0, 10] x [0, 5]
    cm, in SI units.  The paper gives the states (air: rho 1.29, u -1000 m/s;
    water wall at rest and drop at -1000 m/s, both rho 1000, gamma 7,
    pi 2.1e9 Pa; p 1e5 Pa everywhere) but not the geometry, which its
    figures held.  Reading: the water wall fills x < 1 cm, the drop is a disc
    of radius 1.2 cm centred at (4, 2.5) cm.  Material 0 is air, material 1
    water (wall and drop).  t_end 6 ms."""
    nx, ny = 320 * scale, 160 * scale
    domain = (0.0, 0.1, 0.0, 0.05)
    (X, Y), dx, dy = _cell_centres(nx, ny, domain)
    kd = circle_fraction(nx, ny, domain, 0.04, 0.025, 0.012)
    wall = X < 0.01
    kw = np.where(wall, 1.0, kd)
    k = np.stack([1.0 - kw, kw])
    gam, pinfs = [1.4, 7.0], [0.0, 2.1e9]
    rho = np.stack([np.full((ny, nx), 1.29), np.full((ny, nx), 1000.0)])
    e = np.stack([np.full((ny, nx), _energy(1e5, 1.29, 1.4)),
                  np.full((ny, nx), _stiff_energy(1e5, 1000.0, 7.0, 2.1e9))])
    rho = np.where(k > 0, rho, 0.0)
    e = np.where(k > 0, e, 0.0)
    ucell = np.where(wall, 0.0, -1000.0)
    mass = (k * rho).sum(0)
    ux, uy = nodal_velocity(mass, ucell, np.zeros_like(ucell))
    return dict(name=f"water_impact_{nx}x{ny}", nx=nx, ny=ny, gammas=gam, pinfs=pinfs, domain=domain,
                k=k, rho=rho, e=e, ux=ux, uy=uy, t_end=6e-3)


def shock_bubble_batch(n=256, seed=BASE_SEED):
    return [shock_bubble(seed + b) for b in range(n)]


def four_quadrant(seed, n=None):
    """One four-quadrant Riemann problem on [0,1]^2 with n x n cells (n
    log-uniform on [128, 1024] rounded to a multiple of 32 unless given):
    material 0 in the NE and SW quadrants, material 1 in NW and SE, each
    quadrant with rho ~ U[0.1,2], p ~ U[0.1,1], u, v ~ U[-1,1]; gamma of each
    material drawn from {1.4, 1.67}; t_end 0.25.  Draw order: n, the two
    gammas, then (rho, p, u, v) for NE, NW, SW, SE."""
    rng = np.random.Generator(np.random.PCG64(seed))
    nn = float(np.exp(rng.uniform(math.log(128.0), math.log(1024.0))))
    gam = [float(rng.choice([1.4, 1.67])), float(rng.choice([1.4, 1.67]))]
    quads = []
    for _ in range(4):
        quads.append((rng.uniform(0.1, 2.0), rng.uniform(0.1, 1.0),
                      rng.uniform(-1.0, 1.0), rng.uniform(-1.0, 1.0)))
    if n is None:
        n = int(max(128, min(1024, 32 * round(nn / 32.0))))
    domain = (0.0, 1.0, 0.0, 1.0)
    (X, Y), dx, dy = _cell_centres(n, n, domain)
    east, north = X > 0.5, Y > 0.5
    qid = np.where(north, np.where(east, 0, 1), np.where(east, 3, 2))  # NE, NW, SW, SE
    mat1 = (qid == 1) | (qid == 3)
    k = np.stack([~mat1, mat1]).astype(float)
    qr = np.array([q[0] for q in quads])[qid]
    qp = np.array([q[1] for q in quads])[qid]
    qu = np.array([q[2] for q in quads])[qid]
    qv = np.array([q[3] for q in quads])[qid]
    rho = np.stack([np.where(mat1, 0.0, qr), np.where(mat1, qr, 0.0)])
    e = np.stack([np.where(mat1, 0.0, _energy(qp, qr, gam[0])),
                  np.where(mat1, _energy(qp, qr, gam[1]), 0.0)])
    ux, uy = nodal_velocity(qr, qu, qv)
    return dict(name=f"four_quadrant_{seed}_{n}", nx=n, ny=n, gammas=gam, domain=domain,
                k=k, rho=rho, e=e, ux=ux, uy=uy, t_end=0.25)


def poisson_arrivals(n_req=1000, rate=50.0, seed=BASE_SEED):
    """Arrival times (s) of a Poisson stream with the given mean rate."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.cumsum(rng.exponential(1.0 / rate, size=n_req))


def random_mixed(seed, nx, ny, nmat=2, blobs=3, speed=0.3, gammas=None, domain=None):
    """Random smooth multimaterial state for parity tests: material 0 fills
    the background, each later material gets `blobs` discs (fractions by 8x8
    sub-sampling, later discs overwrite earlier ones), every material a smooth
    random density and pressure field, and a smooth random nodal velocity of
    magnitude ~ speed.  Draw order: gammas (if not given), disc centres and
    radii, field phases and amplitudes."""
    rng = np.random.Generator(np.random.PCG64(seed))
    if gammas is None:
        gammas = [float(g) for g in rng.uniform(1.3, 1.8, size=nmat)]
    if domain is None:
        domain = (0.0, 1.0, 0.0, ny / nx)
    x0, x1, y0, y1 = domain
    (X, Y), dx, dy = _cell_centres(nx, ny, domain)
    owner_frac = [np.ones((ny, nx))]
    for a in range(1, nmat):
        ka = np.zeros((ny, nx))
        for _ in range(blobs):
            cx = rng.uniform(x0, x1)
            cy = rng.uniform(y0, y1)
            r = rng.uniform(0.08, 0.25) * min(x1 - x0, y1 - y0)
            kd = circle_fraction(nx, ny, domain, cx, cy, r, sub=8)
            ka = ka + kd * (1.0 - ka)
        owner_frac.append(ka)
    # later materials take their fraction out of everything before them
    k = np.zeros((nmat, ny, nx))
    rest = np.ones((ny, nx))
    for a in range(nmat - 1, 0, -1):
        k[a] = owner_frac[a] * rest
        rest = rest - k[a]
    k[0] = rest
    k = np.clip(k, 0.0, 1.0)
    k[k < 1e-6] = 0.0
    k /= k.sum(0, keepdims=True)
    rho = np.zeros((nmat, ny, nx))
    e = np.zeros((nmat, ny, nx))
    for a in range(nmat):
        ph = rng.uniform(0, 2 * math.pi, size=4)
        amp = rng.uniform(0.0, 0.3, size=2)
        r0 = rng.uniform(0.3, 2.0)
        p0 = rng.uniform(0.3, 2.0)
        ra = r0 * (1.0 + amp[0] * np.sin(2 * math.pi * X / (x1 - x0) + ph[0]) *
                   np.cos(2 * math.pi * Y / (y1 - y0) + ph[1]))
        pa = p0 * (1.0 + amp[1] * np.sin(4 * math.pi * X / (x1 - x0) + ph[2]) *
                   np.sin(2 * math.pi * Y / (y1 - y0) + ph[3]))
        rho[a] = np.where(k[a] > 0, ra, 0.0)
        e[a] = np.where(k[a] > 0, _energy(pa, ra, gammas[a]), 0.0)
    xn = np.linspace(x0, x1, nx + 1)
    yn = np.linspace(y0, y1, ny + 1)
    XN, YN = np.meshgrid(xn, yn)
    ph = rng.uniform(0, 2 * math.pi, size=4)
    ux = speed * np.sin(2 * math.pi * XN / (x1 - x0) + ph[0]) * np.cos(2 * math.pi * YN / (y1 - y0) + ph[1])
    uy = speed * np.cos(2 * math.pi * XN / (x1 - x0) + ph[2]) * np.sin(2 * math.pi * YN / (y1 - y0) + ph[3])
    return dict(name=f"random_mixed_{seed}_{nx}x{ny}_{nmat}", nx=nx, ny=ny, gammas=gammas,
                domain=domain, k=k, rho=rho, e=e, ux=ux, uy=uy, t_end=1.0)


def square_advection(n=100, u=(5.0, 5.0), rho_in=10.0, rho_out=0.1, nmat=1, gamma=1.4):
    """Square of density rho_in in a field of rho_out on [0,1]^2 with a
    constant prescribed velocity (advection tests with prescribed velocities).
    With nmat=2 the square is material 1 and the field material 0."""
    domain = (0.0, 1.0, 0.0, 1.0)
    (X, Y), dx, dy = _cell_centres(n, n, domain)
    sq = (np.abs(X - 0.3) < 0.1) & (np.abs(Y - 0.3) < 0.1)
    if nmat == 1:
        k = np.ones((1, n, n))
        rho = np.where(sq, rho_in, rho_out)[None]
        e = np.full((1, n, n), 1.0)
        gam = [gamma]
    else:
        k = np.stack([~sq, sq]).astype(float)
        rho = np.stack([np.where(sq, 0.0, rho_out), np.where(sq, rho_in, 0.0)])
        e = np.stack([np.where(sq, 0.0, 1.0), np.where(sq, 1.0, 0.0)])
        gam = [gamma, gamma]
    ux = np.full((n + 1, n + 1), float(u[0]))
    uy = np.full((n + 1, n + 1), float(u[1]))
    return dict(name=f"square_advection_{n}", nx=n, ny=n, gammas=gam, domain=domain, k=k,
                rho=rho, e=e, ux=ux, uy=uy, t_end=0.02)


def solid_rotation(n=100, omega=2.0 * math.pi, rho_in=10.0, rho_out=0.1, nmat=1, gamma=1.4):
    """Solid rotation of §5.1: a square of density rho_in in a field of
    rho_out on [0,1]^2, turning about the centre with the prescribed velocity
    u = r omega e_theta (kinematic runs keep it at every step); one turn is
    t = 2 pi / omega (t_end).  The paper does not place the square; here it is
    the square of side 0.2 centred at (0.5, 0.7).  The rotation is confined to
    the inscribed disc r <= 0.5 (at rest outside it), so that the flow is
    tangent to the reflective walls: the rigid rotation of the whole square
    domain would push into the walls at its corners.  With nmat=2 the square
    is material 1 and the field material 0."""
    domain = (0.0, 1.0, 0.0, 1.0)
    (X, Y), dx, dy = _cell_centres(n, n, domain)
    sq = (np.abs(X - 0.5) < 0.1) & (np.abs(Y - 0.7) < 0.1)
    if nmat == 1:
        k = np.ones((1, n, n))
        rho = np.where(sq, rho_in, rho_out)[None]
        e = np.full((1, n, n), 1.0)
        gam = [gamma]
    else:
        k = np.stack([~sq, sq]).astype(float)
        rho = np.stack([np.where(sq, 0.0, rho_out), np.where(sq, rho_in, 0.0)])
        e = np.stack([np.where(sq, 0.0, 1.0), np.where(sq, 1.0, 0.0)])
        gam = [gamma, gamma]
    xn = np.arange(n + 1) / n
    XN, YN = np.meshgrid(xn, xn)
    inside = np.hypot(XN - 0.5, YN - 0.5) <= 0.5
    ux = np.where(inside, -omega * (YN - 0.5), 0.0)
    uy = np.where(inside, omega * (XN - 0.5), 0.0)
    return dict(name=f"solid_rotation_{n}", nx=n, ny=n, gammas=gam, domain=domain, k=k,
                rho=rho, e=e, ux=ux, uy=uy, t_end=2.0 * math.pi / omega)


def restart_state(fields, A):
    """An initial state (k, rho, e, ux, uy) that lr_set_state accepts, from a
    problem's conserved fields (dict with vol, mass, ie [nmat][ny][nx] and
    ux, uy [ny+1][nx+1]; A = cell area): traces below 1e-14 of a cell, and
    any with a non-positive mass or a negative energy, are dropped and their
    fraction given to the cell's largest material."""
    V, M, E = fields["vol"], fields["mass"], fields["ie"]
    keep = (V > 1e-14 * A) & (M > 0.0) & (E >= 0.0)
    k = np.where(keep, V / A, 0.0)
    big = np.argmax(k, axis=0)
    rows = np.arange(k.shape[1])[:, None]
    cols = np.arange(k.shape[2])[None, :]
    k[big, rows, cols] = 0.0
    k[big, rows, cols] = 1.0 - k.sum(0)
    rho = np.where(keep, M / np.where(keep, V, 1.0), 0.0)
    e = np.where(keep, E / np.where(keep, M, 1.0), 0.0)
    return k, rho, e, fields["ux"], fields["uy"]
