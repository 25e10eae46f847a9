"""A second reader of one DirectCF Lagrange-Remap step, in 50-digit arithmetic.

TEST INFRASTRUCTURE (the scope table's brute-force pin of the oracle).  It is
written from the readings of the scheme in the paper's order (Lagrangian
phase of §1.2 and §4.1, DirectCF regions of §2.3, interface and partial
volumes of §4.4, reconstruction of §2.1.1 and §3.3, primal and dual update of
§2.3), one cell, face, corner or node at a time, with Python loops and
mpmath numbers, on tiny grids.  It shares nothing with the C oracle: areas
of a rectangle cut by a half-plane come from integrating the cut length
along x (exact on each linear piece), interface offsets from bisection in 50
digits, quadrilateral areas from two triangles.  Only reflective walls and
the default options are covered; kinematic mode and order 1 are switches.
"""
import mpmath as mp

mp.mp.dps = 50
ZERO, HALF, ONE, TWO = mp.mpf(0), mp.mpf("0.5"), mp.mpf(1), mp.mpf(2)
QUARTER = mp.mpf("0.25")


def mref_cell(i, n):
    """index of the real cell a ghost cell mirrors"""
    return -1 - i if i < 0 else (2 * n - 1 - i if i >= n else i)


def mref_node(i, n):
    """index of the real node a ghost node mirrors"""
    return -i if i < 0 else (2 * n - i if i > n else i)


def van_leer(dm, dp):
    """the harmonic mean of two one-sided slopes of the same sign, else 0"""
    return TWO * dm * dp / (dm + dp) if dm * dp > 0 else ZERO


def halfplane_area(x0, x1, y0, y1, nx, ny, s):
    """area of {(x, y) in [x0,x1] x [y0,y1] : nx x + ny y >= s}: the cut
    length along y is piecewise linear in x; integrate it exactly"""
    if not (x1 > x0 and y1 > y0):
        return ZERO
    H = y1 - y0

    def length(x):
        if ny == 0:
            return H if nx * x >= s else ZERO
        t = (s - nx * x) / ny
        if ny > 0:
            v = y1 - max(y0, t)
        else:
            v = min(y1, t) - y0
        return min(max(v, ZERO), H)

    pts = [x0, x1]
    if nx != 0:
        for yb in (y0, y1):
            xb = (s - ny * yb) / nx
            if x0 < xb < x1:
                pts.append(xb)
    elif ny == 0:
        pass
    pts.sort()
    if ny == 0 and nx != 0:
        xb = s / nx
        if x0 < xb < x1:
            pts.append(xb)
            pts.sort()
    area = ZERO
    for a, b in zip(pts[:-1], pts[1:]):
        if b > a:
            # linear on (a, b): the midpoint rule is exact (and avoids the
            # jump of the ny = 0 case sitting on a breakpoint)
            area += (b - a) * length((a + b) / 2)
    return area


def interface_offset(R, n, frac):
    """s such that the part of rectangle R = (x0, x1, y0, y1) where n.x >= s
    has area frac |R|: bisection (the area falls as s grows)"""
    x0, x1, y0, y1 = R
    corners = [n[0] * x + n[1] * y for x in (x0, x1) for y in (y0, y1)]
    lo, hi = min(corners), max(corners)
    target = frac * (x1 - x0) * (y1 - y0)
    for _ in range(170):
        mid = (lo + hi) / 2
        if halfplane_area(x0, x1, y0, y1, n[0], n[1], mid) > target:
            lo = mid
        else:
            hi = mid
    return (lo + hi) / 2


def tri_area(ax, ay, bx, by, cx, cy):
    return abs((bx - ax) * (cy - ay) - (cx - ax) * (by - ay)) / 2


class MiniStep:
    """One problem: nx x ny cells, materials with gamma (and pi), reflective
    walls.  State: V, M, E [m][j][i] and nodal ux, uy [J][I], all mpf."""

    def __init__(self, nx, ny, gammas, domain, pinfs=None, cfl=0.5, a1=0.5, a2=1.0, k_eps=1e-10,
                 recon_order=2, kinematic=False, fixed_dt=0.0):
        self.nx, self.ny, self.nm = nx, ny, len(gammas)
        self.g = [mp.mpf(x) for x in gammas]
        self.pi = [mp.mpf(x) for x in (pinfs or [0.0] * self.nm)]
        self.x0, self.x1, self.y0, self.y1 = (mp.mpf(v) for v in domain)
        self.dx = (self.x1 - self.x0) / nx
        self.dy = (self.y1 - self.y0) / ny
        self.A = self.dx * self.dy
        self.cfl, self.a1, self.a2 = mp.mpf(cfl), mp.mpf(a1), mp.mpf(a2)
        self.k_eps = mp.mpf(k_eps)
        self.order = recon_order
        self.kinematic = kinematic
        self.fixed_dt = mp.mpf(fixed_dt)
        self.t = ZERO

    # ------------------------------------------------------------ state
    def set_state(self, k, rho, e, ux, uy):
        nx, ny, nm = self.nx, self.ny, self.nm
        self.V = [[[mp.mpf(float(k[a][j][i])) * self.A for i in range(nx)] for j in range(ny)] for a in range(nm)]
        self.M = [[[self.V[a][j][i] * mp.mpf(float(rho[a][j][i])) if k[a][j][i] > 0 else ZERO
                    for i in range(nx)] for j in range(ny)] for a in range(nm)]
        self.E = [[[self.M[a][j][i] * mp.mpf(float(e[a][j][i])) for i in range(nx)] for j in range(ny)]
                  for a in range(nm)]
        self.ux = [[mp.mpf(float(ux[J][I])) for I in range(nx + 1)] for J in range(ny + 1)]
        self.uy = [[mp.mpf(float(uy[J][I])) for I in range(nx + 1)] for J in range(ny + 1)]
        for J in range(ny + 1):
            for I in range(nx + 1):
                if I in (0, nx):
                    self.ux[J][I] = ZERO
                if J in (0, ny):
                    self.uy[J][I] = ZERO

    # ------------------------------------------------------------ helpers
    def cell(self, arr, i, j):
        return arr[mref_cell(j, self.ny)][mref_cell(i, self.nx)]

    def node_vec(self, ax, ay, I, J):
        """a nodal vector at any node; beyond a wall the normal part flips"""
        rI, rJ = mref_node(I, self.nx), mref_node(J, self.ny)
        vx, vy = ax[rJ][rI], ay[rJ][rI]
        return (-vx if rI != I else vx), (-vy if rJ != J else vy)

    def node_pos(self, I, J):
        """Lagrangian position of any node; beyond a wall, the reflection"""
        rI, rJ = mref_node(I, self.nx), mref_node(J, self.ny)
        x = self.x0 + rI * self.dx + self.dpx[rJ][rI]
        y = self.y0 + rJ * self.dy + self.dpy[rJ][rI]
        if rI != I:
            x = TWO * (self.x0 if I < 0 else self.x1) - x
        if rJ != J:
            y = TWO * (self.y0 if J < 0 else self.y1) - y
        return x, y

    def disp(self, I, J):
        return self.node_vec(self.dpx, self.dpy, I, J)

    def eos(self, a, rho, e):
        return (self.g[a] - 1) * rho * e - self.pi[a]

    def quad(self, i, j, hx, hy):
        """area of cell (i, j) with its nodes moved by (hx, hy) (node arrays),
        two triangles split along the BR-TL diagonal"""
        X = lambda I, J: self.x0 + I * self.dx + hx[J][I]
        Y = lambda I, J: self.y0 + J * self.dy + hy[J][I]
        bl, br = (X(i, j), Y(i, j)), (X(i + 1, j), Y(i + 1, j))
        tl, tr = (X(i, j + 1), Y(i, j + 1)), (X(i + 1, j + 1), Y(i + 1, j + 1))
        return tri_area(*bl, *br, *tl) + tri_area(*br, *tr, *tl)

    # ------------------------------------------------------------ step
    def step(self):
        nx, ny, nm, A = self.nx, self.ny, self.nm, self.A
        dx, dy = self.dx, self.dy
        cells = [(i, j) for j in range(ny) for i in range(nx)]
        nodes = [(I, J) for J in range(ny + 1) for I in range(nx + 1)]
        V, M, E = self.V, self.M, self.E
        # derived state at t^n
        pres = [[[V[a][j][i] > self.k_eps * A for i in range(nx)] for j in range(ny)] for a in range(nm)]
        k = [[[V[a][j][i] / A for i in range(nx)] for j in range(ny)] for a in range(nm)]
        rho = [[[M[a][j][i] / V[a][j][i] if pres[a][j][i] else ZERO for i in range(nx)] for j in range(ny)]
               for a in range(nm)]
        e = [[[E[a][j][i] / M[a][j][i] if M[a][j][i] > 0 else ZERO for i in range(nx)] for j in range(ny)]
             for a in range(nm)]
        P = [[[self.eos(a, rho[a][j][i], e[a][j][i]) if pres[a][j][i] else ZERO for i in range(nx)]
              for j in range(ny)] for a in range(nm)]
        Mc = [[sum(M[a][j][i] for a in range(nm)) for i in range(nx)] for j in range(ny)]
        cs = [[ZERO] * nx for _ in range(ny)]
        for i, j in cells:
            rc2 = sum(k[a][j][i] * (self.g[a] * P[a][j][i] + self.pi[a]) for a in range(nm) if pres[a][j][i])
            rhoc = Mc[j][i] / A
            cs[j][i] = mp.sqrt(rc2 / rhoc) if rhoc > 0 and rc2 > 0 else ZERO
        # time step: the Courant bound over every cell and each of its nodes
        dt = None
        for i, j in cells:
            for I, J in ((i, j), (i + 1, j), (i, j + 1), (i + 1, j + 1)):
                b = min(dx / (cs[j][i] + abs(self.ux[J][I])), dy / (cs[j][i] + abs(self.uy[J][I])))
                dt = b if dt is None else min(dt, b)
        dt = self.fixed_dt if self.fixed_dt > 0 else self.cfl * dt
        # nodal mass from the four cells around each node (mirrored)
        mp_ = [[QUARTER * (self.cell(Mc, I - 1, J - 1) + self.cell(Mc, I, J - 1) + self.cell(Mc, I - 1, J) +
                           self.cell(Mc, I, J)) for I in range(nx + 1)] for J in range(ny + 1)]
        eL = [[[e[a][j][i] for i in range(nx)] for j in range(ny)] for a in range(nm)]
        if self.kinematic:
            uhx, uhy = self.ux, self.uy
            uLx, uLy = self.ux, self.uy
        else:
            # pseudo-viscosity
            Q = [[ZERO] * nx for _ in range(ny)]
            L = mp.sqrt(A)
            for i, j in cells:
                ux, uy = self.ux, self.uy
                div = (ux[j][i + 1] + ux[j + 1][i + 1] - ux[j][i] - ux[j + 1][i]) / (2 * dx) + \
                      (uy[j + 1][i] + uy[j + 1][i + 1] - uy[j][i] - uy[j][i + 1]) / (2 * dy)
                if div < 0:
                    Q[j][i] = (Mc[j][i] / A) * (self.a1 * L * cs[j][i] * abs(div) + self.a2 * L * L * div * div)
            # predictor
            hx = [[dt / 2 * self.ux[J][I] for I in range(nx + 1)] for J in range(ny + 1)]
            hy = [[dt / 2 * self.uy[J][I] for I in range(nx + 1)] for J in range(ny + 1)]
            Ph = [[[ZERO] * nx for _ in range(ny)] for a in range(nm)]
            S = [[ZERO] * nx for _ in range(ny)]
            for i, j in cells:
                Vh = self.quad(i, j, hx, hy)
                Pc = ZERO
                for a in range(nm):
                    if not pres[a][j][i]:
                        continue
                    rh = M[a][j][i] / (k[a][j][i] * Vh)
                    eh = e[a][j][i] - (P[a][j][i] + Q[j][i]) * (1 / rh - 1 / rho[a][j][i])
                    Ph[a][j][i] = self.eos(a, rh, eh)
                    Pc += k[a][j][i] * Ph[a][j][i]
                S[j][i] = Pc + Q[j][i]
            uhx = [[ZERO] * (nx + 1) for _ in range(ny + 1)]
            uhy = [[ZERO] * (nx + 1) for _ in range(ny + 1)]
            for I, J in nodes:
                sNE, sSE = self.cell(S, I, J), self.cell(S, I, J - 1)
                sNW, sSW = self.cell(S, I - 1, J), self.cell(S, I - 1, J - 1)
                Gx = (sNE + sSE - sNW - sSW) / (2 * dx)
                Gy = (sNW + sNE - sSW - sSE) / (2 * dy)
                rp = mp_[J][I] / A
                uhx[J][I] = ZERO if I in (0, nx) else self.ux[J][I] - dt / 2 * Gx / rp
                uhy[J][I] = ZERO if J in (0, ny) else self.uy[J][I] - dt / 2 * Gy / rp
            uLx = [[ZERO if I in (0, nx) else 2 * uhx[J][I] - self.ux[J][I] for I in range(nx + 1)]
                   for J in range(ny + 1)]
            uLy = [[ZERO if J in (0, ny) else 2 * uhy[J][I] - self.uy[J][I] for I in range(nx + 1)]
                   for J in range(ny + 1)]
        self.dpx = [[dt * uhx[J][I] for I in range(nx + 1)] for J in range(ny + 1)]
        self.dpy = [[dt * uhy[J][I] for I in range(nx + 1)] for J in range(ny + 1)]
        if not self.kinematic:
            # corrector: e^{lag} with the material's own volume k F(x^{lag})
            for i, j in cells:
                VL = self.quad(i, j, self.dpx, self.dpy)
                for a in range(nm):
                    if pres[a][j][i]:
                        rL = M[a][j][i] / (k[a][j][i] * VL)
                        eL[a][j][i] = e[a][j][i] - (Ph[a][j][i] + Q[j][i]) * (1 / rL - 1 / rho[a][j][i])

        # ---- DirectCF regions (§2.3)
        regions = {}

        def add(key, vol, donor, recv, sgn, rect, kind, w=None):
            regions[key] = dict(vol=vol, donor=donor, recv=recv, sgn=sgn, rect=rect, kind=kind, w=w,
                                W=[ZERO] * nm, mu=[ZERO] * nm, eps=[ZERO] * nm)

        for j in range(ny):
            for I in range(1, nx):  # x-faces (walls carry nothing)
                xI = self.x0 + I * dx
                (dxm, dym), (dxp, dyp) = self.disp(I, j), self.disp(I, j + 1)
                ym, yp = self.y0 + j * dy, self.y0 + (j + 1) * dy
                xLm, yLm, xLp, yLp = xI + dxm, ym + dym, xI + dxp, yp + dyp
                ylo, yhi = ym + max(ZERO, dym), yp + min(ZERO, dyp)
                h = max(ZERO, yhi - ylo)
                X = lambda y: xLm + (y - yLm) * (xLp - xLm) / (yLp - yLm)
                w = ((X(ylo) - xI) + (X(yhi) - xI)) / 2
                fwd = w >= 0
                add(("x", I, j), abs(w * h), (I - 1, j) if fwd else (I, j), (I, j) if fwd else (I - 1, j),
                    1 if fwd else -1, (xI + min(ZERO, w), xI + max(ZERO, w), ylo, ylo + h), "x", w)
        for J in range(1, ny):
            for i in range(nx):  # y-faces
                yJ = self.y0 + J * dy
                (dxm, dym), (dxp, dyp) = self.disp(i, J), self.disp(i + 1, J)
                xm, xp = self.x0 + i * dx, self.x0 + (i + 1) * dx
                xLm, yLm, xLp, yLp = xm + dxm, yJ + dym, xp + dxp, yJ + dyp
                xlo, xhi = xm + max(ZERO, dxm), xp + min(ZERO, dxp)
                h = max(ZERO, xhi - xlo)
                Yf = lambda x: yLm + (x - xLm) * (yLp - yLm) / (xLp - xLm)
                w = ((Yf(xlo) - yJ) + (Yf(xhi) - yJ)) / 2
                fwd = w >= 0
                add(("y", i, J), abs(w * h), (i, J - 1) if fwd else (i, J), (i, J) if fwd else (i, J - 1),
                    1 if fwd else -1, (xlo, xlo + h, yJ + min(ZERO, w), yJ + max(ZERO, w)), "y", w)
        for J in range(1, ny):
            for I in range(1, nx):  # corners at interior nodes
                ddx, ddy = self.disp(I, J)
                xp, yp = self.x0 + I * dx, self.y0 + J * dy
                rect = (xp + min(ZERO, ddx), xp + max(ZERO, ddx), yp + min(ZERO, ddy), yp + max(ZERO, ddy))
                vol = abs(ddx * ddy)
                if ddx >= 0 and ddy >= 0:
                    add(("c", I, J), vol, (I - 1, J - 1), (I, J), 1, rect, "main")
                elif ddx < 0 and ddy < 0:
                    add(("c", I, J), vol, (I, J), (I - 1, J - 1), -1, rect, "main")
                elif ddx >= 0:
                    add(("c", I, J), vol, (I - 1, J), (I, J - 1), 1, rect, "anti")
                else:
                    add(("c", I, J), vol, (I, J - 1), (I - 1, J), -1, rect, "anti")

        def cell_regions(i, j):
            keys = [("x", i, j), ("x", i + 1, j), ("y", i, j), ("y", i, j + 1),
                    ("c", i, j), ("c", i + 1, j), ("c", i, j + 1), ("c", i + 1, j + 1)]
            return [regions[kk] for kk in keys if kk in regions]

        # flux-consistent Lagrangian volume, centres, widths, rho^{lag}, purity
        volcf = [[ZERO] * nx for _ in range(ny)]
        xc = [[ZERO] * nx for _ in range(ny)]
        yc = [[ZERO] * nx for _ in range(ny)]
        wxL = [[ZERO] * nx for _ in range(ny)]
        wyL = [[ZERO] * nx for _ in range(ny)]
        pure = [[-1] * nx for _ in range(ny)]
        rhocf = [[[ZERO] * nx for _ in range(ny)] for a in range(nm)]
        for i, j in cells:
            v = A
            for r in cell_regions(i, j):
                if r["donor"] == (i, j):
                    v += r["vol"]
                elif r["recv"] == (i, j):
                    v -= r["vol"]
            volcf[j][i] = v
            ps = [self.node_pos(I, J) for I, J in ((i, j), (i + 1, j), (i, j + 1), (i + 1, j + 1))]
            xc[j][i] = sum(p[0] for p in ps) / 4
            yc[j][i] = sum(p[1] for p in ps) / 4
            d = [self.disp(I, J) for I, J in ((i, j), (i + 1, j), (i, j + 1), (i + 1, j + 1))]
            wxL[j][i] = dx + ((d[1][0] + d[3][0]) - (d[0][0] + d[2][0])) / 2
            wyL[j][i] = dy + ((d[2][1] + d[3][1]) - (d[0][1] + d[1][1])) / 2
            present = [a for a in range(nm) if pres[a][j][i]]
            if len(present) == 1:
                pure[j][i] = present[0]
            for a in present:
                rhocf[a][j][i] = M[a][j][i] / (k[a][j][i] * v)

        def centre(i, j):
            """Lagrangian centre of any cell: beyond a wall, the reflection"""
            ri, rj = mref_cell(i, nx), mref_cell(j, ny)
            x, y = xc[rj][ri], yc[rj][ri]
            if ri != i:
                x = TWO * (self.x0 if i < 0 else self.x1) - x
            if rj != j:
                y = TWO * (self.y0 if j < 0 else self.y1) - y
            return x, y

        # ---- partial volumes (§4.4) and clipping, per donor
        gmin = mp.mpf("1e-10") / min(dx, dy)
        for i, j in cells:
            outs = [r for r in cell_regions(i, j) if r["donor"] == (i, j)]
            if not outs:
                continue
            present = [a for a in range(nm) if pres[a][j][i]]
            if pure[j][i] >= 0:
                for r in outs:
                    r["W"][pure[j][i]] = r["vol"]
                continue
            cx, cy = self.x0 + (i + HALF) * dx, self.y0 + (j + HALF) * dy
            pbl, pbr = self.node_pos(i, j), self.node_pos(i + 1, j)
            ptl, ptr = self.node_pos(i, j + 1), self.node_pos(i + 1, j + 1)
            Rr = ((pbl[0] + ptl[0]) / 2 - cx, (pbr[0] + ptr[0]) / 2 - cx,
                  (pbl[1] + pbr[1]) / 2 - cy, (ptl[1] + ptr[1]) / 2 - cy)
            Vp = sum(V[a][j][i] for a in present)

            def youngs(a):
                kk = lambda ii, jj: self.cell(k[a], ii, jj)
                gx = ((kk(i + 1, j - 1) + 2 * kk(i + 1, j) + kk(i + 1, j + 1)) -
                      (kk(i - 1, j - 1) + 2 * kk(i - 1, j) + kk(i - 1, j + 1))) / (8 * dx)
                gy = ((kk(i - 1, j + 1) + 2 * kk(i, j + 1) + kk(i + 1, j + 1)) -
                      (kk(i - 1, j - 1) + 2 * kk(i, j - 1) + kk(i + 1, j - 1))) / (8 * dy)
                return gx, gy

            lines, degenerate = {}, False
            if len(present) == 2:
                a0, b0 = present
                ga, gb = youngs(a0), youngs(b0)
                n = (ga[0] - gb[0], ga[1] - gb[1])
                nr = mp.sqrt(n[0] ** 2 + n[1] ** 2)
                if nr <= gmin:
                    degenerate = True
                else:
                    n = (n[0] / nr, n[1] / nr)
                    lines[a0] = (n, interface_offset(Rr, n, V[a0][j][i] / Vp))
            else:
                for a in present:
                    n = youngs(a)
                    nr = mp.sqrt(n[0] ** 2 + n[1] ** 2)
                    if nr <= gmin:
                        degenerate = True
                        continue
                    n = (n[0] / nr, n[1] / nr)
                    lines[a] = (n, interface_offset(Rr, n, V[a][j][i] / Vp))
            for r in outs:
                if r["vol"] == 0:
                    continue
                x0, x1, y0, y1 = r["rect"]
                rect = (x0 - cx, x1 - cx, y0 - cy, y1 - cy)
                if degenerate:
                    for a in present:
                        r["W"][a] = r["vol"] * (V[a][j][i] / Vp)
                elif len(present) == 2:
                    a0, b0 = present
                    (n, s) = lines[a0]
                    wa = min(max(halfplane_area(*rect, n[0], n[1], s), ZERO), r["vol"])
                    r["W"][a0], r["W"][b0] = wa, r["vol"] - wa
                else:
                    raw = {a: halfplane_area(*rect, lines[a][0][0], lines[a][0][1], lines[a][1]) for a in present}
                    tot = sum(raw.values())
                    for a in present:
                        r["W"][a] = r["vol"] * (raw[a] / tot) if tot > 0 else r["vol"] * (V[a][j][i] / Vp)
            # donor-side clipping against k_a Vol^CF
            Vcf = [k[a][j][i] * volcf[j][i] for a in range(nm)]
            O = [sum(r["W"][a] for r in outs) for a in range(nm)]
            over = [pres[a][j][i] and O[a] > Vcf[a] for a in range(nm)]
            if any(over):
                room = [max(ZERO, Vcf[a] - O[a]) if pres[a][j][i] and not over[a] else ZERO for a in range(nm)]
                H = sum(room)
                if H > 0:
                    for r in outs:
                        freed = ZERO
                        for a in range(nm):
                            if over[a]:
                                keep = r["W"][a] * (Vcf[a] / O[a])
                                freed += r["W"][a] - keep
                                r["W"][a] = keep
                        for a in range(nm):
                            if room[a] > 0:
                                r["W"][a] += freed * (room[a] / H)

        # ---- reconstruction (§2.1.1, §3.3) and fluxes, per donor
        sq = mp.sqrt(dx * dx + dy * dy)

        def stencil_pure(i, j, si, sj):
            m = pure[j][i]
            return m >= 0 and self.cell(pure, i - si, j - sj) == m and self.cell(pure, i + si, j + sj) == m

        def value(r, arr, order):
            i, j = r["donor"]
            aD = arr[j][i]
            if order == 1:
                return aD
            if r["kind"] in ("x", "y"):
                si, sj = (1, 0) if r["kind"] == "x" else (0, 1)
                if not stencil_pure(i, j, si, sj):
                    return aD
                c0, cm, cp = centre(i, j), centre(i - si, j - sj), centre(i + si, j + sj)
                ax = 0 if si else 1
                dm = (aD - self.cell(arr, i - si, j - sj)) / (c0[ax] - cm[ax])
                dpv = (self.cell(arr, i + si, j + sj) - aD) / (cp[ax] - c0[ax])
                d = van_leer(dm, dpv)
                if r["kind"] == "x":
                    I, jj = r["key"][1], r["key"][2]
                    df = (self.disp(I, jj)[0] + self.disp(I, jj + 1)[0]) / 2
                    return aD + d * (r["sgn"] * wxL[j][i] - df) / 2
                ii, J = r["key"][1], r["key"][2]
                df = (self.disp(ii, J)[1] + self.disp(ii + 1, J)[1]) / 2
                return aD + d * (r["sgn"] * wyL[j][i] - df) / 2
            main = r["kind"] == "main"
            si, sj = (1, 1) if main else (1, -1)
            if not stencil_pure(i, j, si, sj):
                return aD
            vx, vy = dx / sq, (dy if main else -dy) / sq
            c0, cm, cp = centre(i, j), centre(i - si, j - sj), centre(i + si, j + sj)
            dm = (aD - self.cell(arr, i - si, j - sj)) / ((c0[0] - cm[0]) * vx + (c0[1] - cm[1]) * vy)
            dpv = (self.cell(arr, i + si, j + sj) - aD) / ((cp[0] - c0[0]) * vx + (cp[1] - c0[1]) * vy)
            d = van_leer(dm, dpv)
            I, J = r["key"][1], r["key"][2]
            ddx, ddy = self.disp(I, J)
            sx = ONE if ddx >= 0 else -ONE
            off = (sx * wxL[j][i] - ddx) * vx + ((sx if main else -sx) * wyL[j][i] - ddy) * vy
            return aD + d * off / 2

        for key, r in regions.items():
            r["key"] = key
        for i, j in cells:
            outs = [r for r in cell_regions(i, j) if r["donor"] == (i, j)]
            if not outs:
                continue
            order = self.order if pure[j][i] >= 0 else 1
            while True:
                Mout, Eout = [ZERO] * nm, [ZERO] * nm
                for r in outs:
                    for a in range(nm):
                        r["mu"][a] = r["eps"][a] = ZERO
                        if not r["W"][a] > 0:
                            continue
                        rv = value(r, rhocf[a], order)
                        ev = value(r, eL[a], order)
                        r["mu"][a] = rv * r["W"][a]
                        r["eps"][a] = r["mu"][a] * ev
                        Mout[a] += r["mu"][a]
                        Eout[a] += r["eps"][a]
                if order == 1:
                    break
                a = pure[j][i]
                if not (Mout[a] > M[a][j][i] or Eout[a] > M[a][j][i] * eL[a][j][i]):
                    break
                order = 1  # positivity guard

        # ---- primal update
        Vn = [[[ZERO] * nx for _ in range(ny)] for a in range(nm)]
        Mn = [[[ZERO] * nx for _ in range(ny)] for a in range(nm)]
        En = [[[ZERO] * nx for _ in range(ny)] for a in range(nm)]
        for i, j in cells:
            rs = cell_regions(i, j)
            for a in range(nm):
                v, m, en = k[a][j][i] * volcf[j][i], M[a][j][i], M[a][j][i] * eL[a][j][i]
                for r in rs:
                    if r["recv"] == (i, j):
                        v, m, en = v + r["W"][a], m + r["mu"][a], en + r["eps"][a]
                    elif r["donor"] == (i, j):
                        v, m, en = v - r["W"][a], m - r["mu"][a], en - r["eps"][a]
                Vn[a][j][i], Mn[a][j][i], En[a][j][i] = v, m, en

        # ---- dual (momentum) update
        if not self.kinematic:
            def flux(key):
                r = regions.get(key)
                return r["sgn"] * sum(r["mu"]) if r is not None else ZERO

            def muX(I, j):  # x-face mass flux along +x, any index (mirrored)
                rI, rj = mref_node(I, nx), mref_cell(j, ny)
                v = flux(("x", rI, rj))
                return -v if rI != I else v

            def muY(i, J):
                ri, rJ = mref_cell(i, nx), mref_node(J, ny)
                v = flux(("y", ri, rJ))
                return -v if rJ != J else v

            def corner(I, J):  # (main, anti) mass flux of the corner at any node
                rI, rJ = mref_node(I, nx), mref_node(J, ny)
                r = regions.get(("c", rI, rJ))
                f = r["sgn"] * sum(r["mu"]) if r is not None else ZERO
                dmain, danti = (f, ZERO) if (r is not None and r["kind"] == "main") else (ZERO, f)
                if rI != I:  # x-mirror: (main, anti) -> (-anti, -main)
                    dmain, danti = -danti, -dmain
                if rJ != J:  # y-mirror: (main, anti) -> (anti, main)
                    dmain, danti = danti, dmain
                return dmain, danti

            def uL(I, J):
                return self.node_vec(uLx, uLy, I, J)

            def dual_w(I, J, axis):
                if axis == 0:
                    return dx + (self.disp(I + 1, J)[0] - self.disp(I - 1, J)[0]) / 2
                return dy + (self.disp(I, J + 1)[1] - self.disp(I, J - 1)[1]) / 2

            def dual_value(D, comp, si, sj, off):
                """u^{lag} component of donor node D, order 2: limited slope
                along (si, sj) between Lagrangian node positions, times off"""
                I, J = D
                u0 = uL(I, J)[comp]
                if self.order == 1:
                    return u0
                um, up = uL(I - si, J - sj)[comp], uL(I + si, J + sj)[comp]
                p0, pm, pp = self.node_pos(I, J), self.node_pos(I - si, J - sj), self.node_pos(I + si, J + sj)
                nrm = mp.sqrt(si * si * dx * dx + sj * sj * dy * dy)
                vx, vy = si * dx / nrm, sj * dy / nrm
                dm = (u0 - um) / ((p0[0] - pm[0]) * vx + (p0[1] - pm[1]) * vy)
                dpv = (up - u0) / ((pp[0] - p0[0]) * vx + (pp[1] - p0[1]) * vy)
                return u0 + van_leer(dm, dpv) * off / 2

            def face_x(Ip, J):  # dual x-face between nodes (Ip-1, J) and (Ip, J)
                phi = QUARTER * (muX(Ip - 1, J - 1) + muX(Ip, J - 1) + muX(Ip - 1, J) + muX(Ip, J))
                D, sg = ((Ip - 1, J), ONE) if phi > 0 else ((Ip, J), -ONE)
                df = (self.disp(Ip - 1, J)[0] + self.disp(Ip, J)[0]) / 2
                off = sg * dual_w(*D, 0) - df
                return phi, [dual_value(D, c, 1, 0, off) for c in (0, 1)]

            def face_y(I, Jp):
                phi = QUARTER * (muY(I - 1, Jp - 1) + muY(I, Jp - 1) + muY(I - 1, Jp) + muY(I, Jp))
                D, sg = ((I, Jp - 1), ONE) if phi > 0 else ((I, Jp), -ONE)
                df = (self.disp(I, Jp - 1)[1] + self.disp(I, Jp)[1]) / 2
                off = sg * dual_w(*D, 1) - df
                return phi, [dual_value(D, c, 0, 1, off) for c in (0, 1)]

            def dual_corner(i, j, main):
                """dual corner at cell (i, j): main from node (i, j) to (i+1, j+1),
                anti from (i, j+1) to (i+1, j)"""
                ns = ((i, j), (i + 1, j), (i, j + 1), (i + 1, j + 1))
                phi = QUARTER * sum(corner(I, J)[0 if main else 1] for I, J in ns)
                dc = [sum(self.disp(I, J)[ax] for I, J in ns) / 4 for ax in (0, 1)]
                if main:
                    D, sg = ((i, j), ONE) if phi > 0 else ((i + 1, j + 1), -ONE)
                    si, sj = 1, 1
                else:
                    D, sg = ((i, j + 1), ONE) if phi > 0 else ((i + 1, j), -ONE)
                    si, sj = 1, -1
                vx, vy = dx / sq, (dy if main else -dy) / sq
                off = (sg * dual_w(*D, 0) - dc[0]) * vx + ((sg if main else -sg) * dual_w(*D, 1) - dc[1]) * vy
                return phi, [dual_value(D, c, si, sj, off) for c in (0, 1)]

            ux_new = [[ZERO] * (nx + 1) for _ in range(ny + 1)]
            uy_new = [[ZERO] * (nx + 1) for _ in range(ny + 1)]
            for I, J in nodes:
                m = mp_[J][I]
                mu = [m * uLx[J][I], m * uLy[J][I]]
                for sign, (phi, u) in ((1, face_x(I, J)), (-1, face_x(I + 1, J)), (1, face_y(I, J)),
                                       (-1, face_y(I, J + 1)), (1, dual_corner(I - 1, J - 1, True)),
                                       (-1, dual_corner(I, J, True)), (1, dual_corner(I - 1, J, False)),
                                       (-1, dual_corner(I, J - 1, False))):
                    m += sign * phi
                    mu[0] += sign * phi * u[0]
                    mu[1] += sign * phi * u[1]
                ux_new[J][I] = ZERO if I in (0, nx) else mu[0] / m
                uy_new[J][I] = ZERO if J in (0, ny) else mu[1] / m
            self.ux, self.uy = ux_new, uy_new
        self.V, self.M, self.E = Vn, Mn, En
        self.t += dt
        return dt
