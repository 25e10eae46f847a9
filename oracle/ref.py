"""ctypes wrapper of the oracle library ``liblr_ref.so`` (test infrastructure)."""
import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIBS = {}
REMAP_DIRECTCF, REMAP_AD = 0, 1
COUNT_NAMES = ("mixed", "three_or_more", "degenerate_normal", "clipped", "guard")

F_RHO, F_P, F_E, F_K, F_RHOA, F_EA, F_PA, F_UX, F_UY, F_VOL, F_MASS, F_IE = (
    1 << i for i in range(12))
PER_MAT = {F_K, F_RHOA, F_EA, F_PA, F_VOL, F_MASS, F_IE}
NODE = {F_UX, F_UY}
FIELD_BITS = {"rho": F_RHO, "p": F_P, "e": F_E, "k": F_K, "rho_a": F_RHOA, "e_a": F_EA,
              "p_a": F_PA, "ux": F_UX, "uy": F_UY, "vol": F_VOL, "mass": F_MASS, "ie": F_IE}


class Eos(C.Structure):
    _fields_ = [("gamma", C.c_double), ("pinf", C.c_double)]


class Opts(C.Structure):
    _fields_ = [("x0", C.c_double), ("x1", C.c_double), ("y0", C.c_double),
                ("y1", C.c_double), ("cfl", C.c_double), ("a1", C.c_double),
                ("a2", C.c_double), ("precision", C.c_int), ("recon_order", C.c_int),
                ("kinematic", C.c_int), ("k_eps", C.c_double), ("fixed_dt", C.c_double),
                ("remap", C.c_int)]


def load(omp=False):
    """Load (building first if absent) the oracle library: the single-threaded
    build, or with omp=True the OpenMP build (same bits)."""
    if omp in _LIBS:
        return _LIBS[omp]
    # LR_REF_SO lets the mutation test point the suite at a deliberately
    # broken copy of the oracle
    so = os.environ.get("LR_REF_SO") or os.path.join(
        _HERE, "liblr_ref_omp.so" if omp else "liblr_ref.so")
    if not os.path.exists(so):
        from .build import build
        build()
    lib = C.CDLL(so)
    P = C.POINTER
    dp = P(C.c_double)
    lib.lr_ref_default_opts.argtypes = [P(Opts)]
    lib.lr_ref_create.argtypes = [C.c_int, C.c_int, C.c_int, P(Eos), P(C.c_int), P(Opts),
                                  P(C.c_void_p)]
    lib.lr_ref_set_state.argtypes = [C.c_void_p, C.c_double, dp, dp, dp, dp, dp]
    lib.lr_ref_step.argtypes = [C.c_void_p, dp]
    lib.lr_ref_run.argtypes = [C.c_void_p, C.c_double, C.c_long, P(C.c_long), dp]
    lib.lr_ref_get_fields.argtypes = [C.c_void_p, C.c_uint, P(dp)]
    lib.lr_ref_totals.argtypes = [C.c_void_p, dp]
    lib.lr_ref_debug_get.argtypes = [C.c_void_p, C.c_char_p, dp]
    lib.lr_ref_last_error.argtypes = [C.c_void_p]
    lib.lr_ref_last_error.restype = C.c_char_p
    lib.lr_ref_destroy.argtypes = [C.c_void_p]
    lib.lr_ref_destroy.restype = None
    lib.lr_ref_rect_halfplane_area.argtypes = [C.c_double] * 7
    lib.lr_ref_rect_halfplane_area.restype = C.c_double
    lib.lr_ref_interface_offset.argtypes = [C.c_double] * 7
    lib.lr_ref_interface_offset.restype = C.c_double
    for name in ("lr_ref_create", "lr_ref_set_state", "lr_ref_step", "lr_ref_run",
                 "lr_ref_get_fields", "lr_ref_totals", "lr_ref_debug_get"):
        getattr(lib, name).restype = C.c_int
    _LIBS[omp] = lib
    return lib


def rect_halfplane_area(x0, x1, y0, y1, nx, ny, s):
    return load().lr_ref_rect_halfplane_area(x0, x1, y0, y1, nx, ny, s)


def interface_offset(x0, x1, y0, y1, nx, ny, frac):
    return load().lr_ref_interface_offset(x0, x1, y0, y1, nx, ny, frac)


def _dptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


class OracleError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"oracle error {code}: {msg}")
        self.code = code


class RefSolver:
    """One problem on the oracle; mirrors the GPU binding's ``Solver``."""

    def __init__(self, nx, ny, gammas, domain=(0.0, 1.0, 0.0, 1.0), cfl=0.5, a1=0.5,
                 a2=1.0, recon_order=2, kinematic=False, k_eps=1e-10, fixed_dt=0.0,
                 pinfs=None, remap=REMAP_DIRECTCF, omp=False):
        self.lib = load(omp)
        self.nx, self.ny, self.nmat = int(nx), int(ny), len(gammas)
        pinfs = [0.0] * self.nmat if pinfs is None else list(pinfs)
        eos = (Eos * self.nmat)(*[Eos(float(g), float(pi)) for g, pi in zip(gammas, pinfs)])
        o = Opts()
        self.lib.lr_ref_default_opts(C.byref(o))
        o.x0, o.x1, o.y0, o.y1 = map(float, domain)
        o.cfl, o.a1, o.a2 = float(cfl), float(a1), float(a2)
        o.recon_order, o.kinematic = int(recon_order), int(bool(kinematic))
        o.k_eps, o.fixed_dt = float(k_eps), float(fixed_dt)
        o.remap = int(remap)
        bc = (C.c_int * 4)(0, 0, 0, 0)
        h = C.c_void_p()
        rc = self.lib.lr_ref_create(self.nx, self.ny, self.nmat, eos, bc, C.byref(o), C.byref(h))
        if rc != 0:
            raise OracleError(rc, "create failed")
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.lib.lr_ref_destroy(self.h)
            self.h = None

    __del__ = close

    def _check(self, rc):
        if rc != 0:
            raise OracleError(rc, self.lib.lr_ref_last_error(self.h).decode())
        return rc

    def set_state(self, t, k, rho, e, ux, uy):
        arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (k, rho, e, ux, uy)]
        self._check(self.lib.lr_ref_set_state(self.h, float(t), *[_dptr(a) for a in arrs]))

    def step(self):
        dt = C.c_double()
        self._check(self.lib.lr_ref_step(self.h, C.byref(dt)))
        return dt.value

    def run(self, t_end, max_steps=1 << 40):
        n, t = C.c_long(), C.c_double()
        rc = self.lib.lr_ref_run(self.h, float(t_end), int(max_steps), C.byref(n), C.byref(t))
        self._check(rc)
        return n.value, t.value

    def run_raw(self, t_end, max_steps=1 << 40):
        n, t = C.c_long(), C.c_double()
        rc = self.lib.lr_ref_run(self.h, float(t_end), int(max_steps), C.byref(n), C.byref(t))
        return rc, n.value, t.value

    def fields(self, *names):
        mask, outs = 0, []
        for nm_ in names:
            mask |= FIELD_BITS[nm_]
        bufs = {}
        for bit in sorted(FIELD_BITS.values()):
            if not mask & bit:
                continue
            if bit in PER_MAT:
                shape = (self.nmat, self.ny, self.nx)
            elif bit in NODE:
                shape = (self.ny + 1, self.nx + 1)
            else:
                shape = (self.ny, self.nx)
            bufs[bit] = np.zeros(shape)
            outs.append(bufs[bit])
        ptrs = (C.POINTER(C.c_double) * len(outs))(*[_dptr(b) for b in outs])
        self._check(self.lib.lr_ref_get_fields(self.h, mask, ptrs))
        return {n_: bufs[FIELD_BITS[n_]] for n_ in names}

    def totals(self):
        out = np.zeros(3 * self.nmat + 3)
        self._check(self.lib.lr_ref_totals(self.h, _dptr(out)))
        return out

    def counts(self):
        """Cells (summed over the steps since set_state) that took each branch:
        mixed, three or more materials, degenerate normal, clipped, guard."""
        out = np.zeros(len(COUNT_NAMES))
        self._check(self.lib.lr_ref_debug_get(self.h, b"counts", _dptr(out)))
        return dict(zip(COUNT_NAMES, out.astype(np.int64).tolist()))

    def stage(self, name):
        nx, ny, nm = self.nx, self.ny, self.nmat
        shapes = {"Q": (ny, nx), "Pc": (ny, nx), "cc": (ny, nx), "S": (ny, nx), "VL": (ny, nx),
                  "volcf": (ny, nx), "xcL": (ny, nx), "ycL": (ny, nx), "dxL": (ny, nx),
                  "dyL": (ny, nx), "eL": (nm, ny, nx), "rhocf": (nm, ny, nx),
                  "P_half": (nm, ny, nx), "e_half": (nm, ny, nx),
                  "muX": (ny, nx + 1), "Wx": (ny, nx + 1), "Wpx": (nm, ny, nx + 1),
                  "muY": (ny + 1, nx), "Wy": (ny + 1, nx), "Wpy": (nm, ny + 1, nx),
                  "Wpc": (nm, ny + 1, nx + 1), "dt": (1,), "t": (1,)}
        shape = shapes.get(name, (ny + 1, nx + 1))
        out = np.zeros(shape)
        self._check(self.lib.lr_ref_debug_get(self.h, name.encode(), _dptr(out)))
        return out
