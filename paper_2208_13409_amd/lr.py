"""ctypes binding of ``liblr.so`` (the C-ABI in ``include/lr.h``).

Argument marshalling only: every step of the scheme runs in the library's HIP
kernels.  The functions keep the C names (``lr_create``, ``lr_set_state``,
``lr_step``, ``lr_run``, ``lr_get_fields``, ``lr_totals``, ``lr_debug_get``,
``lr_bind_stream``, ``lr_destroy``); ``Solver`` wraps one context.  There is
no fallback: if the library is missing or the device is absent, the calls
raise.
"""
import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SO_PATH = os.path.join(_HERE, "liblr.so")
_LIB = None

LR_OK, LR_EINVAL, LR_ENOMEM, LR_EDEVICE, LR_ENEGATIVE, LR_ENAN, LR_EDT, LR_EAGAIN, LR_ESTATE = (
    0, -1, -2, -3, -4, -5, -6, -7, -8)
LR_FP64, LR_FP32 = 0, 1
LR_REMAP_DIRECTCF, LR_REMAP_AD = 0, 1
LR_TILE_AUTO, LR_TILE_32x8, LR_TILE_16x16, LR_TILE_32x16, LR_TILE_32x12 = -1, 0, 1, 2, 3
LR_NTILE = 4
LR_NTUNE_TILE = 3
LR_NSCHED = 4 * LR_NTUNE_TILE
TILE_SHAPES = ((32, 8), (16, 16), (32, 16), (32, 12))
F_RHO, F_P, F_E, F_K, F_RHOA, F_EA, F_PA, F_UX, F_UY, F_VOL, F_MASS, F_IE = (1 << i for i in range(12))
PER_MAT = {F_K, F_RHOA, F_EA, F_PA, F_VOL, F_MASS, F_IE}
NODE = {F_UX, F_UY}
FIELD_BITS = {"rho": F_RHO, "p": F_P, "e": F_E, "k": F_K, "rho_a": F_RHOA, "e_a": F_EA,
              "p_a": F_PA, "ux": F_UX, "uy": F_UY, "vol": F_VOL, "mass": F_MASS, "ie": F_IE}
EXPORTS = ("lr_default_opts", "lr_create", "lr_bind_stream", "lr_set_state", "lr_set_state_device",
           "lr_step", "lr_run", "lr_get_fields", "lr_totals", "lr_debug_get", "lr_last_error",
           "lr_destroy", "lr_profile", "lr_profile_read", "lr_kernel_count", "lr_kernel_name",
           "lr_batch_default_opts", "lr_batch_create", "lr_batch_bind_stream", "lr_batch_footprint",
           "lr_batch_submit", "lr_batch_step", "lr_batch_step_begin", "lr_batch_step_end",
           "lr_batch_poll", "lr_batch_status",
           "lr_batch_get_fields", "lr_batch_totals", "lr_batch_release", "lr_batch_running",
           "lr_batch_schedule", "lr_batch_last_error", "lr_batch_destroy", "lr_run_noalloc")
LR_F64_IN, LR_F32_IN = 0, 1  # element types of lr_set_state_device


class lr_eos(C.Structure):
    _fields_ = [("gamma", C.c_double), ("pinf", C.c_double)]


class lr_opts(C.Structure):
    _fields_ = [("x0", C.c_double), ("x1", C.c_double), ("y0", C.c_double),
                ("y1", C.c_double), ("cfl", C.c_double), ("a1", C.c_double),
                ("a2", C.c_double), ("precision", C.c_int), ("recon_order", C.c_int),
                ("kinematic", C.c_int), ("k_eps", C.c_double), ("fixed_dt", C.c_double),
                ("stages", C.c_int), ("remap", C.c_int), ("mix_list", C.c_int), ("tile", C.c_int)]


class lr_batch_opts(C.Structure):
    _fields_ = [("max_slots", C.c_int), ("pool_bytes", C.c_size_t), ("nmat", C.c_int),
                ("precision", C.c_int), ("chunk_steps", C.c_int), ("use_graph", C.c_int),
                ("persistent", C.c_int), ("autotune", C.c_int), ("tile", C.c_int)]


class LRError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"liblr error {code}: {msg}")
        self.code = code


def load():
    """Load liblr.so (built by ``paper_2208_13409_amd.build``); raise if absent."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(SO_PATH):
        raise FileNotFoundError(f"{SO_PATH} is missing: run paper_2208_13409_amd/build.py "
                                "(the HIP library is required; there is no fallback)")
    # PyTorch ships its own HIP runtime under the same soname: loading it
    # first makes the library bind to that one, so that one runtime owns the
    # device and torch's streams and device pointers are valid here too
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = C.CDLL(SO_PATH)
    P = C.POINTER
    dp = P(C.c_double)
    lib.lr_default_opts.argtypes = [P(lr_opts)]
    lib.lr_default_opts.restype = None
    lib.lr_create.argtypes = [C.c_int, C.c_int, C.c_int, P(lr_eos), P(C.c_int), P(lr_opts),
                              P(C.c_void_p)]
    lib.lr_bind_stream.argtypes = [C.c_void_p, C.c_void_p]
    lib.lr_set_state.argtypes = [C.c_void_p, C.c_double, dp, dp, dp, dp, dp]
    lib.lr_step.argtypes = [C.c_void_p, dp]
    lib.lr_run.argtypes = [C.c_void_p, C.c_double, C.c_long, P(C.c_long), dp]
    lib.lr_get_fields.argtypes = [C.c_void_p, C.c_uint, P(dp)]
    lib.lr_totals.argtypes = [C.c_void_p, dp]
    lib.lr_debug_get.argtypes = [C.c_void_p, C.c_char_p, dp]
    lib.lr_last_error.argtypes = [C.c_void_p]
    lib.lr_last_error.restype = C.c_char_p
    lib.lr_destroy.argtypes = [C.c_void_p]
    lib.lr_destroy.restype = None
    lib.lr_profile.argtypes = [C.c_void_p, C.c_int]
    lib.lr_profile_read.argtypes = [C.c_void_p, dp, P(C.c_long), C.c_int]
    lib.lr_kernel_count.argtypes = []
    lib.lr_kernel_name.argtypes = [C.c_int]
    lib.lr_kernel_name.restype = C.c_char_p
    vp = C.c_void_p
    lib.lr_set_state_device.argtypes = [vp, C.c_double, vp, vp, vp, vp, vp, C.c_int]
    lib.lr_batch_default_opts.argtypes = [P(lr_batch_opts)]
    lib.lr_batch_default_opts.restype = None
    lib.lr_batch_create.argtypes = [P(lr_batch_opts), P(vp)]
    lib.lr_batch_bind_stream.argtypes = [vp, vp]
    lib.lr_batch_footprint.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int]
    lib.lr_batch_footprint.restype = C.c_size_t
    lib.lr_batch_submit.argtypes = [vp, C.c_int, C.c_int, P(lr_eos), P(lr_opts), C.c_double, C.c_long,
                                    dp, dp, dp, dp, dp, P(C.c_long)]
    lib.lr_batch_step.argtypes = [vp, P(C.c_int)]
    lib.lr_batch_step_begin.argtypes = [vp]
    lib.lr_batch_step_end.argtypes = [vp, P(C.c_int)]
    lib.lr_batch_poll.argtypes = [vp, P(C.c_long), C.c_int, P(C.c_int)]
    lib.lr_batch_status.argtypes = [vp, C.c_long, P(C.c_int), P(C.c_long), dp]
    lib.lr_batch_get_fields.argtypes = [vp, C.c_long, C.c_uint, P(dp)]
    lib.lr_batch_totals.argtypes = [vp, C.c_long, dp]
    lib.lr_batch_release.argtypes = [vp, C.c_long]
    lib.lr_batch_running.argtypes = [vp]
    lib.lr_batch_schedule.argtypes = [vp, P(C.c_int), P(C.c_int), P(C.c_int), dp]
    lib.lr_batch_schedule.restype = C.c_int
    lib.lr_batch_last_error.argtypes = [vp]
    lib.lr_batch_last_error.restype = C.c_char_p
    lib.lr_batch_destroy.argtypes = [vp]
    lib.lr_batch_destroy.restype = None
    lib.lr_run_noalloc.argtypes = [C.c_int, C.c_int, C.c_int, P(lr_eos), P(C.c_int), P(lr_opts),
                                   C.c_double, C.c_double, C.c_long, vp, vp, vp, vp, vp, C.c_uint,
                                   P(vp), vp, P(C.c_long), dp, C.c_char_p, C.c_size_t]
    lib.lr_run_noalloc.restype = C.c_int
    for n in ("lr_create", "lr_bind_stream", "lr_set_state", "lr_set_state_device", "lr_step",
              "lr_run", "lr_get_fields", "lr_totals", "lr_debug_get", "lr_profile",
              "lr_profile_read", "lr_kernel_count", "lr_batch_create", "lr_batch_bind_stream",
              "lr_batch_submit", "lr_batch_step", "lr_batch_step_begin", "lr_batch_step_end",
              "lr_batch_poll", "lr_batch_status", "lr_batch_get_fields", "lr_batch_totals",
              "lr_batch_release", "lr_batch_running"):
        getattr(lib, n).restype = C.c_int
    _LIB = lib
    return lib


def _dptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def lr_default_opts():
    o = lr_opts()
    load().lr_default_opts(C.byref(o))
    return o


def _eos(gammas, pinfs=None):
    pinfs = [0.0] * len(gammas) if pinfs is None else pinfs
    if len(pinfs) != len(gammas):
        raise ValueError("one pinf per material expected")
    return (lr_eos * len(gammas))(*[lr_eos(float(g), float(pi)) for g, pi in zip(gammas, pinfs)])


def lr_create(nx, ny, gammas, opts, pinfs=None):
    eos = _eos(gammas, pinfs)
    bc = (C.c_int * 4)(0, 0, 0, 0)
    h = C.c_void_p()
    rc = load().lr_create(int(nx), int(ny), len(gammas), eos, bc, C.byref(opts), C.byref(h))
    if rc != LR_OK:
        raise LRError(rc, "lr_create failed")
    return h


class Solver:
    """One problem on the GPU library (same methods as the oracle's RefSolver)."""

    def __init__(self, nx, ny, gammas, domain=(0.0, 1.0, 0.0, 1.0), cfl=0.5, a1=0.5, a2=1.0,
                 recon_order=2, kinematic=False, k_eps=1e-10, fixed_dt=0.0, precision=LR_FP64,
                 stages=False, stream=None, pinfs=None, remap=0, mix_list=0, tile=LR_TILE_AUTO):
        self.lib = load()
        self.nx, self.ny, self.nmat = int(nx), int(ny), len(gammas)
        o = lr_default_opts()
        o.x0, o.x1, o.y0, o.y1 = map(float, domain)
        o.cfl, o.a1, o.a2 = float(cfl), float(a1), float(a2)
        o.recon_order, o.kinematic = int(recon_order), int(bool(kinematic))
        o.k_eps, o.fixed_dt, o.precision = float(k_eps), float(fixed_dt), int(precision)
        o.stages = int(bool(stages))
        o.remap = int(remap)
        o.mix_list = int(mix_list)
        o.tile = int(tile)
        self.h = lr_create(nx, ny, gammas, o, pinfs)
        if stream is not None:
            self.bind_stream(stream)

    def close(self):
        if getattr(self, "h", None):
            self.lib.lr_destroy(self.h)
            self.h = None

    __del__ = close

    def _check(self, rc):
        if rc != LR_OK:
            raise LRError(rc, self.lib.lr_last_error(self.h).decode())
        return rc

    def bind_stream(self, stream):
        """stream: a torch.cuda.Stream (its cuda_stream handle is used) or a raw handle."""
        handle = getattr(stream, "cuda_stream", stream)
        self._check(self.lib.lr_bind_stream(self.h, C.c_void_p(handle)))

    def set_state(self, t, k, rho, e, ux, uy):
        arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (k, rho, e, ux, uy)]
        self._check(self.lib.lr_set_state(self.h, float(t), *[_dptr(a) for a in arrs]))

    def set_state_device(self, t, k, rho, e, ux, uy):
        """State from device tensors (torch, float64 or float32, contiguous),
        copied on the context's stream."""
        ts = (k, rho, e, ux, uy)
        dt = {str(x.dtype) for x in ts}
        if len(dt) != 1 or not all(x.is_cuda and x.is_contiguous() for x in ts):
            raise ValueError("five contiguous device tensors of one dtype expected")
        code = LR_F32_IN if "float32" in dt.pop() else LR_F64_IN
        self._check(self.lib.lr_set_state_device(self.h, float(t), *[C.c_void_p(x.data_ptr()) for x in ts],
                                                 code))

    def step(self):
        dt = C.c_double()
        self._check(self.lib.lr_step(self.h, C.byref(dt)))
        return dt.value

    def run(self, t_end, max_steps=1 << 40):
        n, t = C.c_long(), C.c_double()
        self._check(self.lib.lr_run(self.h, float(t_end), int(max_steps), C.byref(n), C.byref(t)))
        return n.value, t.value

    def run_raw(self, t_end, max_steps=1 << 40):
        n, t = C.c_long(), C.c_double()
        rc = self.lib.lr_run(self.h, float(t_end), int(max_steps), C.byref(n), C.byref(t))
        return rc, n.value, t.value

    def fields(self, *names):
        return _fields(self.lib.lr_get_fields, self.h, self.nx, self.ny, self.nmat, self._check, names)

    def totals(self):
        out = np.zeros(3 * self.nmat + 3)
        self._check(self.lib.lr_totals(self.h, _dptr(out)))
        return out

    def profile(self, enable=True):
        self._check(self.lib.lr_profile(self.h, int(bool(enable))))

    def profile_read(self):
        """{kernel name: (total ms, launches)} since the last read."""
        n = self.lib.lr_kernel_count()
        ms = np.zeros(n)
        cnt = (C.c_long * n)()
        self._check(self.lib.lr_profile_read(self.h, _dptr(ms), cnt, n))
        return {self.lib.lr_kernel_name(i).decode(): (float(ms[i]), int(cnt[i])) for i in range(n)}

    def stage(self, name):
        nx, ny, nm = self.nx, self.ny, self.nmat
        shapes = {"Q": (ny, nx), "S": (ny, nx), "volcf": (ny, nx), "VL": (ny, nx),
                  "dxL": (ny, nx), "dyL": (ny, nx), "eL": (nm, ny, nx), "rhocf": (nm, ny, nx),
                  "P_half": (nm, ny, nx), "muX": (ny, nx + 1), "muY": (ny + 1, nx),
                  "Wpx": (nm, ny, nx + 1), "Wpy": (nm, ny + 1, nx), "Wpc": (nm, ny + 1, nx + 1),
                  "dt": (1,), "t": (1,), "run": (4,)}
        out = np.zeros(shapes.get(name, (ny + 1, nx + 1)))
        self._check(self.lib.lr_debug_get(self.h, name.encode(), _dptr(out)))
        return out


def _fields(fn, h, nx, ny, nmat, check, names, *lead):
    mask = 0
    for n_ in names:
        mask |= FIELD_BITS[n_]
    bufs, outs = {}, []
    for bit in sorted(FIELD_BITS.values()):
        if not mask & bit:
            continue
        if bit in PER_MAT:
            shape = (nmat, ny, nx)
        elif bit in NODE:
            shape = (ny + 1, nx + 1)
        else:
            shape = (ny, nx)
        bufs[bit] = np.zeros(shape)
        outs.append(bufs[bit])
    ptrs = (C.POINTER(C.c_double) * len(outs))(*[_dptr(b) for b in outs])
    check(fn(h, *lead, mask, ptrs))
    return {n_: bufs[FIELD_BITS[n_]] for n_ in names}


def run_noalloc(nx, ny, gammas, domain, t_end, k, rho, e, ux, uy, names, outs, t0=0.0,
                max_steps=1 << 40, cfl=0.5, a1=0.5, a2=1.0, recon_order=2, kinematic=False,
                k_eps=1e-10, fixed_dt=0.0, precision=LR_FP64, stream=None, pinfs=None):
    """lr_run_noalloc: inputs k, rho, e, ux, uy and outputs outs[name] are
    contiguous float64 device tensors (torch); names are field names in any
    order (written in the library's bit order).  Returns (steps, t)."""
    lib = load()
    o = lr_default_opts()
    o.x0, o.x1, o.y0, o.y1 = map(float, domain)
    o.cfl, o.a1, o.a2 = float(cfl), float(a1), float(a2)
    o.recon_order, o.kinematic = int(recon_order), int(bool(kinematic))
    o.k_eps, o.fixed_dt, o.precision = float(k_eps), float(fixed_dt), int(precision)
    eos = _eos(gammas, pinfs)
    ins = (k, rho, e, ux, uy)
    for x in ins + tuple(outs[n_] for n_ in names):
        if not (x.is_cuda and x.is_contiguous() and str(x.dtype) == "torch.float64"):
            raise ValueError("contiguous float64 device tensors expected")
    mask = 0
    for n_ in names:
        mask |= FIELD_BITS[n_]
    order = sorted(names, key=lambda n_: FIELD_BITS[n_])
    ptrs = (C.c_void_p * max(len(order), 1))(*[outs[n_].data_ptr() for n_ in order])
    handle = getattr(stream, "cuda_stream", stream) if stream is not None else None
    steps, t = C.c_long(), C.c_double()
    err = C.create_string_buffer(256)
    rc = lib.lr_run_noalloc(int(nx), int(ny), len(gammas), eos, (C.c_int * 4)(0, 0, 0, 0), C.byref(o),
                            float(t0), float(t_end), int(max_steps),
                            *[C.c_void_p(x.data_ptr()) for x in ins], mask, ptrs, C.c_void_p(handle),
                            C.byref(steps), C.byref(t), err, len(err))
    if rc != LR_OK:
        raise LRError(rc, err.value.decode())
    return steps.value, t.value


def lr_batch_default_opts():
    o = lr_batch_opts()
    load().lr_batch_default_opts(C.byref(o))
    return o


class Batch:
    """Many problems stepped together (continuous batching); see lr_batch_* in
    include/lr.h.  submit() returns a request id, or None when the batch has
    no room now (LR_EAGAIN)."""

    def __init__(self, nmat=2, precision=LR_FP32, max_slots=256, pool_bytes=4 << 30,
                 chunk_steps=16, use_graph=True, persistent=False, autotune=False, tile=LR_TILE_32x8,
                 stream=None):
        self.lib = load()
        o = lr_batch_default_opts()
        o.max_slots, o.pool_bytes, o.nmat, o.precision = int(max_slots), int(pool_bytes), int(nmat), int(precision)
        o.chunk_steps, o.use_graph, o.persistent = int(chunk_steps), int(bool(use_graph)), int(bool(persistent))
        o.autotune, o.tile = int(bool(autotune)), int(tile)
        self.nmat, self.precision = int(nmat), int(precision)
        h = C.c_void_p()
        rc = self.lib.lr_batch_create(C.byref(o), C.byref(h))
        if rc != LR_OK:
            raise LRError(rc, "lr_batch_create failed")
        self.h = h
        self.shapes = {}
        if stream is not None:
            handle = getattr(stream, "cuda_stream", stream)
            self._check(self.lib.lr_batch_bind_stream(self.h, C.c_void_p(handle)))

    def close(self):
        if getattr(self, "h", None):
            self.lib.lr_batch_destroy(self.h)
            self.h = None

    __del__ = close

    def _check(self, rc):
        if rc != LR_OK:
            raise LRError(rc, self.lib.lr_batch_last_error(self.h).decode())
        return rc

    def footprint(self, nx, ny):
        return int(self.lib.lr_batch_footprint(int(nx), int(ny), self.nmat, self.precision))

    def submit(self, prob, t_end, max_steps=1 << 40, cfl=0.5, a1=0.5, a2=1.0, recon_order=2,
               kinematic=False, k_eps=1e-10, fixed_dt=0.0, mix_list=0):
        """prob: dict with nx, ny, gammas, domain, k, rho, e, ux, uy."""
        o = lr_default_opts()
        o.x0, o.x1, o.y0, o.y1 = map(float, prob["domain"])
        o.cfl, o.a1, o.a2 = float(cfl), float(a1), float(a2)
        o.recon_order, o.kinematic = int(recon_order), int(bool(kinematic))
        o.k_eps, o.fixed_dt, o.precision = float(k_eps), float(fixed_dt), self.precision
        o.mix_list = int(mix_list)
        gam = prob["gammas"]
        if len(gam) != self.nmat:
            raise LRError(LR_EINVAL, f"{len(gam)} materials in a batch of nmat={self.nmat}")
        eos = _eos(gam, prob.get("pinfs"))
        arrs = [np.ascontiguousarray(prob[n], dtype=np.float64) for n in ("k", "rho", "e", "ux", "uy")]
        rid = C.c_long()
        rc = self.lib.lr_batch_submit(self.h, int(prob["nx"]), int(prob["ny"]), eos, C.byref(o),
                                      float(t_end), int(max_steps), *[_dptr(a) for a in arrs],
                                      C.byref(rid))
        if rc == LR_EAGAIN:
            return None
        self._check(rc)
        self.shapes[rid.value] = (int(prob["nx"]), int(prob["ny"]))
        return rid.value

    def step(self):
        """one chunk of steps; returns the number of problems still running"""
        n = C.c_int()
        self._check(self.lib.lr_batch_step(self.h, C.byref(n)))
        return n.value

    def step_begin(self):
        """launch one chunk and return at once (host work may overlap it)"""
        self._check(self.lib.lr_batch_step_begin(self.h))

    def step_end(self):
        """wait for the chunk in flight; returns the number still running"""
        n = C.c_int()
        self._check(self.lib.lr_batch_step_end(self.h, C.byref(n)))
        return n.value

    def poll(self, cap=4096):
        ids = (C.c_long * cap)()
        n = C.c_int()
        self._check(self.lib.lr_batch_poll(self.h, ids, cap, C.byref(n)))
        return [ids[i] for i in range(n.value)]

    def status(self, rid):
        rc, st, t = C.c_int(), C.c_long(), C.c_double()
        self._check(self.lib.lr_batch_status(self.h, int(rid), C.byref(rc), C.byref(st), C.byref(t)))
        return rc.value, st.value, t.value

    def fields(self, rid, *names):
        nx, ny = self.shapes[rid]
        return _fields(self.lib.lr_batch_get_fields, self.h, nx, ny, self.nmat, self._check, names,
                       C.c_long(int(rid)))

    def totals(self, rid):
        out = np.zeros(3 * self.nmat + 3)
        self._check(self.lib.lr_batch_totals(self.h, int(rid), _dptr(out)))
        return out

    def release(self, rid):
        self._check(self.lib.lr_batch_release(self.h, int(rid)))
        self.shapes.pop(rid, None)

    def running(self):
        return int(self.lib.lr_batch_running(self.h))

    def schedule(self):
        """(persistent, use_graph, tile, measured rates or None while tuning);
        rates[c] is schedule c = persistent + 2 use_graph + 4 tile"""
        pe, ug, ti = C.c_int(), C.c_int(), C.c_int()
        rates = np.zeros(LR_NSCHED)
        rc = self.lib.lr_batch_schedule(self.h, C.byref(pe), C.byref(ug), C.byref(ti), _dptr(rates))
        return bool(pe.value), bool(ug.value), int(ti.value), (rates if rc == LR_OK else None)
