"""Python binding of the HIP ODF engine (libodf.so, C ABI in include/odf.h).

Argument marshalling only: every computational step runs in the library's
gfx950 kernels.  PyTorch provides device memory (the workspace and output
tensors) and the HIP stream.  There is no CPU fallback: importing this module
raises if the library is missing, and every call raises on a library error.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libodf.so")

ODF_OK, ODF_E_INVALID, ODF_E_NOMEM, ODF_E_DEVICE, ODF_E_UNKNOWN_TICKET, ODF_E_CANCELLED, ODF_E_INTERNAL = \
    0, -1, -2, -3, -4, -5, -6
PREC = {"fp64": 0, "mixed": 1}
MEAN = {"geometric": 0, "arithmetic": 1}
OUTPUT = {"table": 0, "fine": 1}
ELECTRONS = {"fixed": 0, "equilibrium": 1}
STATE = {0: "PENDING", 1: "RUNNING", 2: "DONE", 3: "FAILED"}

_D = C.POINTER(C.c_double)
_I32 = C.POINTER(C.c_int32)
_I64 = C.POINTER(C.c_int64)


class OdfLines(C.Structure):
    _fields_ = [("n_lines", C.c_int64), ("lambda_nm", _D), ("log_gf", _D), ("e_low_ev", _D),
                ("species", _I32), ("stage", _I32), ("log_g_rad", _D), ("log_g_stark", _D),
                ("log_g_vdw", _D)]


class OdfSpecies(C.Structure):
    _fields_ = [("n_species", C.c_int32), ("n_stages", C.c_int32), ("mass_amu", _D), ("chi_ev", _D),
                ("part_fn", _D)]


class OdfLayout(C.Structure):
    _fields_ = [("lambda_first_nm", C.c_double), ("lambda_last_nm", C.c_double),
                ("resolving_power", C.c_double), ("n_bins", C.c_int32), ("bin_edges", _I64),
                ("n_steps", C.c_int32), ("step_frac", _D)]


class OdfOptions(C.Structure):
    _fields_ = [("precision", C.c_int), ("mean", C.c_int), ("cutoff", C.c_double),
                ("window_cap_doppler", C.c_double), ("pe_over_p", C.c_double),
                ("kappa_c_ref", C.c_double), ("lambda_c_ref_nm", C.c_double),
                ("kappa_c_power", C.c_double), ("workspace", C.c_void_p),
                ("workspace_bytes", C.c_int64), ("stream", C.c_void_p),
                ("max_batch_points", C.c_int32), ("loop_streams", C.c_int32),
                ("kernel_timing", C.c_int32), ("output", C.c_int32), ("electrons", C.c_int32)]


class OdfRequest(C.Structure):
    _fields_ = [("abundance", _D), ("n_points", C.c_int32), ("T_K", _D), ("log10_P_cgs", _D),
                ("vturb_kms", _D), ("out", C.c_void_p)]


class OdfStats(C.Structure):
    _fields_ = [("state", C.c_int), ("t_submit", C.c_double), ("t_admit", C.c_double),
                ("t_done", C.c_double), ("points", C.c_int64), ("line_evals", C.c_int64),
                ("survivors", C.c_int64), ("voigt_samples", C.c_int64), ("msg", C.c_char * 128)]

    def as_dict(self):
        return dict(state=STATE.get(self.state, str(self.state)), t_submit=self.t_submit,
                    t_admit=self.t_admit, t_done=self.t_done, points=self.points,
                    line_evals=self.line_evals, survivors=self.survivors,
                    voigt_samples=self.voigt_samples, msg=self.msg.decode(errors="replace"))


class OdfLoopInfo(C.Structure):
    _fields_ = [("pool_bytes", C.c_int64), ("resident_bytes", C.c_int64), ("peak_resident_bytes", C.c_int64),
                ("resident_requests", C.c_int32), ("peak_resident_requests", C.c_int32),
                ("queued_requests", C.c_int32), ("batches_in_flight", C.c_int32),
                ("slot_points", C.c_int32), ("slots_per_request", C.c_int32)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


#: every function the C ABI exports, with its ctypes signature
SIGNATURES = {
    "odf_plan": (C.c_int, [C.POINTER(OdfLines), C.POINTER(OdfSpecies), C.POINTER(OdfLayout),
                           C.POINTER(OdfOptions), C.POINTER(C.c_void_p)]),
    "odf_compute": (C.c_int, [C.c_void_p, C.POINTER(OdfRequest), C.POINTER(OdfStats)]),
    "odf_submit": (C.c_int, [C.c_void_p, C.POINTER(OdfRequest), _I64]),
    "odf_poll": (C.c_int, [C.c_void_p, C.c_int64, C.POINTER(OdfStats)]),
    "odf_wait": (C.c_int, [C.c_void_p, C.c_int64, C.c_double, C.POINTER(OdfStats)]),
    "odf_plan_destroy": (C.c_int, [C.c_void_p]),
    "odf_grid_points": (C.c_int64, [C.POINTER(OdfLayout)]),
    "odf_point_footprint": (C.c_int64, [C.c_void_p]),
    "odf_request_footprint": (C.c_int64, [C.c_void_p, C.c_int32]),
    "odf_loop_status": (C.c_int, [C.c_void_p, C.POINTER(OdfLoopInfo)]),
    "odf_last_error": (C.c_char_p, []),
    "odf_stage_lines": (C.c_int, [C.c_void_p, C.POINTER(OdfRequest), C.c_int32, _I64, _I64, _I64,
                                  _I32, _I32, _D, _D, _D]),
    "odf_stage_state": (C.c_int, [C.c_void_p, C.POINTER(OdfRequest), C.c_int32, _D, _I32]),
    "odf_stage_fine": (C.c_int, [C.c_void_p, C.POINTER(OdfRequest), C.c_int32, C.c_void_p]),
    "odf_stage_reduce": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "odf_debug_fail_next_batch": (C.c_int, [C.c_void_p, C.c_int64]),
    "odf_debug_set_newton_limit": (C.c_int, [C.c_void_p, C.c_int32]),
    "odf_stage_times": (C.c_int, [C.c_void_p, _D, _D, _I64, C.c_int32]),
    "odf_stage_records": (C.c_int, [C.c_void_p, C.POINTER(OdfRequest), C.c_int32, _I64, _I64, _I32,
                                    C.c_void_p, C.c_int64, _I32]),
    "odf_reduce_noalloc": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p]),
    "odf_noalloc_scratch_need": (C.c_int64, [C.c_void_p, C.c_int32]),
}


def load_library(path: str = LIB_PATH):
    if not os.path.exists(path):
        raise RuntimeError(f"HIP library {path} is not built; run __graft_entry__.build() "
                           "or python -m paper_2105_13611_amd.build")
    # One HIP runtime per process: import torch first so that the library's
    # libamdhip64.so.7 dependency resolves to the runtime torch has loaded.
    import torch  # noqa: F401
    lib = C.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_LIB = None


def lib():
    global _LIB
    if _LIB is None:
        _LIB = load_library()
    return _LIB


class OdfError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"odf error {code}: {msg}")
        self.code = code


def _check(code):
    if code != ODF_OK:
        raise OdfError(code, lib().odf_last_error().decode(errors="replace"))


def _f64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _i32(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.int32))


def _i64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.int64))


def _ptr(a, t):
    return a.ctypes.data_as(t)


def make_layout(layout):
    keep = dict(edges=_i64(layout.bin_edges), frac=_f64(layout.step_frac))
    st = OdfLayout(float(layout.lambda_first_nm), float(layout.lambda_last_nm),
                   float(layout.resolving_power), int(keep["edges"].size - 1),
                   _ptr(keep["edges"], _I64), int(keep["frac"].size), _ptr(keep["frac"], _D))
    return st, keep


def grid_points(layout) -> int:
    st, keep = make_layout(layout)
    return int(lib().odf_grid_points(C.byref(st)))


@dataclass
class _PointArrays:
    abundance: np.ndarray
    T: np.ndarray
    logP: np.ndarray
    vt: np.ndarray


def _request(abundance, points, out_ptr):
    a = _PointArrays(_f64(abundance), _f64(points.T_K), _f64(points.log10_P), _f64(points.vturb_kms))
    r = OdfRequest(_ptr(a.abundance, _D), int(a.T.size), _ptr(a.T, _D), _ptr(a.logP, _D),
                   _ptr(a.vt, _D), C.c_void_p(out_ptr))
    return r, a


class Plan:
    """A resident line list, species table and bin layout on one GPU.

    workspace_bytes of device memory are taken as a torch tensor and used for
    every intermediate array; the line list is uploaded once.
    """

    def __init__(self, lines, species, layout, options, workspace_bytes=None, device="cuda:0",
                 max_batch_points=0, loop_streams=0, stream=None, kernel_timing=False):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.precision = options.precision
        self.out_dtype = torch.float64 if options.precision == "fp64" else torch.float32
        torch.cuda.set_device(self.device)
        # The library shares torch's HIP runtime; it must be initialised on the
        # device before the library registers its code objects.
        if workspace_bytes is None:
            workspace_bytes = 1 << 30
        self.workspace = torch.empty(int(workspace_bytes), dtype=torch.uint8, device=self.device)
        torch.cuda.synchronize(self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        L = lines
        self._keep = dict(
            lam=_f64(L.lambda_nm), gf=_f64(L.log_gf), e=_f64(L.e_low_ev), sp=_i32(L.species),
            st=_i32(L.stage), gr=_f64(L.log_g_rad), gs=_f64(L.log_g_stark), gw=_f64(L.log_g_vdw),
            mass=_f64(species.mass_amu), chi=_f64(species.chi_ev), part=_f64(species.part_fn))
        k = self._keep
        self.n_lines = int(k["lam"].size)
        self.n_species = int(k["mass"].size)
        cl = OdfLines(self.n_lines, _ptr(k["lam"], _D), _ptr(k["gf"], _D), _ptr(k["e"], _D),
                      _ptr(k["sp"], _I32), _ptr(k["st"], _I32), _ptr(k["gr"], _D),
                      _ptr(k["gs"], _D), _ptr(k["gw"], _D))
        cs = OdfSpecies(self.n_species, int(species.part_fn.shape[1]), _ptr(k["mass"], _D),
                        _ptr(k["chi"], _D), _ptr(k["part"], _D))
        self.layout_c, self._layout_keep = make_layout(layout)
        self.n_bins = int(self.layout_c.n_bins)
        self.n_steps = int(self.layout_c.n_steps)
        self.N = int(lib().odf_grid_points(C.byref(self.layout_c)))
        opts = OdfOptions(PREC[options.precision], MEAN[options.mean], options.cutoff,
                          options.window_cap_doppler, options.pe_over_p, options.kappa_c_ref,
                          options.lambda_c_ref_nm, options.kappa_c_power,
                          C.c_void_p(self.workspace.data_ptr()), int(workspace_bytes),
                          C.c_void_p(self.stream.cuda_stream), int(max_batch_points), int(loop_streams),
                          int(bool(kernel_timing)), OUTPUT[getattr(options, "output", "table")],
                          ELECTRONS[getattr(options, "electrons", "fixed")])
        self.output = getattr(options, "output", "table")
        h = C.c_void_p()
        _check(lib().odf_plan(C.byref(cl), C.byref(cs), C.byref(self.layout_c), C.byref(opts), C.byref(h)))
        self.handle = h
        self._outs = {}

    # -- lifecycle ---------------------------------------------------------
    def destroy(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            lib().odf_plan_destroy(self.handle)
            self.handle = None
        # the library no longer uses the workspace: release it
        self.workspace = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.destroy()

    # -- queries -------------------------------------------------------------
    def point_footprint(self) -> int:
        return int(lib().odf_point_footprint(self.handle))

    def request_footprint(self, n_points: int) -> int:
        return int(lib().odf_request_footprint(self.handle, int(n_points)))

    def loop_status(self):
        """The request loop's pool occupancy (odf_loop_info as a dict)."""
        st = OdfLoopInfo()
        _check(lib().odf_loop_status(self.handle, C.byref(st)))
        return st.as_dict()

    def out_shape(self, n_points):
        """[points][bins][steps] for ODF tables, [points][N] for fine-grid opacity."""
        if self.output == "fine":
            return (n_points, self.N)
        return (n_points, self.n_bins, self.n_steps)

    def new_out(self, n_points):
        return self.torch.empty(self.out_shape(n_points), dtype=self.out_dtype, device=self.device)

    # -- compute ---------------------------------------------------------------
    def compute(self, abundance, points, out=None):
        """Blocking ODF table for every point: returns (out tensor, stats dict)."""
        if out is None:
            out = self.new_out(points.n_points)
        self._check_out(out, points.n_points)
        r, keep = _request(abundance, points, out.data_ptr())
        st = OdfStats()
        _check(lib().odf_compute(self.handle, C.byref(r), C.byref(st)))
        del keep
        return out, st.as_dict()

    def submit(self, abundance, points, out=None):
        """Queue a request; returns (ticket, out tensor).  Keep `out` alive."""
        if out is None:
            out = self.new_out(points.n_points)
        self._check_out(out, points.n_points)
        r, keep = _request(abundance, points, out.data_ptr())
        t = C.c_int64()
        _check(lib().odf_submit(self.handle, C.byref(r), C.byref(t)))
        self._outs[t.value] = out
        return t.value, out

    def poll(self, ticket):
        st = OdfStats()
        _check(lib().odf_poll(self.handle, int(ticket), C.byref(st)))
        d = st.as_dict()
        if d["state"] in ("DONE", "FAILED"):
            self._outs.pop(int(ticket), None)
        return d

    def wait(self, ticket, timeout_s=600.0):
        st = OdfStats()
        _check(lib().odf_wait(self.handle, int(ticket), float(timeout_s), C.byref(st)))
        d = st.as_dict()
        if d["state"] in ("DONE", "FAILED"):
            self._outs.pop(int(ticket), None)
        return d

    STAGES = ("point_state", "select", "scan", "emit", "voigt", "odf")

    def stage_times(self, reset=True):
        """{stage: {"ms", "busy_ms", "launches"}} from the HIP events of
        odf_compute: summed launch durations, the union of the launch
        intervals, and the launch count."""
        ms = np.zeros(6)
        busy = np.zeros(6)
        n = np.zeros(6, np.int64)
        _check(lib().odf_stage_times(self.handle, _ptr(ms, _D), _ptr(busy, _D), _ptr(n, _I64),
                                     int(bool(reset))))
        return {k: dict(ms=float(ms[i]), busy_ms=float(busy[i]), launches=int(n[i]))
                for i, k in enumerate(self.STAGES)}

    def fail_next_batch(self, ticket):
        _check(lib().odf_debug_fail_next_batch(self.handle, int(ticket)))

    def set_newton_limit(self, max_steps):
        _check(lib().odf_debug_set_newton_limit(self.handle, int(max_steps)))

    def _check_out(self, out, n_points):
        t = self.torch
        if out.dtype != self.out_dtype or out.device != self.device or not out.is_contiguous():
            raise ValueError(f"out must be a contiguous {self.out_dtype} tensor on {self.device}")
        if tuple(out.shape) != self.out_shape(n_points):
            raise ValueError(f"out shape {tuple(out.shape)} != {self.out_shape(n_points)}")
        del t

    # -- stage entry points ------------------------------------------------------
    def stage_lines(self, abundance, points, point=0):
        L = max(self.n_lines, 1)
        o = dict(orig=np.zeros(L, np.int64), jlo=np.zeros(L, np.int32), jhi=np.zeros(L, np.int32),
                 S=np.zeros(L), a=np.zeros(L), b=np.zeros(L))
        ns, nsamp = C.c_int64(), C.c_int64()
        r, keep = _request(abundance, points, 0)
        _check(lib().odf_stage_lines(self.handle, C.byref(r), int(point), C.byref(ns), C.byref(nsamp),
                                     _ptr(o["orig"], _I64), _ptr(o["jlo"], _I32), _ptr(o["jhi"], _I32),
                                     _ptr(o["S"], _D), _ptr(o["a"], _D), _ptr(o["b"], _D)))
        n = ns.value
        res = {k: v[:n].copy() for k, v in o.items()}
        res["n_surv"] = n
        res["voigt_samples"] = nsamp.value
        return res

    #: the FP32 survivor record of mixed plans (48 bytes) and the FP64 one (64 bytes)
    REC32 = np.dtype([("J", "<i4"), ("jlo", "<i4"), ("jhi", "<i4"), ("czh", "<i4"), ("phi", "<f4"),
                      ("c1", "<f4"), ("A", "<f4"), ("B", "<f4"), ("D", "<f4"), ("E", "<f4"),
                      ("S", "<f4"), ("y", "<f4")])
    REC64 = np.dtype([("J", "<i4"), ("jlo", "<i4"), ("jhi", "<i4"), ("czh", "<i4"), ("z40", "<i4"),
                      ("li", "<i4"), ("pad0", "<i4"), ("pad1", "<i4"), ("phi", "<f8"), ("S", "<f8"),
                      ("y", "<f8"), ("c1", "<f8")])

    def stage_records(self, abundance, points, point=0):
        """Survivor records of one point as the plan's Voigt kernel reads
        them: (structured array, (J, packed zones) int32 pairs or None, the
        number of narrow-class records, which come first)."""
        dt = self.REC32 if self.precision == "mixed" else self.REC64
        cap = max(self.n_lines, 1)
        rec = np.zeros(cap, dtype=dt)
        wz = np.zeros((cap, 2), dtype=np.int32)
        ns, nn, rb = C.c_int64(), C.c_int64(), C.c_int32()
        r, keep = _request(abundance, points, 0)
        _check(lib().odf_stage_records(self.handle, C.byref(r), int(point), C.byref(ns), C.byref(nn),
                                       C.byref(rb), C.c_void_p(rec.ctypes.data), cap, _ptr(wz, _I32)))
        assert rb.value == dt.itemsize
        n = ns.value
        return rec[:n].copy(), (wz[:n].copy() if self.precision == "mixed" else None), nn.value

    def stage_state(self, abundance, points, point=0):
        """Gas state of one point: dict(n_e, n_heavy, n_H, rho, iterations)."""
        st = np.zeros(4)
        it = C.c_int32()
        r, keep = _request(abundance, points, 0)
        _check(lib().odf_stage_state(self.handle, C.byref(r), int(point), _ptr(st, _D), C.byref(it)))
        return dict(n_e=float(st[0]), n_heavy=float(st[1]), n_H=float(st[2]), rho=float(st[3]),
                    iterations=int(it.value))

    def stage_fine(self, abundance, points, point=0):
        kap = self.torch.empty(self.N, dtype=self.out_dtype, device=self.device)
        r, keep = _request(abundance, points, 0)
        _check(lib().odf_stage_fine(self.handle, C.byref(r), int(point), C.c_void_p(kap.data_ptr())))
        return kap

    def noalloc_scratch_need(self, n_points):
        return int(lib().odf_noalloc_scratch_need(self.handle, int(n_points)))

    def reduce_noalloc(self, kappa, out):
        """ODF tables of kappa [n][N] into out [n][bins][steps] (both device
        tensors of the plan's type, caller-allocated) through the
        allocation-free entry point, on the plan's stream; not waited for."""
        n = int(kappa.shape[0])
        for t, shape in ((kappa, (n, self.N)), (out, (n, self.n_bins, self.n_steps))):
            if t.dtype != self.out_dtype or t.device != self.device or not t.is_contiguous() \
                    or tuple(t.shape) != shape:
                raise ValueError(f"expected a contiguous {self.out_dtype} tensor {shape} on {self.device}")
        _check(lib().odf_reduce_noalloc(self.handle, C.c_void_p(kappa.data_ptr()), n,
                                        C.c_void_p(out.data_ptr()), C.c_void_p(self.stream.cuda_stream)))
        return out

    def stage_reduce(self, kappa):
        kappa = kappa.to(device=self.device, dtype=self.out_dtype).contiguous()
        if kappa.numel() != self.N:
            raise ValueError(f"kappa must hold N={self.N} values")
        out = self.torch.empty((self.n_bins, self.n_steps), dtype=self.out_dtype, device=self.device)
        self.stream.synchronize()
        _check(lib().odf_stage_reduce(self.handle, C.c_void_p(kappa.data_ptr()), C.c_void_p(out.data_ptr())))
        return out


def plan_for(workload, precision=None, **kw):
    """Plan for a workload from paper_2105_13611_amd.workload."""
    from dataclasses import replace
    opts = workload.options if precision is None else replace(workload.options, precision=precision)
    return Plan(workload.lines, workload.species, workload.layout, opts, **kw)
