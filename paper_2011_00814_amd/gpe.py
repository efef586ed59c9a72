"""Thin ctypes binding of libgpe (include/gpe.h): argument marshalling only.

Every step of the method runs in the HIP kernels of libgpe.so; PyTorch only
provides the device workspace and the stream.  Importing this module does not
load the library; the first call does, and fails loudly when the library has
not been built (``python -m paper_2011_00814_amd.build``).
"""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "_lib", "libgpe.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "gpe.h")

GPE_OK, GPE_EINVAL, GPE_EUNSTABLE, GPE_EWORKSPACE, GPE_EHIP, GPE_ENONFINITE = 0, -1, -2, -3, -4, -5
GPE_GEOM_2D, GPE_GEOM_AXISYM, GPE_GEOM_3D = 0, 1, 2
GPE_FP64, GPE_FP32 = 0, 1
GPE_FIELD_P, GPE_FIELD_U, GPE_FIELD_V, GPE_FIELD_W, GPE_FIELD_PHI = 0, 1, 2, 3, 4
GPE_H2D, GPE_D2H = 0, 1
GPE_INIT_NONE, GPE_INIT_DROP, GPE_INIT_BUBBLE, GPE_INIT_LAYER, GPE_INIT_ELLIPSE = 0, 1, 2, 3, 4
GPE_CH_CONSERVATIVE, GPE_CH_ADVECTIVE = 0, 1
GPE_SCHEME_PAPER, GPE_SCHEME_NO_PAVG, GPE_SCHEME_NO_BULK = 0, 1, 2

i32, f64 = ctypes.c_int32, ctypes.c_double


class gpe_params(ctypes.Structure):
    _fields_ = [
        ("geometry", i32), ("precision", i32), ("n", i32 * 3), ("bc", i32 * 6),
        ("lattice", i32), ("allow_unstable", i32), ("ch_transport", i32), ("dt", f64), ("cs2", f64),
        ("rho_l", f64), ("rho_g", f64), ("eta_l", f64), ("eta_g", f64),
        ("sigma", f64), ("mobility", f64), ("width", f64), ("g", f64 * 3), ("rho_ref", f64),
        ("init_kind", i32), ("scheme", i32), ("zchunk", i32), ("reserved", i32), ("init_center", f64 * 3),
        ("init_radius", f64),
        ("init_width", f64), ("init_amp", f64),
    ]


class gpe_problem(ctypes.Structure):
    _fields_ = [
        ("geometry", i32), ("precision", i32), ("n", i32 * 3), ("bc", i32 * 6), ("lattice", i32),
        ("ch_transport", i32), ("scheme", i32), ("time_scale", i32), ("visc_group", i32), ("st_group", i32),
        ("gravity", i32), ("rho_ref_kind", i32), ("reserved", i32),
        ("N_L", f64), ("N_t", f64), ("Ma", f64), ("L_g_factor", f64), ("r_rho", f64), ("r_eta", f64),
        ("Re", f64), ("Oh", f64), ("Mo", f64), ("We", f64), ("Eo", f64), ("sigma", f64), ("Pe", f64),
        ("Cn", f64), ("G", f64 * 3), ("Fr", f64), ("rho_ref_value", f64),
    ]


GPE_TIME_NT, GPE_TIME_MA = 0, 1
VISC_GROUP = {"Re": 0, "Oh": 1, "Mo": 2, "capillary": 3}
ST_GROUP = {"none": 0, "We": 1, "Eo": 2, "sigma": 3, "capillary": 4}
GRAVITY = {"G": 0, "Fr": 1, "Eo": 2}
RHO_REF = {"zero": 0, "liquid": 1, "gas": 2}
GPE_RHO_REF_VALUE = 3


class gpe_diag(ctypes.Structure):
    _fields_ = [
        ("step", ctypes.c_int64), ("t", f64), ("mass", f64), ("mass_abs0", f64), ("ke", f64),
        ("max_div", f64), ("phi_min", f64), ("phi_max", f64), ("umax", f64),
        ("finite", i32), ("reserved", i32),
    ]


class GpeError(RuntimeError):
    def __init__(self, code, what):
        self.code = code
        super().__init__(f"{what}: {gpe_strerror(code)} ({code})")


_lib = None


def header_functions():
    """Names of the functions declared in include/gpe.h."""
    src = open(HEADER).read()
    return re.findall(r"^\s*(?:int|int64_t|size_t|void|void\*|const char\*|gpe_state\*)\s+(gpe_\w+)\s*\(", src, re.M)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2011_00814_amd.build`")
        # torch provides the device memory and streams: load its HIP runtime
        # first so that the library binds to the same runtime instance
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        vp, sz = ctypes.c_void_p, ctypes.c_size_t
        L.gpe_params_from_dimensionless.argtypes = [ctypes.POINTER(gpe_problem), ctypes.POINTER(gpe_params)]
        L.gpe_params_from_dimensionless.restype = ctypes.c_int
        L.gpe_hbm_stream.argtypes = [ctypes.c_int32, vp, vp, sz, ctypes.c_int32, vp]
        L.gpe_hbm_stream.restype = ctypes.c_int
        L.gpe_workspace_bytes.argtypes = [ctypes.POINTER(gpe_params)]
        L.gpe_workspace_bytes.restype = sz
        L.gpe_init_state.argtypes = [ctypes.POINTER(gpe_params), vp, sz, vp, vp, vp, ctypes.POINTER(vp)]
        L.gpe_init_state.restype = ctypes.c_int
        L.gpe_rk3_step.argtypes = [vp]
        L.gpe_rk3_step.restype = ctypes.c_int
        L.gpe_run_n.argtypes = [vp, ctypes.c_int64]
        L.gpe_run_n.restype = ctypes.c_int
        L.gpe_diagnostics.argtypes = [vp, ctypes.POINTER(gpe_diag)]
        L.gpe_diagnostics.restype = ctypes.c_int
        d7 = ctypes.POINTER(ctypes.c_double)
        L.gpe_phase_stats.argtypes = [vp, d7]
        L.gpe_phase_stats.restype = ctypes.c_int
        L.gpe_interface_extent.argtypes = [vp, d7]
        L.gpe_interface_extent.restype = ctypes.c_int
        L.gpe_line_crossings.argtypes = [vp, i32, i32, i32, d7]
        L.gpe_line_crossings.restype = ctypes.c_int
        L.gpe_copy_field.argtypes = [vp, ctypes.c_int, ctypes.c_int, vp, sz]
        L.gpe_copy_field.restype = ctypes.c_int
        L.gpe_field_offset.argtypes = [vp, ctypes.c_int]
        L.gpe_field_offset.restype = sz
        L.gpe_field_pointer.argtypes = [vp, ctypes.c_int]
        L.gpe_field_pointer.restype = vp
        L.gpe_field_pitch.argtypes = [vp]
        L.gpe_field_pitch.restype = ctypes.c_int64
        L.gpe_set_step_time.argtypes = [vp, ctypes.c_int64, f64]
        L.gpe_set_step_time.restype = ctypes.c_int
        L.gpe_kernel_times.argtypes = [vp, ctypes.c_int64, ctypes.c_int, ctypes.POINTER(ctypes.c_char_p),
                                       ctypes.POINTER(f64), ctypes.POINTER(f64)]
        L.gpe_kernel_times.restype = ctypes.c_int
        L.gpe_kernel_times_masked.argtypes = [vp, ctypes.c_int64, ctypes.c_uint32, ctypes.c_int,
                                              ctypes.POINTER(ctypes.c_char_p), ctypes.POINTER(f64),
                                              ctypes.POINTER(f64)]
        L.gpe_kernel_times_masked.restype = ctypes.c_int
        L.gpe_destroy.argtypes = [vp]
        L.gpe_destroy.restype = None
        L.gpe_strerror.argtypes = [ctypes.c_int]
        L.gpe_strerror.restype = ctypes.c_char_p
        L.gpe_ensemble_workspace_bytes.argtypes = [ctypes.POINTER(gpe_params), i32]
        L.gpe_ensemble_workspace_bytes.restype = sz
        L.gpe_ensemble_create.argtypes = [ctypes.POINTER(gpe_params), i32, vp, sz, vp, ctypes.POINTER(vp)]
        L.gpe_ensemble_create.restype = ctypes.c_int
        L.gpe_ensemble_run_n.argtypes = [vp, ctypes.c_int64]
        L.gpe_ensemble_run_n.restype = ctypes.c_int
        L.gpe_ensemble_autotune.argtypes = [vp, i32, ctypes.POINTER(i32)]
        L.gpe_ensemble_autotune.restype = ctypes.c_int
        L.gpe_ensemble_finite.argtypes = [vp, ctypes.POINTER(i32)]
        L.gpe_ensemble_finite.restype = ctypes.c_int
        L.gpe_ensemble_case.argtypes = [vp, i32]
        L.gpe_ensemble_case.restype = vp
        L.gpe_ensemble_destroy.argtypes = [vp]
        L.gpe_ensemble_destroy.restype = None
        _lib = L
    return _lib


# ---- functions with the names of the C-ABI ---------------------------------
def gpe_strerror(code: int) -> str:
    return lib().gpe_strerror(int(code)).decode()


def gpe_params_from_dimensionless(problem: gpe_problem) -> gpe_params:
    out = gpe_params()
    rc = lib().gpe_params_from_dimensionless(ctypes.byref(problem), ctypes.byref(out))
    if rc:
        raise GpeError(rc, "gpe_params_from_dimensionless")
    return out


def gpe_workspace_bytes(params: gpe_params) -> int:
    return int(lib().gpe_workspace_bytes(ctypes.byref(params)))


def gpe_init_state(params, d_workspace: int, nbytes: int, stream: int, h_phi0=None, h_p0=None):
    handle = ctypes.c_void_p()
    phi = None if h_phi0 is None else np.ascontiguousarray(h_phi0, dtype=np.float64)
    p0 = None if h_p0 is None else np.ascontiguousarray(h_p0, dtype=np.float64)
    rc = lib().gpe_init_state(ctypes.byref(params), ctypes.c_void_p(d_workspace), nbytes,
                              ctypes.c_void_p(stream),
                              None if phi is None else phi.ctypes.data_as(ctypes.c_void_p),
                              None if p0 is None else p0.ctypes.data_as(ctypes.c_void_p),
                              ctypes.byref(handle))
    if rc:
        raise GpeError(rc, "gpe_init_state")
    return handle


def gpe_rk3_step(h):
    rc = lib().gpe_rk3_step(h)
    if rc:
        raise GpeError(rc, "gpe_rk3_step")


def gpe_run_n(h, n: int):
    rc = lib().gpe_run_n(h, int(n))
    if rc:
        raise GpeError(rc, "gpe_run_n")


def gpe_diagnostics(h, check=True) -> dict:
    d = gpe_diag()
    rc = lib().gpe_diagnostics(h, ctypes.byref(d))
    if rc and (check or rc != GPE_ENONFINITE):
        raise GpeError(rc, "gpe_diagnostics")
    return {k: getattr(d, k) for k, _ in gpe_diag._fields_ if k != "reserved"}


def gpe_phase_stats(h) -> dict:
    """Liquid region (phi > 0): weighted volume, centroid and mean centre
    velocity per axis (NaN where undefined)."""
    out = (ctypes.c_double * 7)()
    rc = lib().gpe_phase_stats(h, out)
    if rc:
        raise GpeError(rc, "gpe_phase_stats")
    return {"volume": out[0], "centroid": tuple(out[1:4]), "velocity": tuple(out[4:7])}


def gpe_interface_extent(h) -> list:
    """[(smallest, largest) phi = 0 crossing] per axis (NaN if none)."""
    out = (ctypes.c_double * 6)()
    rc = lib().gpe_interface_extent(h, out)
    if rc:
        raise GpeError(rc, "gpe_interface_extent")
    return [(out[2 * a], out[2 * a + 1]) for a in range(3)]


def gpe_line_crossings(h, axis: int, i0: int, i1: int = 0) -> tuple:
    """(first, last) phi = 0 crossing on one grid line (NaN if none)."""
    out = (ctypes.c_double * 2)()
    rc = lib().gpe_line_crossings(h, int(axis), int(i0), int(i1), out)
    if rc:
        raise GpeError(rc, "gpe_line_crossings")
    return out[0], out[1]


def gpe_copy_field(h, field: int, direction: int, host: np.ndarray):
    assert host.dtype == np.float64 and host.flags["C_CONTIGUOUS"]
    rc = lib().gpe_copy_field(h, int(field), int(direction), host.ctypes.data_as(ctypes.c_void_p),
                              host.nbytes)
    if rc:
        raise GpeError(rc, "gpe_copy_field")


def gpe_field_offset(h, field: int) -> int:
    return int(lib().gpe_field_offset(h, int(field)))


def gpe_field_pointer(h, field: int) -> int:
    p = lib().gpe_field_pointer(h, int(field))
    if not p:
        raise GpeError(GPE_EINVAL, "gpe_field_pointer")
    return int(p)


def gpe_field_pitch(h) -> int:
    n = int(lib().gpe_field_pitch(h))
    if n < 0:
        raise GpeError(n, "gpe_field_pitch")
    return n


def gpe_set_step_time(h, step: int, t: float):
    rc = lib().gpe_set_step_time(h, int(step), float(t))
    if rc:
        raise GpeError(rc, "gpe_set_step_time")


def gpe_kernel_times(h, nsteps: int, maxk: int = 16):
    names = (ctypes.c_char_p * maxk)()
    ms = (f64 * maxk)()
    nb = (f64 * maxk)()
    rc = lib().gpe_kernel_times(h, int(nsteps), maxk, names, ms, nb)
    if rc < 0:
        raise GpeError(rc, "gpe_kernel_times")
    return [(names[q].decode(), ms[q], nb[q]) for q in range(rc)]


def gpe_kernel_times_masked(h, nsteps: int, mask: int, maxk: int = 16):
    names = (ctypes.c_char_p * maxk)()
    ms = (f64 * maxk)()
    nb = (f64 * maxk)()
    rc = lib().gpe_kernel_times_masked(h, int(nsteps), int(mask) & 0xFFFFFFFF, maxk, names, ms, nb)
    if rc < 0:
        raise GpeError(rc, "gpe_kernel_times_masked")
    return [(names[q].decode(), ms[q], nb[q]) for q in range(rc)]


GPE_STREAM_READ, GPE_STREAM_WRITE, GPE_STREAM_COPY = 0, 1, 2


def gpe_hbm_stream(mode: int, d_dst: int, d_src: int, nbytes: int, workgroups: int, stream: int):
    rc = lib().gpe_hbm_stream(int(mode), ctypes.c_void_p(d_dst), ctypes.c_void_p(d_src), ctypes.c_size_t(nbytes),
                              int(workgroups), ctypes.c_void_p(stream))
    if rc:
        raise GpeError(rc, "gpe_hbm_stream")


def gpe_destroy(h):
    lib().gpe_destroy(h)


def _params_array(params_list):
    arr = (gpe_params * len(params_list))()
    for q, P in enumerate(params_list):
        arr[q] = P
    return arr


def gpe_ensemble_workspace_bytes(params_list) -> int:
    return int(lib().gpe_ensemble_workspace_bytes(_params_array(params_list), len(params_list)))


def gpe_ensemble_create(params_list, d_workspace: int, nbytes: int, stream: int):
    handle = ctypes.c_void_p()
    rc = lib().gpe_ensemble_create(_params_array(params_list), len(params_list), ctypes.c_void_p(d_workspace),
                                   nbytes, ctypes.c_void_p(stream), ctypes.byref(handle))
    if rc:
        raise GpeError(rc, "gpe_ensemble_create")
    return handle


def gpe_ensemble_run_n(e, n: int):
    rc = lib().gpe_ensemble_run_n(e, int(n))
    if rc:
        raise GpeError(rc, "gpe_ensemble_run_n")


def gpe_ensemble_autotune(e, trial_steps: int, count: int) -> np.ndarray:
    rows = (i32 * count)()
    rc = lib().gpe_ensemble_autotune(e, int(trial_steps), rows)
    if rc:
        raise GpeError(rc, "gpe_ensemble_autotune")
    return np.array(rows[:], dtype=np.int32)


def gpe_ensemble_finite(e, count: int) -> np.ndarray:
    out = (i32 * count)()
    rc = lib().gpe_ensemble_finite(e, out)
    if rc:
        raise GpeError(rc, "gpe_ensemble_finite")
    return np.array(out[:], dtype=np.int32)


def gpe_ensemble_case(e, i: int):
    h = lib().gpe_ensemble_case(e, int(i))
    if not h:
        raise GpeError(GPE_EINVAL, "gpe_ensemble_case")
    return ctypes.c_void_p(h)


def gpe_ensemble_destroy(e):
    lib().gpe_ensemble_destroy(e)


# ---- problem statement (dimensionless groups) -> lattice-unit dictionary ------
STRUCTURAL = ("dim", "axisym", "n", "bc", "lattice", "precision", "ch_transport", "scheme",
              "allow_unstable", "init", "meta", "zchunk")


def problem_struct(st: dict) -> gpe_problem:
    """gpe_problem of a problem statement dictionary (see workloads.py)."""
    pr = gpe_problem()
    if st["dim"] == 3:
        pr.geometry = GPE_GEOM_3D
    else:
        pr.geometry = GPE_GEOM_AXISYM if st.get("axisym") else GPE_GEOM_2D
    pr.precision = GPE_FP32 if st.get("precision", "fp64") == "fp32" else GPE_FP64
    for a in range(3):
        pr.n[a] = int(st["n"][a])
    for q in range(6):
        pr.bc[q] = int(st["bc"][q])
    pr.lattice = int(st["lattice"])
    pr.ch_transport = int(st.get("ch_transport", GPE_CH_CONSERVATIVE))
    pr.scheme = int(st.get("scheme", GPE_SCHEME_PAPER))
    if "N_t" in st:
        pr.time_scale, pr.N_t = GPE_TIME_NT, float(st["N_t"])
    else:
        pr.time_scale, pr.Ma = GPE_TIME_MA, float(st["Ma"])
    pr.visc_group = VISC_GROUP[st["visc"]]
    pr.st_group = ST_GROUP[st.get("st", "none")]
    pr.gravity = GRAVITY[st.get("gravity", "G")]
    ref = st.get("rho_ref", "zero")
    if isinstance(ref, str):
        pr.rho_ref_kind = RHO_REF[ref]
    else:
        pr.rho_ref_kind, pr.rho_ref_value = GPE_RHO_REF_VALUE, float(ref)
    pr.N_L = float(st["N_L"])
    pr.L_g_factor = float(st.get("L_g", 1.0))
    for key in ("r_rho", "r_eta", "Re", "Oh", "Mo", "We", "Eo", "sigma", "Pe", "Cn", "Fr"):
        setattr(pr, key, float(st.get(key, 0.0)))
    for a, x in enumerate(st.get("G", (0.0, 0.0, 0.0))):
        pr.G[a] = float(x)
    return pr


def lattice_problem(prob: dict) -> dict:
    """Lattice-unit problem dictionary: a problem statement (it has N_L) is
    mapped by the library's gpe_params_from_dimensionless; a lattice-unit
    dictionary is returned as it is."""
    if "N_L" not in prob:
        return prob
    P = gpe_params_from_dimensionless(problem_struct(prob))
    out = {k: prob[k] for k in STRUCTURAL if k in prob}
    out.setdefault("axisym", 0)
    out.update(dt=P.dt, cs2=P.cs2, rho_l=P.rho_l, rho_g=P.rho_g, eta_l=P.eta_l, eta_g=P.eta_g, sigma=P.sigma,
               mob=P.mobility, width=P.width, g=tuple(P.g), rho_ref=P.rho_ref)
    return out


# ---- problem dictionary -> gpe_params ----------------------------------------
def params_from_problem(prob: dict) -> gpe_params:
    """gpe_params of a problem dictionary (a statement in dimensionless
    groups goes through gpe_params_from_dimensionless first)."""
    prob = lattice_problem(prob)
    P = gpe_params()
    if prob["dim"] == 3:
        P.geometry = GPE_GEOM_3D
    else:
        P.geometry = GPE_GEOM_AXISYM if prob.get("axisym") else GPE_GEOM_2D
    P.precision = GPE_FP32 if prob.get("precision", "fp64") == "fp32" else GPE_FP64
    for a in range(3):
        P.n[a] = int(prob["n"][a])
    for s in range(6):
        P.bc[s] = int(prob["bc"][s])
    P.lattice = int(prob["lattice"])
    P.allow_unstable = int(prob.get("allow_unstable", 0))
    P.ch_transport = int(prob.get("ch_transport", GPE_CH_CONSERVATIVE))
    P.scheme = int(prob.get("scheme", GPE_SCHEME_PAPER))
    P.zchunk = int(prob.get("zchunk", 0))
    P.dt, P.cs2 = float(prob["dt"]), float(prob["cs2"])
    P.rho_l, P.rho_g = float(prob["rho_l"]), float(prob["rho_g"])
    P.eta_l, P.eta_g = float(prob["eta_l"]), float(prob["eta_g"])
    P.sigma, P.mobility, P.width = float(prob["sigma"]), float(prob["mob"]), float(prob["width"])
    for a in range(3):
        P.g[a] = float(prob["g"][a])
    P.rho_ref = float(prob["rho_ref"])
    init = prob.get("init")
    if init:
        P.init_kind = int(init["kind"])
        for a in range(3):
            P.init_center[a] = float(init.get("center", (0, 0, 0))[a])
        P.init_radius = float(init.get("radius", 0.0))
        P.init_width = float(init.get("width", prob["width"]))
        P.init_amp = float(init.get("amp", 0.0))
    return P


class _Grid:
    """Field access and diagnostics of one grid handle (self.h, self.prob,
    self.shape, self.stream)."""

    FIELDS = {"p": GPE_FIELD_P, "u": GPE_FIELD_U, "v": GPE_FIELD_V, "w": GPE_FIELD_W, "phi": GPE_FIELD_PHI}

    def synchronize(self):
        self.stream.synchronize()

    def diagnostics(self, check=True) -> dict:
        return gpe_diagnostics(self.h, check)

    def phase_stats(self) -> dict:
        return gpe_phase_stats(self.h)

    def interface_extent(self) -> list:
        return gpe_interface_extent(self.h)

    def line_crossings(self, axis: int, i0: int, i1: int = 0) -> tuple:
        return gpe_line_crossings(self.h, axis, i0, i1)

    def get(self, key: str) -> np.ndarray:
        out = np.empty(self.shape, dtype=np.float64)
        gpe_copy_field(self.h, self.FIELDS[key], GPE_D2H, out)
        return out

    def set(self, key: str, arr):
        a = np.ascontiguousarray(np.asarray(arr, dtype=np.float64).reshape(self.shape))
        gpe_copy_field(self.h, self.FIELDS[key], GPE_H2D, a)

    def state(self) -> dict:
        keys = ("p", "u", "v", "phi") + (("w",) if self.prob["dim"] == 3 else ())
        st = {k: self.get(k) for k in keys}
        if self.prob["dim"] != 3:
            st["w"] = None
        return st


class Solver(_Grid):
    """One simulation on one GPU: a torch-allocated workspace, a torch stream
    and a libgpe handle.  Marshalling only."""

    def __init__(self, prob: dict, state: dict | None = None, device: str = "cuda:0", stream=None):
        import torch

        self.prob = lattice_problem(prob)
        self.params = params_from_problem(self.prob)
        nbytes = gpe_workspace_bytes(self.params)
        if nbytes == 0:
            raise GpeError(GPE_EINVAL, "gpe_workspace_bytes")
        self.device = torch.device(device)
        self.ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self.ws.data_ptr()
        self.ws_ptr = (base + 255) // 256 * 256
        self.ws_bytes = nbytes
        self.stream = stream if stream is not None else torch.cuda.Stream(device=self.device)
        nx, ny, nz = prob["n"]
        self.shape = (nz, ny, nx)
        phi0 = p0 = None
        if state is not None:
            phi0 = np.ascontiguousarray(state["phi"], dtype=np.float64).reshape(self.shape)
            p0 = np.ascontiguousarray(state["p"], dtype=np.float64).reshape(self.shape)
        self.h = gpe_init_state(self.params, self.ws_ptr, nbytes, self.stream.cuda_stream, phi0, p0)
        if state is not None:
            for key in ("u", "v") + (("w",) if prob["dim"] == 3 else ()):
                if state.get(key) is not None and np.any(state[key]):
                    self.set(key, state[key])

    def rk3_step(self):
        gpe_rk3_step(self.h)

    def run(self, n: int):
        gpe_run_n(self.h, n)

    def kernel_times(self, nsteps: int, mask=None):
        if mask is None:
            return gpe_kernel_times(self.h, nsteps)
        return gpe_kernel_times_masked(self.h, nsteps, mask)

    def close(self):
        if getattr(self, "h", None) is not None:
            gpe_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class EnsembleCase(_Grid):
    """Borrowed view of one case of an Ensemble (owned by the ensemble)."""

    def __init__(self, ens: "Ensemble", i: int):
        self.prob = ens.probs[i]
        self.h = gpe_ensemble_case(ens.e, i)
        self.stream = ens.stream
        nx, ny, nz = self.prob["n"]
        self.shape = (nz, ny, nx)


class Ensemble:
    """A batch of independent 2-D (or axisymmetric) cases advanced together:
    one torch-allocated workspace, one stream, one libgpe ensemble handle.
    Marshalling only."""

    def __init__(self, probs: list, device: str = "cuda:0", stream=None):
        import torch

        self.probs = [lattice_problem(p) for p in probs]
        self.params = [params_from_problem(p) for p in self.probs]
        nbytes = gpe_ensemble_workspace_bytes(self.params)
        if nbytes == 0:
            raise GpeError(GPE_EINVAL, "gpe_ensemble_workspace_bytes")
        self.device = torch.device(device)
        self.ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        self.ws_ptr = (self.ws.data_ptr() + 255) // 256 * 256
        self.ws_bytes = nbytes
        self.stream = stream if stream is not None else torch.cuda.Stream(device=self.device)
        self.e = gpe_ensemble_create(self.params, self.ws_ptr, nbytes, self.stream.cuda_stream)

    @property
    def count(self) -> int:
        return len(self.probs)

    def run(self, n: int):
        gpe_ensemble_run_n(self.e, n)

    def synchronize(self):
        self.stream.synchronize()

    def finite(self) -> np.ndarray:
        return gpe_ensemble_finite(self.e, self.count)

    def autotune(self, trial_steps: int = 10) -> np.ndarray:
        """Pick the tile height per grid size (advances every case by the
        trial steps); returns each case's chosen height."""
        return gpe_ensemble_autotune(self.e, trial_steps, self.count)

    def case(self, i: int) -> EnsembleCase:
        return EnsembleCase(self, i)

    def close(self):
        if getattr(self, "e", None) is not None:
            gpe_ensemble_destroy(self.e)
            self.e = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
