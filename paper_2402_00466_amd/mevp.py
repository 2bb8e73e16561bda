"""Python binding of the C ABI in include/mevp.h (argument marshalling only).

Every step of the mEVP subcycle runs in the HIP kernels of ``libmevp.so``;
this module checks tensor shapes, dtypes and devices, passes raw device
pointers and the current HIP stream, and turns status codes into exceptions.
PyTorch supplies device memory (the workspace and the input/output tensors)
and the stream. There is no fallback: if the library is missing, loading
fails with an error.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, asdict, field

from . import build as _build

FP64 = 0
MIXED = 1
MIXED_BF16 = 2  # mixed precision with bfloat16 element matrices (a trial; see mevp.h)
STRATEGIES = {"fused": 0, "two_phase": 1, "persistent": 2, "fused_pair": 3,
              "fused_triple": 4}
STRATEGY_NAMES = {v: k for k, v in STRATEGIES.items()}
TILES = [(16, 14), (16, 16), (32, 15), (13, 13)]
_PREC = {"fp64": FP64, "f64": FP64, "mixed": MIXED, "mixed_bf16": MIXED_BF16}

STATUS = {0: "MEVP_OK", -1: "MEVP_EINVAL", -2: "MEVP_ENOMEM", -3: "MEVP_EDEVICE",
          -4: "MEVP_ESTATE", -5: "MEVP_ENONFINITE", -6: "MEVP_EUNSUPPORTED", -7: "MEVP_EINTERNAL",
          -8: "MEVP_EHOSTMEM"}


class MevpError(RuntimeError):
    def __init__(self, func: str, status: int):
        self.status = status
        self.func = func
        super().__init__(f"{func} failed: {STATUS.get(status, status)} "
                         f"({_lib_msg(status)})")


class CParams(C.Structure):
    _fields_ = [(n, C.c_double) for n in ("Pstar", "C", "DeltaMin", "alpha", "beta", "rho_i",
                                          "rho_a", "C_a", "rho_o", "C_o", "f_cor", "dt")] + \
               [("relax_form", C.c_int)]


class CConfig(C.Structure):
    _fields_ = [("strategy", C.c_int), ("tile_nx", C.c_int), ("tile_ny", C.c_int)]


class CDomain(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("n_s", C.c_int), ("n_a", C.c_int)]


_lib = None

EXPORTS = ["mevp_default_params", "mevp_workspace_size", "mevp_create", "mevp_set_strategy",
           "mevp_set_config", "mevp_get_config", "mevp_get_launch_depth", "mevp_set_graph", "mevp_tune",
           "mevp_advect", "mevp_get_fields",
           "mevp_set_params",
           "mevp_set_geometry", "mevp_set_geometry_cg2", "mevp_set_fields", "mevp_set_forcing",
           "mevp_set_state",
           "mevp_step", "mevp_begin_step", "mevp_subcycles", "mevp_get_state", "mevp_sync",
           "mevp_check_inputs", "mevp_check_state", "mevp_timing_enable", "mevp_timing_read",
           "mevp_step_static",
           "mevp_destroy", "mevp_status_string", "mevp_version"]

# bytes of the device array mevp_step_static works in (MEVP_STATIC_SCRATCH_BYTES)
STATIC_SCRATCH_BYTES = 64 << 20


def lib_path() -> str:
    return _build.LIB


def lib():
    """Load libmevp.so (built by paper_2402_00466_amd/build.py). Raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    path = lib_path()
    if not os.path.exists(path):
        raise RuntimeError(f"HIP library not built: {path} is missing "
                           "(run python -m paper_2402_00466_amd.build)")
    L = C.CDLL(path)
    vp, dp, i = C.c_void_p, C.c_void_p, C.c_int
    L.mevp_default_params.argtypes = [C.POINTER(CParams)]
    L.mevp_workspace_size.argtypes = [C.POINTER(CDomain), i, i, C.POINTER(C.c_size_t)]
    L.mevp_create.argtypes = [C.POINTER(CParams), i, C.POINTER(CDomain), i, vp, C.c_size_t, vp,
                              C.POINTER(vp)]
    L.mevp_set_params.argtypes = [vp, C.POINTER(CParams)]
    L.mevp_set_strategy.argtypes = [vp, i]
    L.mevp_set_config.argtypes = [vp, C.POINTER(CConfig)]
    L.mevp_set_graph.argtypes = [vp, i]
    L.mevp_tune.argtypes = [vp, i, C.c_char_p, C.POINTER(CConfig)]
    L.mevp_advect.argtypes = [vp]
    L.mevp_get_fields.argtypes = [vp, i, dp, dp]
    L.mevp_get_config.argtypes = [vp, C.POINTER(CConfig)]
    L.mevp_get_launch_depth.argtypes = [vp, C.POINTER(C.c_int)]
    L.mevp_set_geometry.argtypes = [vp, i, dp]
    L.mevp_set_geometry_cg2.argtypes = [vp, i, dp]
    L.mevp_set_fields.argtypes = [vp, i, dp, dp]
    L.mevp_set_forcing.argtypes = [vp, i, dp, dp]
    L.mevp_set_state.argtypes = [vp, i, dp, dp]
    L.mevp_step.argtypes = [vp, i]
    L.mevp_begin_step.argtypes = [vp]
    L.mevp_subcycles.argtypes = [vp, i]
    L.mevp_get_state.argtypes = [vp, i, dp, dp]
    L.mevp_sync.argtypes = [vp]
    L.mevp_check_inputs.argtypes = [vp]
    L.mevp_check_state.argtypes = [vp]
    L.mevp_timing_enable.argtypes = [vp, i]
    L.mevp_timing_read.argtypes = [vp, C.POINTER(C.c_int), C.POINTER(C.c_double)]
    L.mevp_step_static.argtypes = [C.POINTER(CParams), i, C.POINTER(CDomain), dp, dp, dp, dp, dp,
                                   dp, dp, i, vp]
    L.mevp_destroy.argtypes = [vp]
    L.mevp_status_string.argtypes = [i]
    L.mevp_version.argtypes = []
    for name in EXPORTS:
        getattr(L, name).restype = C.c_int
    L.mevp_destroy.restype = None
    L.mevp_status_string.restype = C.c_char_p
    L.mevp_version.restype = C.c_char_p
    _lib = L
    return L


def _lib_msg(status: int) -> str:
    try:
        return lib().mevp_status_string(status).decode()
    except Exception:  # pragma: no cover - only reached while reporting another error
        return "?"


def _check(func: str, status: int):
    if status != 0:
        raise MevpError(func, status)


@dataclass
class Params:
    """mevp_params; defaults are mevp_default_params (P* = 27500 N/m^2 and the
    factor 20 of the stress listings, alpha = beta = 300, 100 subcycles per
    120 s step of the paper's Sec. 4)."""
    Pstar: float = 27500.0
    C: float = 20.0
    DeltaMin: float = 2e-9
    alpha: float = 300.0
    beta: float = 300.0
    rho_i: float = 900.0
    rho_a: float = 1.3
    C_a: float = 1.2e-3
    rho_o: float = 1026.0
    C_o: float = 5.5e-3
    f_cor: float = 1.46e-4
    dt: float = 120.0
    relax_form: int = 0

    def to_c(self) -> CParams:
        return CParams(**asdict(self))


@dataclass
class Domain:
    nx: int
    ny: int
    n_s: int = 6
    n_a: int = 1

    @property
    def ne(self):
        return self.nx * self.ny

    @property
    def nn(self):
        return (2 * self.nx + 1) * (2 * self.ny + 1)

    @property
    def nv(self):
        return (self.nx + 1) * (self.ny + 1)


def default_params() -> Params:
    cp = CParams()
    _check("mevp_default_params", lib().mevp_default_params(C.byref(cp)))
    return Params(**{n: getattr(cp, n) for n, _ in CParams._fields_})


def _domains_c(domains):
    arr = (CDomain * len(domains))()
    for k, d in enumerate(domains):
        arr[k] = CDomain(int(d.nx), int(d.ny), int(d.n_s), int(d.n_a))
    return arr


def workspace_size(domains, precision="fp64") -> int:
    out = C.c_size_t(0)
    _check("mevp_workspace_size",
           lib().mevp_workspace_size(_domains_c(domains), len(domains), _PREC[precision],
                                     C.byref(out)))
    return out.value


def step_static(domain, vertices, H, A, wind, ocean, v, S, n_subcycles: int,
                params: Params | None = None, precision: str = "fp64", stream=None):
    """One time step of one domain through mevp_step_static (no context, no
    workspace, nothing allocated by the library). Every array is a contiguous
    float64 tensor on the current device in the layouts of mevp.h; v and S
    hold the state and are overwritten with the state after the step
    (stream-ordered on ``stream``, default: the current torch stream)."""
    import torch
    d = domain if isinstance(domain, Domain) else Domain(*domain)
    dev = torch.device("cuda", torch.cuda.current_device())
    shapes = {"vertices": (vertices, (2, d.nv)), "H": (H, (d.n_a, d.ne)), "A": (A, (d.n_a, d.ne)),
              "wind": (wind, (2, d.nn)), "ocean": (ocean, (2, d.nn)), "v": (v, (2, d.nn)),
              "S": (S, (3, d.n_s, d.ne))}
    ptrs = []
    for name, (t, shape) in shapes.items():
        if not isinstance(t, torch.Tensor) or t.device != dev or t.dtype != torch.float64:
            raise ValueError(f"{name} must be a float64 tensor on {dev}")
        if tuple(t.shape) != shape or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous tensor of shape {shape}")
        ptrs.append(C.c_void_p(t.data_ptr()))
    stream = stream if stream is not None else torch.cuda.current_stream(dev)
    dc = CDomain(int(d.nx), int(d.ny), int(d.n_s), int(d.n_a))
    _check("mevp_step_static", lib().mevp_step_static(
        C.byref((params or Params()).to_c()), _PREC[precision], C.byref(dc), *ptrs,
        int(n_subcycles), C.c_void_p(stream.cuda_stream)))


class Context:
    """One mevp context: its workspace is a torch uint8 tensor on the current
    device, its stream the current torch stream at creation."""

    def __init__(self, domains, params: Params | None = None, precision: str = "fp64",
                 stream=None, strategy: str = "fused"):
        import torch
        self._torch = torch
        self.domains = [d if isinstance(d, Domain) else Domain(*d) for d in domains]
        self.params = params or Params()
        self.precision = precision
        size = workspace_size(self.domains, precision)
        self.device = torch.device("cuda", torch.cuda.current_device())
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        raw = torch.empty(size + 256, dtype=torch.uint8, device=self.device)
        pad = (-raw.data_ptr()) % 256
        self._raw = raw
        self.workspace = raw[pad:pad + size]
        h = C.c_void_p()
        _check("mevp_create", lib().mevp_create(
            C.byref(self.params.to_c()), _PREC[precision], _domains_c(self.domains),
            len(self.domains), C.c_void_p(self.workspace.data_ptr()), C.c_size_t(size),
            C.c_void_p(self.stream.cuda_stream), C.byref(h)))
        self._h = h
        self.set_strategy(strategy)

    # -- helpers --------------------------------------------------------
    def _arg(self, t, shape, name):
        torch = self._torch
        if not isinstance(t, torch.Tensor):
            raise TypeError(f"{name} must be a torch tensor")
        if t.device != self.device or t.dtype != torch.float64:
            raise ValueError(f"{name} must be float64 on {self.device}, got {t.dtype} on {t.device}")
        if tuple(t.shape) != tuple(shape) or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous tensor of shape {tuple(shape)}, "
                             f"got {tuple(t.shape)}")
        return C.c_void_p(t.data_ptr())

    def _dom(self, dom):
        if not 0 <= dom < len(self.domains):
            raise IndexError(dom)
        return self.domains[dom]

    # -- copy-in --------------------------------------------------------
    def set_strategy(self, strategy: str):
        _check("mevp_set_strategy", lib().mevp_set_strategy(self._h, STRATEGIES[strategy]))
        self.strategy = strategy

    def set_config(self, strategy: str, tile=(16, 14)):
        cfg = CConfig(STRATEGIES[strategy], int(tile[0]), int(tile[1]))
        _check("mevp_set_config", lib().mevp_set_config(self._h, C.byref(cfg)))
        self.strategy = strategy

    def set_graph(self, enable: bool):
        _check("mevp_set_graph", lib().mevp_set_graph(self._h, int(bool(enable))))

    def tune(self, n_trial: int = 20, cache_path: str | None = None):
        """Autotune the launch configuration (see mevp_tune); returns (strategy, tile)."""
        cfg = CConfig()
        path = cache_path.encode() if cache_path else None
        _check("mevp_tune", lib().mevp_tune(self._h, int(n_trial), path, C.byref(cfg)))
        self.strategy = STRATEGY_NAMES[cfg.strategy]
        return STRATEGY_NAMES[cfg.strategy], (cfg.tile_nx, cfg.tile_ny)

    def get_config(self):
        cfg = CConfig()
        _check("mevp_get_config", lib().mevp_get_config(self._h, C.byref(cfg)))
        return STRATEGY_NAMES[cfg.strategy], (cfg.tile_nx, cfg.tile_ny)

    def launch_depth(self) -> int:
        """Subcycles per launch of the current configuration (see mevp_get_launch_depth;
        0: all subcycles of a call in one persistent launch)."""
        k = C.c_int()
        _check("mevp_get_launch_depth", lib().mevp_get_launch_depth(self._h, C.byref(k)))
        return k.value

    def set_params(self, params: Params):
        _check("mevp_set_params", lib().mevp_set_params(self._h, C.byref(params.to_c())))
        self.params = params

    def set_geometry(self, dom, vertices):
        d = self._dom(dom)
        _check("mevp_set_geometry", lib().mevp_set_geometry(
            self._h, dom, self._arg(vertices, (2, d.nv), "vertices")))

    def set_geometry_cg2(self, dom, nodes):
        """Curved cells: CG2 node positions [2][(2nx+1)(2ny+1)] (isoparametric map)."""
        d = self._dom(dom)
        _check("mevp_set_geometry_cg2", lib().mevp_set_geometry_cg2(
            self._h, dom, self._arg(nodes, (2, d.nn), "nodes")))

    def set_fields(self, dom, H, A):
        d = self._dom(dom)
        _check("mevp_set_fields", lib().mevp_set_fields(
            self._h, dom, self._arg(H, (d.n_a, d.ne), "H"), self._arg(A, (d.n_a, d.ne), "A")))

    def set_forcing(self, dom, wind, ocean):
        d = self._dom(dom)
        _check("mevp_set_forcing", lib().mevp_set_forcing(
            self._h, dom, self._arg(wind, (2, d.nn), "wind"), self._arg(ocean, (2, d.nn), "ocean")))

    def set_state(self, dom, v, S):
        d = self._dom(dom)
        _check("mevp_set_state", lib().mevp_set_state(
            self._h, dom, self._arg(v, (2, d.nn), "v"), self._arg(S, (3, d.n_s, d.ne), "S")))

    # -- stepping -------------------------------------------------------
    def step(self, n_subcycles: int):
        _check("mevp_step", lib().mevp_step(self._h, int(n_subcycles)))

    def begin_step(self):
        _check("mevp_begin_step", lib().mevp_begin_step(self._h))

    def subcycles(self, n: int):
        _check("mevp_subcycles", lib().mevp_subcycles(self._h, int(n)))

    def advect(self):
        """Advect H and A of every domain over one step (mevp_advect)."""
        _check("mevp_advect", lib().mevp_advect(self._h))

    # -- copy-out -------------------------------------------------------
    def get_fields(self, dom):
        torch = self._torch
        d = self._dom(dom)
        H = torch.empty((d.n_a, d.ne), dtype=torch.float64, device=self.device)
        A = torch.empty((d.n_a, d.ne), dtype=torch.float64, device=self.device)
        _check("mevp_get_fields", lib().mevp_get_fields(
            self._h, dom, C.c_void_p(H.data_ptr()), C.c_void_p(A.data_ptr())))
        return H, A

    def get_state(self, dom):
        torch = self._torch
        d = self._dom(dom)
        v = torch.empty((2, d.nn), dtype=torch.float64, device=self.device)
        S = torch.empty((3, d.n_s, d.ne), dtype=torch.float64, device=self.device)
        _check("mevp_get_state", lib().mevp_get_state(
            self._h, dom, C.c_void_p(v.data_ptr()), C.c_void_p(S.data_ptr())))
        return v, S

    def sync(self):
        _check("mevp_sync", lib().mevp_sync(self._h))

    def check_inputs(self):
        _check("mevp_check_inputs", lib().mevp_check_inputs(self._h))

    def check_state(self):
        _check("mevp_check_state", lib().mevp_check_state(self._h))

    def timing_enable(self, max_launches: int):
        _check("mevp_timing_enable", lib().mevp_timing_enable(self._h, int(max_launches)))

    def timing_read(self):
        """{phase: (launches, total ms)} for phases element, node, begin_step."""
        cnt = (C.c_int * 3)()
        ms = (C.c_double * 3)()
        _check("mevp_timing_read", lib().mevp_timing_read(self._h, cnt, ms))
        return {name: (cnt[k], ms[k]) for k, name in enumerate(("element", "node", "begin_step"))}

    def close(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.mevp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- convenience: upload a generated domain --------------------------
    def upload(self, dom, inputs):
        """Copy a synth_inputs.DomainInputs-like object (numpy arrays) to the device and
        set geometry, fields and forcing of domain ``dom``."""
        torch = self._torch
        dev = self.device
        t = lambda a: torch.as_tensor(a, dtype=torch.float64).contiguous().to(dev)
        nodes = getattr(inputs, "nodes", None)
        if nodes is not None:
            self.set_geometry_cg2(dom, t(nodes))
        else:
            self.set_geometry(dom, t(inputs.vertices))
        self.set_fields(dom, t(inputs.H), t(inputs.A))
        self.set_forcing(dom, t(inputs.wind), t(inputs.ocean))
