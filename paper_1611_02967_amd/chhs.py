"""Thin ctypes binding of libchhs (C ABI in include/chhs.h).

Argument marshalling only: every computation runs in the HIP library.  Device
buffers are PyTorch CUDA (HIP) tensors, passed by their data pointers; the
stream is torch's current stream unless given.  Functions carry the C names.

The library must have been built (``paper_1611_02967_amd.build.build()``);
importing this module without it raises ImportError -- there is no fallback.
"""
import ctypes
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
# CHHS_LIBRARY selects another build of the same library (kernel variants).
LIB_PATH = os.environ.get("CHHS_LIBRARY") or os.path.join(HERE, "libchhs.so")

CHHS_OK = 0
CHHS_E_INVAL = -1
CHHS_E_NOMEM = -2
CHHS_E_HIP = -3
CHHS_E_NOCONV = -4
CHHS_E_NONFINITE = -5
CHHS_E_STATE = -6


class chhs_problem(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("nz", ctypes.c_int32), ("h", ctypes.c_double), ("eps", ctypes.c_double),
                ("gamma", ctypes.c_double), ("dt", ctypes.c_double)]


class chhs_opts(ctypes.Structure):
    _fields_ = [("nu1", ctypes.c_int32), ("nu2", ctypes.c_int32),
                ("max_vcycles", ctypes.c_int32), ("coarse_sweeps", ctypes.c_int32),
                ("tol", ctypes.c_double), ("precision", ctypes.c_int32),
                ("use_graph", ctypes.c_int32), ("timing", ctypes.c_int32),
                ("smoother", ctypes.c_int32), ("autotune", ctypes.c_int32),
                ("order", ctypes.c_int32), ("tile_threads", ctypes.c_int32),
                ("tile_rows", ctypes.c_int32), ("nu1_coarse", ctypes.c_int32),
                ("nu2_coarse", ctypes.c_int32), ("prolong", ctypes.c_int32),
                ("inner_cycles", ctypes.c_int32)]


K_CLASSES = ["pre0", "post0", "transfer0", "coarse", "norm", "setup", "refine", "k7"]


def timing_mask(*classes):
    """opts.timing value that times only the named kernel classes."""
    m = 0
    for c in classes:
        m |= 1 << (K_CLASSES.index(c) + 1)
    return m


class chhs_timing(ctypes.Structure):
    _fields_ = [("ms", ctypes.c_double * 8), ("launches", ctypes.c_int64 * 8)]


class chhs_stats(ctypes.Structure):
    _fields_ = [("vcycles", ctypes.c_int32), ("status", ctypes.c_int32),
                ("total_vcycles", ctypes.c_int32), ("steps_done", ctypes.c_int32),
                ("res", ctypes.c_double * 3), ("res_norm", ctypes.c_double),
                ("res0", ctypes.c_double), ("mass", ctypes.c_double), ("E_h", ctypes.c_double),
                ("F_h", ctypes.c_double), ("diss_mu", ctypes.c_double),
                ("diss_u", ctypes.c_double), ("max_abs_phi", ctypes.c_double)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["res"] = list(self.res)
        return d


_P = ctypes.c_void_p
_I = ctypes.c_int
_SIGS = {
    "chhs_default_opts": (None, [ctypes.POINTER(chhs_opts)]),
    "chhs_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(chhs_problem), ctypes.c_int32,
                                               ctypes.POINTER(chhs_opts)]),
    "chhs_init": (_I, [ctypes.POINTER(chhs_problem), ctypes.c_int32, ctypes.POINTER(chhs_opts),
                       _P, ctypes.c_size_t, _P, ctypes.POINTER(_P)]),
    "chhs_step": (_I, [_P, _P, _P, _P, _P, ctypes.c_int32, ctypes.POINTER(chhs_stats)]),
    "chhs_step_log": (_I, [_P, _P, _P, _P, _P, ctypes.c_int32, ctypes.POINTER(chhs_stats)]),
    "chhs_setup_step": (_I, [_P, _P, _P, _P, _P]),
    "chhs_fas_vcycle": (_I, [_P, ctypes.POINTER(ctypes.c_double)]),
    "chhs_residual_norms": (_I, [_P, ctypes.POINTER(ctypes.c_double)]),
    "chhs_get_solution": (_I, [_P, _P, _P, _P]),
    "chhs_energy_mass": (_I, [_P, _P, _P, ctypes.POINTER(ctypes.c_double)]),
    "chhs_energy_mass_noalloc": (_I, [ctypes.POINTER(chhs_problem), ctypes.c_int32, _P, _P, _P,
                                      _P]),
    "chhs_level_count": (_I, [_P, ctypes.POINTER(ctypes.c_int32)]),
    "chhs_level_shape": (_I, [_P, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]),
    "chhs_level_kernel": (_I, [_P, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]),
    "chhs_graph_count": (_I, [_P, ctypes.POINTER(ctypes.c_int32)]),
    "chhs_copy_field": (_I, [_P, ctypes.c_int32, ctypes.c_int32, _P, ctypes.c_int32]),
    "chhs_smooth": (_I, [_P, ctypes.c_int32, ctypes.c_int32]),
    "chhs_restrict": (_I, [_P, ctypes.c_int32]),
    "chhs_get_timing": (_I, [_P, ctypes.POINTER(chhs_timing), ctypes.c_int32]),
    "chhs_set_timing": (_I, [_P, ctypes.c_int32]),
    "chhs_tune_sweeps": (_I, [_P, _P, _P, _P, _P, ctypes.POINTER(ctypes.c_int32)]),
    "chhs_get_opts": (_I, [_P, ctypes.POINTER(chhs_opts)]),
    "chhs_destroy": (None, [_P]),
    "chhs_strerror": (ctypes.c_char_p, [_I]),
}


def load_library(path=LIB_PATH):
    """dlopen libchhs.so and declare every exported signature.  The in-tree
    library must have been built from the sources as they are now (its
    recorded digest is compared); a stale build is refused, not run."""
    if not os.path.exists(path):
        raise ImportError(f"libchhs.so is not built ({path}); run paper_1611_02967_amd.build.build()")
    if os.path.abspath(path) == os.path.abspath(os.path.join(HERE, "libchhs.so")):
        from . import build as _build
        if not _build.is_current(path):
            raise ImportError(f"{path} was built from other sources than the current ones; "
                              "rebuild with paper_1611_02967_amd.build.build()")
    lib = ctypes.CDLL(path)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_lib = load_library()


class ChhsError(RuntimeError):
    def __init__(self, code, where):
        self.code = code
        super().__init__(f"{where}: {_lib.chhs_strerror(code).decode()} ({code})")


def _check(code, where):
    if code != CHHS_OK:
        raise ChhsError(code, where)


def _ptr(t):
    if t is None:
        return None
    if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise TypeError("device buffers must be contiguous float64 CUDA/HIP tensors")
    return ctypes.c_void_p(t.data_ptr())


def chhs_default_opts(**overrides):
    o = chhs_opts()
    _lib.chhs_default_opts(ctypes.byref(o))
    for k, v in overrides.items():
        setattr(o, k, v)
    return o


def make_problem(shape, h, eps, gamma, dt):
    """chhs_problem for an array shape (ny, nx) or (nz, ny, nx)."""
    if len(shape) == 2:
        return chhs_problem(2, shape[1], shape[0], 1, h, eps, gamma, dt)
    return chhs_problem(3, shape[2], shape[1], shape[0], h, eps, gamma, dt)


def chhs_workspace_bytes(problems, opts):
    arr = (chhs_problem * len(problems))(*problems)
    return int(_lib.chhs_workspace_bytes(arr, len(problems), ctypes.byref(opts)))


def chhs_init(problems, opts, workspace, stream=None):
    """Returns an opaque context handle; ``workspace`` is a uint8 device tensor."""
    arr = (chhs_problem * len(problems))(*problems)
    handle = ctypes.c_void_p()
    st = torch.cuda.current_stream() if stream is None else stream
    _check(_lib.chhs_init(arr, len(problems), ctypes.byref(opts),
                          ctypes.c_void_p(workspace.data_ptr()), workspace.numel(),
                          ctypes.c_void_p(st.cuda_stream), ctypes.byref(handle)), "chhs_init")
    return handle


def chhs_step(ctx, phi_prev, phi_cur, mu, p, nsteps, n_inst=1, check=True):
    stats = (chhs_stats * n_inst)()
    rc = _lib.chhs_step(ctx, _ptr(phi_prev), _ptr(phi_cur), _ptr(mu), _ptr(p), nsteps, stats)
    if check:
        _check(rc, "chhs_step")
    return rc, [s.as_dict() for s in stats]


def chhs_step_log(ctx, phi_prev, phi_cur, mu, p, nsteps, n_inst=1, check=True):
    """Steps with every step's statistics: a list over steps of lists over instances."""
    recs = (chhs_stats * max(1, nsteps * n_inst))()
    rc = _lib.chhs_step_log(ctx, _ptr(phi_prev), _ptr(phi_cur), _ptr(mu), _ptr(p), nsteps, recs)
    if check:
        _check(rc, "chhs_step_log")
    return rc, [[recs[m * n_inst + i].as_dict() for i in range(n_inst)] for m in range(nsteps)]


def chhs_setup_step(ctx, phi_prev, phi_cur, mu, p):
    _check(_lib.chhs_setup_step(ctx, _ptr(phi_prev), _ptr(phi_cur), _ptr(mu), _ptr(p)),
           "chhs_setup_step")


def chhs_fas_vcycle(ctx, n_inst=1):
    out = (ctypes.c_double * n_inst)()
    _check(_lib.chhs_fas_vcycle(ctx, out), "chhs_fas_vcycle")
    return list(out)


def chhs_residual_norms(ctx, n_inst=1):
    out = (ctypes.c_double * (4 * n_inst))()
    _check(_lib.chhs_residual_norms(ctx, out), "chhs_residual_norms")
    return [list(out[4 * i:4 * i + 4]) for i in range(n_inst)]


def chhs_get_solution(ctx, phi=None, mu=None, p=None):
    _check(_lib.chhs_get_solution(ctx, _ptr(phi), _ptr(mu), _ptr(p)), "chhs_get_solution")


def chhs_energy_mass(ctx, phi, phi_prev, n_inst=1):
    out = (ctypes.c_double * (3 * n_inst))()
    _check(_lib.chhs_energy_mass(ctx, _ptr(phi), _ptr(phi_prev), out), "chhs_energy_mass")
    return [list(out[3 * i:3 * i + 3]) for i in range(n_inst)]


def chhs_energy_mass_noalloc(problems, phi, phi_prev, out, stream=None):
    """Enqueues mass, E_h, F_h of every instance into ``out`` (a float64 device
    tensor of 3 * len(problems) values) on ``stream`` (torch's current stream
    by default); allocates nothing."""
    arr = (chhs_problem * len(problems))(*problems)
    st = torch.cuda.current_stream() if stream is None else stream
    _check(_lib.chhs_energy_mass_noalloc(arr, len(problems), _ptr(phi), _ptr(phi_prev), _ptr(out),
                                         ctypes.c_void_p(st.cuda_stream)),
           "chhs_energy_mass_noalloc")


def chhs_level_count(ctx):
    n = ctypes.c_int32()
    _check(_lib.chhs_level_count(ctx, ctypes.byref(n)), "chhs_level_count")
    return n.value


KERNEL_KINDS = ["tiles", "strips", "per-cell", "tail", "zmarch"]


def chhs_level_kernel(ctx, level):
    """(kind, threads per block | rows per segment, blocks per launch) of a level."""
    out = (ctypes.c_int32 * 3)()
    _check(_lib.chhs_level_kernel(ctx, level, out), "chhs_level_kernel")
    return KERNEL_KINDS[out[0]], out[1], out[2]


def chhs_graph_count(ctx):
    """Number of captured cycle graphs (0 when cycles launch directly)."""
    out = ctypes.c_int32(0)
    _check(_lib.chhs_graph_count(ctx, ctypes.byref(out)), "chhs_graph_count")
    return out.value


def chhs_level_shape(ctx, level):
    out = (ctypes.c_int32 * 3)()
    _check(_lib.chhs_level_shape(ctx, level, out), "chhs_level_shape")
    return tuple(out)


def chhs_copy_field(ctx, level, field, dev, direction):
    _check(_lib.chhs_copy_field(ctx, level, field, _ptr(dev), direction), "chhs_copy_field")


def chhs_smooth(ctx, level, nsweeps=1):
    _check(_lib.chhs_smooth(ctx, level, nsweeps), "chhs_smooth")


def chhs_restrict(ctx, level):
    _check(_lib.chhs_restrict(ctx, level), "chhs_restrict")


def chhs_get_timing(ctx, reset=False):
    """{class: (total ms, launches)} of the event-timed kernel classes."""
    t = chhs_timing()
    _check(_lib.chhs_get_timing(ctx, ctypes.byref(t), 1 if reset else 0), "chhs_get_timing")
    return {K_CLASSES[k]: (t.ms[k], t.launches[k]) for k in range(8)}


def chhs_set_timing(ctx, timing):
    """Replaces opts.timing from the next launch on."""
    _check(_lib.chhs_set_timing(ctx, int(timing)), "chhs_set_timing")


def chhs_tune_sweeps(ctx, phi_prev, phi_cur, mu, p):
    """Sweeps per level, prolongation and (mixed precision) FP32 cycles per
    refinement chosen by time to tolerance; returns the kept (nu1, nu2,
    nu1_coarse, nu2_coarse, prolong, inner_cycles)."""
    out = (ctypes.c_int32 * 6)()
    _check(_lib.chhs_tune_sweeps(ctx, _ptr(phi_prev), _ptr(phi_cur), _ptr(mu), _ptr(p), out),
           "chhs_tune_sweeps")
    return tuple(out)


def chhs_get_opts(ctx):
    o = chhs_opts()
    _check(_lib.chhs_get_opts(ctx, ctypes.byref(o)), "chhs_get_opts")
    return o


def chhs_destroy(ctx):
    _lib.chhs_destroy(ctx)


def chhs_strerror(code):
    return _lib.chhs_strerror(code).decode()


FIELDS = {"phi": 0, "mu": 1, "p": 2, "f_phi": 3, "f_mu": 4, "f_p": 5, "phi_star": 6, "psi": 7}


class Solver:
    """Owns a workspace tensor and a context; marshals arrays to the C calls."""

    def __init__(self, problems, opts=None, device="cuda", stream=None):
        if not isinstance(problems, (list, tuple)):
            problems = [problems]
        self.problems = list(problems)
        self.n_inst = len(self.problems)
        self.opts = opts if opts is not None else chhs_default_opts()
        nbytes = chhs_workspace_bytes(self.problems, self.opts)
        if nbytes == 0:
            raise ChhsError(CHHS_E_INVAL, "chhs_workspace_bytes")
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=device)
        self.stream = torch.cuda.current_stream() if stream is None else stream
        self.ctx = chhs_init(self.problems, self.opts, self.workspace, self.stream)
        # packed cells of all instances: the length of every state array
        self.cells = sum(int(q.nx) * int(q.ny) * int(q.nz) for q in self.problems)

    def _check_arrays(self, *ts):
        """Every array must hold the packed cells of all instances and live on
        the workspace's device (the kernels index it up to that length)."""
        for t in ts:
            if t is None:
                continue
            if t.device != self.workspace.device:
                raise ValueError(f"array on {t.device}, workspace on {self.workspace.device}")
            if t.numel() != self.cells:
                raise ValueError(f"array holds {t.numel()} values, the instances {self.cells} cells")

    def close(self):
        if self.ctx is not None:
            chhs_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, phi_prev, phi_cur, mu, p, nsteps=1, check=True):
        self._check_arrays(phi_prev, phi_cur, mu, p)
        return chhs_step(self.ctx, phi_prev, phi_cur, mu, p, nsteps, self.n_inst, check)

    def step_log(self, phi_prev, phi_cur, mu, p, nsteps=1, check=True):
        self._check_arrays(phi_prev, phi_cur, mu, p)
        return chhs_step_log(self.ctx, phi_prev, phi_cur, mu, p, nsteps, self.n_inst, check)

    def setup_step(self, phi_prev, phi_cur, mu, p):
        self._check_arrays(phi_prev, phi_cur, mu, p)
        chhs_setup_step(self.ctx, phi_prev, phi_cur, mu, p)

    def fas_vcycle(self):
        return chhs_fas_vcycle(self.ctx, self.n_inst)

    def residual_norms(self):
        return chhs_residual_norms(self.ctx, self.n_inst)

    def get_solution(self, phi=None, mu=None, p=None):
        self._check_arrays(phi, mu, p)
        chhs_get_solution(self.ctx, phi, mu, p)

    def energy_mass(self, phi, phi_prev):
        self._check_arrays(phi, phi_prev)
        return chhs_energy_mass(self.ctx, phi, phi_prev, self.n_inst)

    def tune_sweeps(self, phi_prev, phi_cur, mu, p):
        self._check_arrays(phi_prev, phi_cur, mu, p)
        return chhs_tune_sweeps(self.ctx, phi_prev, phi_cur, mu, p)

    def get_opts(self):
        return chhs_get_opts(self.ctx)

    def timing(self, reset=False):
        return chhs_get_timing(self.ctx, reset)

    def set_timing(self, timing):
        chhs_set_timing(self.ctx, timing)

    def level_kernels(self):
        """Per level of the batch: (kind, parameter, blocks) as chhs_level_kernel."""
        out = []
        level = 0
        while True:
            try:
                out.append(chhs_level_kernel(self.ctx, level))
            except ChhsError:
                return out
            level += 1

    def graph_count(self):
        return chhs_graph_count(self.ctx)

    def levels(self):
        return [chhs_level_shape(self.ctx, l) for l in range(chhs_level_count(self.ctx))]

    def read_field(self, level, name):
        nx, ny, nz = chhs_level_shape(self.ctx, level)
        shape = (ny, nx) if self.problems[0].dim == 2 else (nz, ny, nx)
        out = torch.empty(shape, dtype=torch.float64, device=self.workspace.device)
        chhs_copy_field(self.ctx, level, FIELDS[name], out, 0)
        return out

    def write_field(self, level, name, value):
        value = value.to(device=self.workspace.device, dtype=torch.float64).contiguous()
        chhs_copy_field(self.ctx, level, FIELDS[name], value, 1)

    def smooth(self, level, nsweeps=1):
        chhs_smooth(self.ctx, level, nsweeps)

    def restrict(self, level):
        chhs_restrict(self.ctx, level)
