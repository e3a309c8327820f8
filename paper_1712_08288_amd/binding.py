"""Python binding of the C ABI in include/lbm.h (argument marshalling only).

Every computation runs in the HIP library `_lib/liblbm.so`; importing this
module fails loudly when the library has not been built.  Host arrays are
numpy; device buffers (state snapshots) may be torch tensors, of which only
the data pointer is used.
"""

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# LBM_LIBRARY may point at another build of the same sources (A/B timing)
LIB_PATH = os.environ.get("LBM_LIBRARY") or os.path.join(_HERE, "_lib", "liblbm.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        "HIP engine library %s is missing; build it with "
        "`python -m paper_1712_08288_amd.build`" % LIB_PATH)

_lib = C.CDLL(LIB_PATH)

_p = C.c_void_p
_i = C.c_int
_i32 = C.c_int32
_i64 = C.c_int64
_d = C.c_double
_dp = C.POINTER(C.c_double)


def _sig(name, res, args):
    f = getattr(_lib, name)
    f.restype = res
    f.argtypes = args
    return f


_create = _sig("lbm_create", _i, [C.POINTER(_p), _i, _i, _i64, _i64, _i64, _dp, _d, _dp])
_set_scheme = _sig("lbm_set_scheme", _i, [_p, _i, _d])
_set_xbc = _sig("lbm_set_x_boundary", _i, [_p, _i, _d])
_set_two_node = _sig("lbm_set_two_node", _i, [_p, _i])
_set_wall_decay = _sig("lbm_set_wall_decay", _i, [_p, C.c_double])
_adj_step = _sig("lbm_adjoint_step", _i, [_p, C.c_int64])
_adj_remaining = _sig("lbm_adjoint_remaining", C.c_int64, [_p])
_set_geometry = _sig("lbm_set_geometry", _i, [_p, _p, _i64, _p, _p, _p, _p, _p])
_update_links = _sig("lbm_update_links", _i, [_p, _p, _p])
_set_params = _sig("lbm_set_parameters", _i, [_p, _p, _p])
_coll_rates = _sig("lbm_collision_rates", _i, [_i, _i, _d, _d, _p])
_set_collision = _sig("lbm_set_collision", _i, [_p, _i, _d, _d])
_init = _sig("lbm_init", _i, [_p, _p, _p])
_init_dev = _sig("lbm_init_deviation", _i, [_p, _p])
_step = _sig("lbm_step", _i, [_p, _i64])
_time = _sig("lbm_time", _i64, [_p])
_moments = _sig("lbm_moments", _i, [_p, _p, _p])
_get_dist = _sig("lbm_get_distribution", _i, [_p, _p])
_reduce = _sig("lbm_reduce", _i, [_p, _p, _p])
_reduce_noalloc = _sig("lbm_reduce_noalloc", _i, [_p, _p, _p])
_force = _sig("lbm_force", _i, [_p, _i32, _p])
_state_bytes = _sig("lbm_state_bytes", _i64, [_p])
_get_state = _sig("lbm_get_state", _i, [_p, _p])
_set_state = _sig("lbm_set_state", _i, [_p, _p, _i64])
_set_obj = _sig("lbm_set_objective", _i, [_p, _i, _i32, _i64, _i64])
_objective = _sig("lbm_objective", _i, [_p, _p])
_set_obj_planes = _sig("lbm_set_objective_planes", _i, [_p, _i64, _i64])
_pressure_drop = _sig("lbm_pressure_drop", _i, [_p, _i64, _i64, _p])
_run_ckpt = _sig("lbm_run_checkpointed", _i, [_p, _i64, _i64])
_adjoint = _sig("lbm_adjoint", _i, [_p])
_grad = _sig("lbm_grad", _i, [_p, _p, _p, _p, _p])
_grad_dev = _sig("lbm_grad_device", _i, [_p, _p, _p, _p, _p])
_set_rate_grad = _sig("lbm_set_rate_gradient", _i, [_p, _i])
_get_adj = _sig("lbm_get_adjoint", _i, [_p, _p])
_set_stream = _sig("lbm_set_stream", _i, [_p, _p])
_lat_info = _sig("lbm_lattice_info", _i, [_i, _p, _p, _p, _p, _p])
_counts = _sig("lbm_counts", _i, [_p, _p, _p])
_set_timing = _sig("lbm_set_timing", _i, [_p, _i])
_last_ms = _sig("lbm_last_step_ms", _i, [_p, _p])
_stream_copy = _sig("lbm_stream_copy", _i, [_p, _p, _i64, _i32, _i32, _p])
_pull_pattern = _sig("lbm_pull_pattern_copy", _i, [_i, _i, _p, _p, _i64, _i64, _i64, _i32, _p])
_adj_pattern = _sig("lbm_adjoint_pattern_copy", _i, [_i, _i, _p, _p, _p, _i64, _i64, _i64, _i32, _p])
_aa_pattern = _sig("lbm_aa_pattern_copy", _i, [_i, _i, _p, _i64, _i64, _i64, _i32, _p, _p])
_blocked_pattern = _sig("lbm_blocked_pull_pattern_copy", _i,
                        [_i, _i, _i32, _p, _p, _i64, _i64, _i64, _i32, _p])
_last_err = _sig("lbm_last_error", C.c_char_p, [_p])
_destroy = _sig("lbm_destroy", _i, [_p])

EXPORTED = ["lbm_create", "lbm_set_scheme", "lbm_set_two_node", "lbm_set_wall_decay",
            "lbm_set_x_boundary",
            "lbm_set_geometry", "lbm_update_links", "lbm_set_parameters",
            "lbm_collision_rates", "lbm_set_collision", "lbm_init",
            "lbm_init_deviation", "lbm_step", "lbm_time", "lbm_moments",
            "lbm_get_distribution", "lbm_reduce", "lbm_reduce_noalloc", "lbm_force",
            "lbm_state_bytes", "lbm_get_state", "lbm_set_state",
            "lbm_set_objective", "lbm_set_objective_planes", "lbm_pressure_drop",
            "lbm_objective", "lbm_run_checkpointed",
            "lbm_adjoint", "lbm_adjoint_step", "lbm_adjoint_remaining", "lbm_set_rate_gradient", "lbm_grad", "lbm_grad_device", "lbm_get_adjoint", "lbm_set_stream",
            "lbm_lattice_info", "lbm_counts", "lbm_set_timing",
            "lbm_last_step_ms", "lbm_last_error", "lbm_destroy"]
# measurement probes (include/lbm_probe.h)
EXPORTED_PROBES = ["lbm_stream_copy", "lbm_pull_pattern_copy", "lbm_adjoint_pattern_copy",
                   "lbm_aa_pattern_copy", "lbm_blocked_pull_pattern_copy"]

LATTICES = {"D2Q9": 0, "D3Q19": 1, "D3Q15": 2}
PRECISIONS = {"fp64": 0, "fp32": 1}
RULES = {"gamma": 0, "1.5gamma": 1, "2gamma": 2, "gamma2": 3,
         "gamma2+gamma": 4, "zero": 5, "min": 6}
X_BC = {"periodic": 0, "pressure": 1, "outflow": 2}
OBJECTIVES = {"none": 0, "force_x": 1, "mean_ux": 2, "pressure_drop": 3}
ERRORS = {-1: "EINVAL", -2: "EGEOM", -3: "ESTATE", -4: "ENOMEM",
          -5: "EDEVICE", -6: "ENONFINITE"}


class LBMError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (%d): %s" % (ERRORS.get(code, "?"), code, msg))
        self.code = code
        self.name = ERRORS.get(code, "?")


def _ptr(a):
    return None if a is None else a.ctypes.data_as(_p)


def _f64(a, n=None):
    if a is None:
        return None
    a = np.ascontiguousarray(a, dtype=np.float64)
    if n is not None and a.size != n:
        raise ValueError("expected %d values, got %d" % (n, a.size))
    return a


def lattice_info(lattice):
    lat = LATTICES[lattice]
    Q, D = _i32(), _i32()
    _lat_info(lat, C.byref(Q), C.byref(D), None, None, None)
    e = np.zeros((Q.value, D.value), np.int8)
    w = np.zeros(Q.value)
    M = np.zeros((Q.value, Q.value))
    rc = _lat_info(lat, None, None, _ptr(e), _ptr(w), _ptr(M))
    if rc:
        raise LBMError(rc, "lattice_info")
    return e.astype(np.int64), w, M


COLLISIONS = {"bgk": 1, "trt": 2}


def collision_rates(lattice, kind, s_nu, magic=3.0 / 16.0):
    """MRT rates that realise the BGK or TRT operator (lbm_collision_rates;
    Remark (1): the boundary scheme does not depend on the collision)."""
    e, _, _ = lattice_info(lattice)
    s = np.zeros(len(e))
    rc = _coll_rates(LATTICES[lattice], COLLISIONS[kind], float(s_nu), float(magic), _ptr(s))
    if rc:
        raise LBMError(rc, "collision_rates")
    return s


def stream_copy(dst, src, nbytes, mode=0, reps=10):
    """Time a plain device copy of nbytes (the practical HBM ceiling);
    dst/src: torch tensors or device pointers.  Returns ms per copy."""
    d = dst.data_ptr() if hasattr(dst, "data_ptr") else int(dst)
    s = src.data_ptr() if hasattr(src, "data_ptr") else int(src)
    ms = np.zeros(1)
    rc = _stream_copy(_p(d), _p(s), int(nbytes), int(mode), int(reps), _ptr(ms))
    if rc:
        raise LBMError(rc, "stream_copy")
    return float(ms[0])


# Nodes per block of the population arrays: population i of node n is
# element (n // B) * Q * B + i * B + n % B.
POPULATION_BLOCK = 2048


def population_elements(lattice, shape):
    """Elements of one population array (distributions or adjoint) of this
    lattice on an nx x ny x nz grid: Q * nx*ny*nz rounded up to whole
    blocks of POPULATION_BLOCK nodes."""
    Q = {"D2Q9": 9, "D3Q15": 15, "D3Q19": 19}[lattice]
    n = int(np.prod((tuple(shape) + (1, 1))[:3]))
    return Q * (-(-n // POPULATION_BLOCK) * POPULATION_BLOCK)


def population_index(lattice, shape):
    """Index array (Q, nx*ny*nz) of the element that holds population i of
    node n in the blocked layout."""
    Q = {"D2Q9": 9, "D3Q15": 15, "D3Q19": 19}[lattice]
    n = np.arange(int(np.prod((tuple(shape) + (1, 1))[:3])), dtype=np.int64)
    B = POPULATION_BLOCK
    i = np.arange(Q, dtype=np.int64)[:, None]
    return (n // B) * Q * B + i * B + n % B


def _check_population_buffers(lattice, shape, *bufs):
    need = population_elements(lattice, shape)
    for t in bufs:
        if hasattr(t, "numel") and t.numel() < need:
            raise LBMError(-1, "population buffer of %d elements, %d needed"
                           % (t.numel(), need))


def pull_pattern_copy(lattice, precision, dst, src, shape, reps=10):
    """Time the step's pull pattern without arithmetic on a periodic
    nx x ny x nz grid, in the engine's blocked population layout (dst/src:
    torch tensors or device pointers of at least population_elements(lattice,
    shape) elements).  Returns ms per pass."""
    _check_population_buffers(lattice, shape, dst, src)
    d = dst.data_ptr() if hasattr(dst, "data_ptr") else int(dst)
    s = src.data_ptr() if hasattr(src, "data_ptr") else int(src)
    nx, ny, nz = (tuple(shape) + (1, 1))[:3]
    ms = np.zeros(1)
    rc = _pull_pattern(LATTICES[lattice], PRECISIONS[precision], _p(d), _p(s), int(nx), int(ny),
                       int(nz), int(reps), _ptr(ms))
    if rc:
        raise LBMError(rc, "pull_pattern_copy")
    return float(ms[0])


def adjoint_pattern_copy(lattice, precision, dst, f_src, lam_src, shape, reps=10):
    """Time the adjoint step's access pattern without arithmetic (f read at
    x - e_i, lambda at x + e_i, their sum written at x; blocked population
    layout, buffers as pull_pattern_copy).  Returns ms per pass."""
    _check_population_buffers(lattice, shape, dst, f_src, lam_src)
    ptr = [t.data_ptr() if hasattr(t, "data_ptr") else int(t) for t in (dst, f_src, lam_src)]
    nx, ny, nz = (tuple(shape) + (1, 1))[:3]
    ms = np.zeros(1)
    rc = _adj_pattern(LATTICES[lattice], PRECISIONS[precision], _p(ptr[0]), _p(ptr[1]), _p(ptr[2]),
                      int(nx), int(ny), int(nz), int(reps), _ptr(ms))
    if rc:
        raise LBMError(rc, "adjoint_pattern_copy")
    return float(ms[0])


def blocked_pull_pattern_copy(lattice, precision, block, dst, src, shape, reps=10):
    """Time the pull pattern in a layout of node blocks of `block` nodes that
    each hold their Q direction runs (dst/src: at least Q * nx*ny*nz
    elements; block = nx*ny*nz is the one-plane-per-direction layout).
    Returns ms per pass."""
    d = dst.data_ptr() if hasattr(dst, "data_ptr") else int(dst)
    s = src.data_ptr() if hasattr(src, "data_ptr") else int(src)
    nx, ny, nz = (tuple(shape) + (1, 1))[:3]
    ms = np.zeros(1)
    rc = _blocked_pattern(LATTICES[lattice], PRECISIONS[precision], int(block), _p(d), _p(s),
                          int(nx), int(ny), int(nz), int(reps), _ptr(ms))
    if rc:
        raise LBMError(rc, "blocked_pull_pattern_copy")
    return float(ms[0])


def aa_pattern_copy(lattice, precision, buf, shape, reps=10):
    """Time the in-place two-pass (AA) access pattern on one buffer of at
    least Q * nx*ny*nz elements (torch tensor or device pointer).  Returns
    (ms per even pass, ms per odd pass)."""
    b = buf.data_ptr() if hasattr(buf, "data_ptr") else int(buf)
    nx, ny, nz = (tuple(shape) + (1, 1))[:3]
    ms = np.zeros(2)
    rc = _aa_pattern(LATTICES[lattice], PRECISIONS[precision], _p(b), int(nx), int(ny), int(nz),
                     int(reps), ms[:1].ctypes.data_as(_p), ms[1:].ctypes.data_as(_p))
    if rc:
        raise LBMError(rc, "aa_pattern_copy")
    return float(ms[0]), float(ms[1])


class Solver:
    """One lattice Boltzmann solver on the current HIP device."""

    def __init__(self, lattice, shape, s, rho0=1.0, g=None, precision="fp64"):
        self.lattice = lattice
        self.shape = tuple(int(v) for v in shape)
        e, w, _ = lattice_info(lattice)
        self.Q, self.D = e.shape
        self.N = int(np.prod(self.shape))
        self.precision = precision
        s = _f64(s, self.Q)
        g = _f64(np.zeros(self.D) if g is None else np.asarray(g, float)[: self.D], self.D)
        h = _p()
        rc = _create(C.byref(h), LATTICES[lattice], PRECISIONS[precision],
                     self.shape[0], self.shape[1], self.shape[2],
                     s.ctypes.data_as(_dp), float(rho0), g.ctypes.data_as(_dp))
        if rc:
            raise LBMError(rc, "lbm_create")
        self._h = h
        self.rho0 = float(rho0)

    # -- helpers
    def _chk(self, rc, what):
        if rc:
            msg = _last_err(self._h)
            raise LBMError(rc, "%s: %s" % (what, msg.decode() if msg else ""))

    def close(self):
        if getattr(self, "_h", None):
            _destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # -- set-up
    def set_scheme(self, l_rule="min", b=1.0):
        self._chk(_set_scheme(self._h, RULES[l_rule], float(b)), "set_scheme")

    def set_two_node(self, on=True):
        self._chk(_set_two_node(self._h, 1 if on else 0), "set_two_node")

    def set_wall_decay(self, lam=1.0):
        """Wall data phi(x_b, t) = phi(x_b, 0) * lam**t (t in steps)."""
        self._chk(_set_wall_decay(self._h, float(lam)), "set_wall_decay")

    def set_x_boundary(self, kind="periodic", drho=0.0):
        self._chk(_set_xbc(self._h, X_BC[kind], float(drho)), "set_x_boundary")

    def set_geometry(self, solid, node, dir, q, wall_u=None, tag=None):
        solid = np.ascontiguousarray(solid, dtype=np.uint8)
        node = np.ascontiguousarray(node, dtype=np.int64)
        dir = np.ascontiguousarray(dir, dtype=np.int8)
        q = _f64(q, node.size)
        wall_u = _f64(wall_u, node.size * self.D) if wall_u is not None else None
        tag = np.ascontiguousarray(tag, dtype=np.int32) if tag is not None else None
        if solid.size != self.N:
            raise ValueError("solid mask must have N entries")
        self._chk(_set_geometry(self._h, _ptr(solid), node.size, _ptr(node),
                                _ptr(dir), _ptr(q), _ptr(wall_u), _ptr(tag)),
                  "set_geometry")

    def update_links(self, q=None, wall_u=None):
        q = _f64(q)
        wall_u = _f64(wall_u)
        self._chk(_update_links(self._h, _ptr(q), _ptr(wall_u)), "update_links")

    def set_parameters(self, s=None, g=None):
        s = _f64(s, self.Q) if s is not None else None
        g = _f64(np.asarray(g, float)[: self.D], self.D) if g is not None else None
        self._chk(_set_params(self._h, _ptr(s), _ptr(g)), "set_parameters")

    def set_collision(self, kind, s_nu, magic=3.0 / 16.0):
        """BGK or TRT through the MRT rates (lbm_set_collision)."""
        self._chk(_set_collision(self._h, COLLISIONS[kind], float(s_nu), float(magic)),
                  "set_collision")

    def counts(self):
        nf, nl = _i64(), _i64()
        _counts(self._h, C.byref(nf), C.byref(nl))
        return nf.value, nl.value

    # -- state
    def init(self, rho=None, u=None):
        rho = _f64(rho, self.N)
        u = _f64(u, self.N * self.D)
        self._chk(_init(self._h, _ptr(rho), _ptr(u)), "init")

    def init_deviation(self, df):
        df = _f64(df, self.Q * self.N)
        self._chk(_init_dev(self._h, _ptr(df)), "init_deviation")

    def step(self, n=1):
        self._chk(_step(self._h, int(n)), "step")

    @property
    def time(self):
        return int(_time(self._h))

    def moments(self):
        rho = np.empty(self.N)
        u = np.empty((self.N, self.D))
        self._chk(_moments(self._h, _ptr(rho), _ptr(u)), "moments")
        return rho, u

    def distribution(self):
        df = np.empty((self.Q, self.N))
        self._chk(_get_dist(self._h, _ptr(df)), "get_distribution")
        return df

    def reduce(self):
        m = np.zeros(1)
        mom = np.zeros(self.D)
        self._chk(_reduce(self._h, _ptr(m), _ptr(mom)), "reduce")
        return float(m[0]), mom

    def reduce_noalloc(self):
        """reduce() through the allocation-free entry point."""
        m = np.zeros(1)
        mom = np.zeros(self.D)
        self._chk(_reduce_noalloc(self._h, _ptr(m), _ptr(mom)), "reduce_noalloc")
        return float(m[0]), mom

    def force(self, n_tags):
        out = np.zeros((n_tags, self.D))
        self._chk(_force(self._h, int(n_tags), _ptr(out)), "force")
        return out

    def state_bytes(self):
        return int(_state_bytes(self._h))

    def get_state(self, dst_ptr):
        """dst_ptr: device pointer (int) or a torch tensor of state_bytes()."""
        ptr = dst_ptr.data_ptr() if hasattr(dst_ptr, "data_ptr") else int(dst_ptr)
        self._chk(_get_state(self._h, _p(ptr)), "get_state")

    def set_state(self, src_ptr, time):
        ptr = src_ptr.data_ptr() if hasattr(src_ptr, "data_ptr") else int(src_ptr)
        self._chk(_set_state(self._h, _p(ptr), int(time)), "set_state")

    def set_stream(self, stream):
        ptr = getattr(stream, "cuda_stream", stream)
        self._chk(_set_stream(self._h, _p(ptr) if ptr else None), "set_stream")

    # -- objective and adjoint
    def set_objective(self, kind, tag=0, t_begin=0, t_end=1, planes=None):
        """planes = (x_in, x_out) for "pressure_drop" (negative values count
        from nx; default (0, nx - 1))."""
        if planes is not None:
            nx = self.shape[0]
            self._chk(_set_obj_planes(self._h, int(planes[0]) % nx, int(planes[1]) % nx),
                      "set_objective_planes")
        self._chk(_set_obj(self._h, OBJECTIVES[kind], int(tag), int(t_begin),
                           int(t_end)), "set_objective")

    def pressure_drop(self, x_in=0, x_out=-1):
        """p_in - p_out (p = rho / 3, plane means over fluid nodes) at the
        current time."""
        nx = self.shape[0]
        dp = np.zeros(1)
        self._chk(_pressure_drop(self._h, int(x_in) % nx, int(x_out) % nx, _ptr(dp)),
                  "pressure_drop")
        return float(dp[0])

    def objective(self):
        J = np.zeros(1)
        self._chk(_objective(self._h, _ptr(J)), "objective")
        return float(J[0])

    def run_checkpointed(self, n, every):
        self._chk(_run_ckpt(self._h, int(n), int(every)), "run_checkpointed")

    def adjoint(self):
        self._chk(_adjoint(self._h), "adjoint")

    def adjoint_step(self, n):
        """n more steps of the reverse sweep (resumable)."""
        self._chk(_adj_step(self._h, int(n)), "adjoint_step")

    def adjoint_remaining(self):
        return int(_adj_remaining(self._h))

    def set_rate_gradient(self, on=True):
        self._chk(_set_rate_grad(self._h, 1 if on else 0), "set_rate_gradient")

    def grad(self):
        nf, nl = self.counts()
        dq = np.zeros(nl)
        du = np.zeros((nl, self.D))
        dg = np.zeros(self.D)
        ds = np.zeros(self.Q)
        self._chk(_grad(self._h, _ptr(dq), _ptr(du), _ptr(dg), _ptr(ds)), "grad")
        return dict(q=dq, wall_u=du, g=dg, s=ds)

    def grad_device(self, dq=None, wall_u=None):
        """Per-link gradients written into caller-owned device tensors
        (float64, contiguous: dq (L,), wall_u (L, D), caller link order) by
        a kernel on the handle's stream; dJ/dg and dJ/ds come back on the
        host."""
        nf, nl = self.counts()
        for t, shape in ((dq, (nl,)), (wall_u, (nl, self.D))):
            if t is not None and (tuple(t.shape) != shape or not t.is_contiguous()
                                  or str(t.dtype) != "torch.float64" or not t.is_cuda):
                raise ValueError("grad_device: expected a contiguous float64 device tensor of shape %s" % (shape,))
        dg = np.zeros(self.D)
        ds = np.zeros(self.Q)
        self._chk(_grad_dev(self._h, dq.data_ptr() if dq is not None else None,
                            wall_u.data_ptr() if wall_u is not None else None,
                            _ptr(dg), _ptr(ds)), "grad_device")
        return dict(g=dg, s=ds)

    def get_adjoint(self):
        lam = np.empty((self.Q, self.N))
        self._chk(_get_adj(self._h, _ptr(lam)), "get_adjoint")
        return lam

    # -- timing
    def set_timing(self, on=True):
        self._chk(_set_timing(self._h, 1 if on else 0), "set_timing")

    def last_step_ms(self):
        ms = np.zeros(1)
        self._chk(_last_ms(self._h, _ptr(ms)), "last_step_ms")
        return float(ms[0])


def solver_for(geom, s, rho0=1.0, g=None, precision="fp64", l_rule="min",
               b=1.0, dp=0.0, two_node=False):
    """Create a Solver and load a workloads.Geometry-like object into it."""
    sv = Solver(geom.lattice, geom.shape, s, rho0=rho0, g=g, precision=precision)
    sv.set_scheme(l_rule, b)
    if two_node:
        sv.set_two_node(True)
    sv.set_x_boundary(geom.x_bc, dp)
    sv.set_geometry(geom.solid, geom.node, geom.dir, geom.q, geom.wall_u, geom.tag)
    return sv
