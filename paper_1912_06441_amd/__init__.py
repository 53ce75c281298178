"""MI355X (gfx950) LABFM hot path: neighbours, weights, operator application, RK4.

Thin ctypes binding over liblabfm.so (C ABI in include/labfm.h).  Arguments
are torch tensors on the GPU; every step runs in the library's HIP kernels on
torch's current stream.  There is no CPU fallback: if liblabfm.so is missing
or no GPU is present, calls raise.

Method: King, Lind & Nasar, "High order difference schemes using the Local
Anisotropic Basis Function Method", arXiv:1912.06441 (Sec. 2, 3.1, 3.2,
App. A, Sec. 4.2, Sec. 5.1).
"""
import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblabfm.so")

ABF_HERMITE, ABF_PAPER, ABF_PAPER_D1 = 0, 1, 2
RBF_WENDLAND_C2, RBF_CONE, RBF_QUADRATIC, RBF_WENDLAND_C6, RBF_GAUSSIAN = 0, 1, 2, 3, 4
OP_DX, OP_DY, OP_LAP, OP_BIHARM, OP_TRIHARM = 1, 2, 4, 8, 16
OP_DZ = 32  # three-dimensional calls only
PREC_FP64, PREC_MIXED, PREC_MLP, PREC_MLP_NOLU = 0, 1, 2, 3
NOALLOC_MAX_NODES = 1 << 20  # largest n of labfm_weights_noalloc
ST_OK, ST_NOT_CONVERGED, ST_SINGULAR, ST_TOO_FEW, ST_DEGENERATE, ST_ORDER_TOO_LOW, ST_TOO_MANY = range(7)
MAX_NEIGHBOURS = 128
MAX_NEIGHBOURS3 = 256  # three-dimensional weights
MAX_ORDER3 = 6
EXPORTED = sorted(["labfm_last_error", "labfm_create", "labfm_destroy", "labfm_build_neighbours", "labfm_weights",
                   "labfm_combine", "labfm_apply_operator", "labfm_step", "labfm_timing_enable",
                   "labfm_timing_read", "labfm_mlp_features", "labfm_mlp_forward", "labfm_mlp_cache_floats",
                   "labfm_mlp_backward", "labfm_mlp_moment_loss", "labfm_mlp_adam", "labfm_mlp_cast_bf16",
                   "labfm_weights_batched", "labfm_autotune_query", "labfm_burgers_step",
                   "labfm_poisson_solve", "labfm_ns_step", "labfm_build_neighbours3", "labfm_weights3",
                   "labfm_weights_noalloc", "labfm_neumann_rows", "labfm_moment_systems"])
MLP_MAX_LAYERS = 8


class LabfmError(RuntimeError):
    pass


class Domain(C.Structure):
    _fields_ = [("lo", C.c_double * 2), ("hi", C.c_double * 2), ("periodic", C.c_int * 2)]


class MLPDesc(C.Structure):
    _fields_ = [("n_layers", C.c_int), ("dims", C.c_int * (MLP_MAX_LAYERS + 1)), ("W", C.c_void_p * MLP_MAX_LAYERS),
                ("b", C.c_void_p * MLP_MAX_LAYERS), ("mu", C.c_void_p), ("sd", C.c_void_p), ("order", C.c_int),
                ("ops", C.c_uint), ("kmax", C.c_int)]


class MLPGrads(C.Structure):
    _fields_ = [("W", C.c_void_p * MLP_MAX_LAYERS), ("b", C.c_void_p * MLP_MAX_LAYERS)]


class Adam(C.Structure):
    _fields_ = [("lr", C.c_double), ("beta1", C.c_double), ("beta2", C.c_double), ("eps", C.c_double)]


class WOpts(C.Structure):
    _fields_ = [("abf", C.c_int), ("rbf", C.c_int), ("sigma", C.c_double), ("ops", C.c_uint),
                ("prec", C.c_int), ("tol_stop", C.c_double), ("tol_pass", C.c_double), ("max_iters", C.c_int),
                ("mlp", C.POINTER(MLPDesc))]


class NodeSetDesc(C.Structure):
    _fields_ = [("x", C.c_void_p), ("y", C.c_void_p), ("n", C.c_int64), ("dom", Domain), ("R", C.c_void_p),
                ("order", C.c_void_p), ("row_ptr", C.c_void_p), ("col", C.c_void_p), ("nnz", C.c_int64),
                ("w64", C.c_void_p), ("w32", C.c_void_p), ("status", C.c_void_p), ("resid", C.c_void_p),
                ("iters", C.c_void_p)]


class BurgersPlan(C.Structure):
    _fields_ = [("row_ptr", C.c_void_p), ("col", C.c_void_p), ("n", C.c_int64), ("nnz", C.c_int64),
                ("dtype", C.c_int), ("w_x", C.c_void_p), ("w_y", C.c_void_p), ("w_lap", C.c_void_p),
                ("w_hv", C.c_void_p), ("nu", C.c_double), ("dt", C.c_double), ("fixed", C.c_void_p),
                ("dfix", C.c_void_p)]


class PoissonPlan(C.Structure):
    _fields_ = [("row_ptr", C.c_void_p), ("col", C.c_void_p), ("n", C.c_int64), ("nnz", C.c_int64),
                ("w_lap", C.c_void_p), ("fixed", C.c_void_p), ("tol", C.c_double), ("max_iters", C.c_int),
                ("check_every", C.c_int), ("center", C.c_void_p)]


class NSPlan(C.Structure):
    _fields_ = [("row_ptr", C.c_void_p), ("col", C.c_void_p), ("n", C.c_int64), ("nnz", C.c_int64),
                ("w_x", C.c_void_p), ("w_y", C.c_void_p), ("w_lap", C.c_void_p), ("psi_fixed", C.c_void_p),
                ("nu", C.c_double), ("dt", C.c_double), ("tol", C.c_double), ("max_iters", C.c_int),
                ("check_every", C.c_int)]


class StepPlan(C.Structure):
    _fields_ = [("row_ptr", C.c_void_p), ("col", C.c_void_p), ("n", C.c_int64), ("nnz", C.c_int64),
                ("dtype", C.c_int), ("w_lin", C.c_void_p), ("w_bh", C.c_void_p), ("gamma", C.c_double),
                ("dt", C.c_double), ("fixed", C.c_void_p)]


_lib = None


def load_library(path=LIB_PATH):
    """Load liblabfm.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise LabfmError("liblabfm.so not built (%s); run paper_1912_06441_amd/build.py" % path)
    L = C.CDLL(path)
    vp, i64, dp = C.c_void_p, C.c_int64, C.c_double
    L.labfm_last_error.restype = C.c_char_p
    L.labfm_create.argtypes = [C.POINTER(vp), C.c_int]
    L.labfm_destroy.argtypes = [vp]
    L.labfm_build_neighbours.argtypes = [vp, vp, vp, i64, C.POINTER(Domain), vp, vp, C.c_int, C.c_int, vp, vp,
                                         C.POINTER(i64), vp]
    L.labfm_weights.argtypes = [vp, vp, vp, i64, C.POINTER(Domain), vp, vp, vp, vp, i64, C.POINTER(WOpts), vp, vp,
                                vp, vp, vp, vp]
    L.labfm_weights_noalloc.argtypes = L.labfm_weights.argtypes
    L.labfm_combine.argtypes = [vp, vp, C.c_int, C.POINTER(dp), i64, vp, vp, vp]
    L.labfm_build_neighbours3.argtypes = [vp, vp, vp, vp, i64, C.POINTER(Domain3), vp, vp, vp, C.POINTER(i64), vp]
    L.labfm_weights3.argtypes = [vp, vp, vp, vp, i64, C.POINTER(Domain3), vp, C.c_int, vp, vp, i64,
                                 C.POINTER(WOpts), vp, vp, vp, vp, vp]
    L.labfm_apply_operator.argtypes = [vp, vp, vp, i64, i64, C.c_int, vp, C.c_int, vp, vp, vp]
    L.labfm_step.argtypes = [vp, C.POINTER(StepPlan), vp, vp, C.c_int, C.c_int, vp]
    L.labfm_burgers_step.argtypes = [vp, C.POINTER(BurgersPlan), vp, vp, vp, C.c_int, C.c_int, vp]
    L.labfm_ns_step.argtypes = [vp, C.POINTER(NSPlan), vp, vp, vp, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int),
                                vp]
    L.labfm_neumann_rows.argtypes = [vp, vp, vp, i64, i64, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, C.POINTER(i64), vp]
    L.labfm_poisson_solve.argtypes = [vp, C.POINTER(PoissonPlan), vp, vp, vp, C.POINTER(C.c_int),
                                      C.POINTER(C.c_double), C.POINTER(C.c_int), vp]
    L.labfm_moment_systems.argtypes = [vp, vp, vp, i64, C.POINTER(Domain), vp, C.c_int, vp, vp, i64, C.POINTER(WOpts),
                                       vp, vp, vp, vp]
    L.labfm_mlp_features.argtypes = [vp, vp, vp, i64, C.POINTER(Domain), vp, vp, vp, C.c_int, vp, vp]
    L.labfm_mlp_forward.argtypes = [vp, C.POINTER(MLPDesc), vp, i64, vp, vp, C.c_int, vp]
    L.labfm_mlp_cache_floats.argtypes = [C.POINTER(MLPDesc), i64]
    L.labfm_mlp_backward.argtypes = [vp, C.POINTER(MLPDesc), vp, vp, vp, i64, C.POINTER(MLPGrads), vp]
    L.labfm_mlp_moment_loss.argtypes = [vp, vp, vp, vp, vp, C.c_int, C.c_uint, i64, vp, vp, vp]
    L.labfm_mlp_adam.argtypes = [vp, vp, vp, vp, vp, vp, i64, C.POINTER(Adam), i64, vp]
    L.labfm_mlp_cast_bf16.argtypes = [vp, vp, vp, i64, vp]
    L.labfm_weights_batched.argtypes = [vp, C.c_int, C.POINTER(NodeSetDesc), C.POINTER(WOpts), C.c_int, vp]
    L.labfm_autotune_query.argtypes = [vp, C.c_int, C.c_int, C.c_uint, C.c_int, C.POINTER(C.c_int),
                                       C.POINTER(dp), C.POINTER(dp), C.POINTER(i64)]
    L.labfm_timing_enable.argtypes = [vp, C.c_int]
    L.labfm_timing_read.argtypes = [vp, C.c_char_p, C.POINTER(i64), C.POINTER(dp)]
    for name in EXPORTED:
        if name != "labfm_last_error":
            getattr(L, name).restype = C.c_int
    L.labfm_mlp_cache_floats.restype = C.c_int64
    _lib = L
    return L


def _check(rc, what):
    if rc != 0:
        msg = _lib.labfm_last_error().decode(errors="replace")
        raise LabfmError("%s failed (%d): %s" % (what, rc, msg))


def _torch():
    import torch

    if not torch.cuda.is_available():
        raise LabfmError("no HIP device: the LABFM path runs only on the GPU")
    return torch


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _need(name, t, dtype=None, n=None):
    """Arguments the kernels dereference must be contiguous GPU tensors of the
    stated dtype holding at least n elements (None: not given, skipped)."""
    if t is None:
        return
    if not getattr(t, "is_cuda", False):
        raise ValueError("%s must be a GPU tensor" % name)
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if dtype is not None and t.dtype != dtype:
        raise ValueError("%s must be %s, not %s" % (name, dtype, t.dtype))
    if n is not None and t.numel() < n:
        raise ValueError("%s holds %d elements, %d are needed" % (name, t.numel(), n))


def _need_csr(torch, row_ptr, col, n):
    _need("row_ptr", row_ptr, torch.int64, n + 1)
    _need("col", col, torch.int32)


def _stream(torch):
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


class Domain3(C.Structure):
    _fields_ = [("lo", C.c_double * 3), ("hi", C.c_double * 3), ("periodic", C.c_int * 3)]


def make_domain3(domain):
    d = Domain3()
    for a in range(3):
        d.lo[a] = float(domain["lo"][a])
        d.hi[a] = float(domain["hi"][a])
        d.periodic[a] = int(bool(domain["periodic"][a]))
    return d


def make_domain(domain):
    d = Domain()
    d.lo[0], d.lo[1] = [float(v) for v in domain["lo"]]
    d.hi[0], d.hi[1] = [float(v) for v in domain["hi"]]
    d.periodic[0], d.periodic[1] = [int(bool(v)) for v in domain["periodic"]]
    return d


def nops_of(ops):
    return bin(int(ops) & 31).count("1")


class Context:
    """A library context on one device (scratch + cached graphs)."""

    def __init__(self, device=0):
        self.torch = _torch()
        self.lib = load_library()
        self.device = device
        h = C.c_void_p()
        _check(self.lib.labfm_create(C.byref(h), int(device)), "labfm_create")
        self.h = h

    def close(self):
        if self.h:
            self.lib.labfm_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------------ timing
    def timing(self, enable=True):
        _check(self.lib.labfm_timing_enable(self.h, int(bool(enable))), "labfm_timing_enable")

    def timing_read(self, name_filter=None):
        """(launches, total_ms) of the recorded kernels whose name contains name_filter."""
        n = C.c_int64(0)
        ms = C.c_double(0.0)
        f = name_filter.encode() if name_filter else None
        _check(self.lib.labfm_timing_read(self.h, f, C.byref(n), C.byref(ms)), "labfm_timing_read")
        return n.value, ms.value

    # ------------------------------------------------------------------ neighbours
    def build_neighbours(self, x, y, R, order, domain, grow=True, max_grow=10):
        """CSR neighbour lists.  R is updated in place when grow.  Returns (row_ptr, col)."""
        torch = self.torch
        n = x.numel()
        for nm, t in (("x", x), ("y", y), ("R", R)):
            _need(nm, t, torch.float64, n)
        _need("order", order, torch.int8, n)
        dom = make_domain(domain)
        row_ptr = torch.empty(n + 1, dtype=torch.int64, device=x.device)
        nnz = C.c_int64(0)
        st = _stream(torch)
        _check(self.lib.labfm_build_neighbours(self.h, _ptr(x), _ptr(y), n, C.byref(dom), _ptr(R), _ptr(order),
                                               int(bool(grow)), int(max_grow), _ptr(row_ptr), None,
                                               C.byref(nnz), st), "labfm_build_neighbours(count)")
        col = torch.empty(max(nnz.value, 1), dtype=torch.int32, device=x.device)
        _check(self.lib.labfm_build_neighbours(self.h, _ptr(x), _ptr(y), n, C.byref(dom), _ptr(R), _ptr(order),
                                               0, 0, _ptr(row_ptr), _ptr(col), None, st),
               "labfm_build_neighbours(fill)")
        return row_ptr, col[:nnz.value]

    # ------------------------------------------------------------------ three dimensions
    def build_neighbours3(self, x, y, z, R, domain):
        """3-D CSR neighbour lists (no growth).  Returns (row_ptr, col)."""
        torch = self.torch
        n = x.numel()
        for nm, t in (("x", x), ("y", y), ("z", z), ("R", R)):
            _need(nm, t, torch.float64, n)
        dom = make_domain3(domain)
        row_ptr = torch.empty(n + 1, dtype=torch.int64, device=x.device)
        nnz = C.c_int64(0)
        st = _stream(torch)
        _check(self.lib.labfm_build_neighbours3(self.h, _ptr(x), _ptr(y), _ptr(z), n, C.byref(dom), _ptr(R),
                                                _ptr(row_ptr), None, C.byref(nnz), st), "labfm_build_neighbours3(count)")
        col = torch.empty(max(nnz.value, 1), dtype=torch.int32, device=x.device)
        _check(self.lib.labfm_build_neighbours3(self.h, _ptr(x), _ptr(y), _ptr(z), n, C.byref(dom), _ptr(R),
                                                _ptr(row_ptr), _ptr(col), None, st), "labfm_build_neighbours3(fill)")
        return row_ptr, col[:nnz.value]

    def weights3(self, x, y, z, R, k, row_ptr, col, domain, ops=OP_DX | OP_DY | OP_LAP | OP_DZ,
                 rbf=RBF_WENDLAND_C2, sigma=1.5, tol_stop=1e-13, tol_pass=1e-10, max_iters=5):
        """3-D FP64 weights [nops, nnz] (operators in bit order: dx, dy, lap, dz),
        status[n] int8, resid[n] f32, iters[n] int8."""
        torch = self.torch
        n = x.numel()
        nnz = col.numel()
        for nm, t in (("x", x), ("y", y), ("z", z), ("R", R)):
            _need(nm, t, torch.float64, n)
        _need_csr(torch, row_ptr, col, n)
        nop = bin(int(ops) & 63).count("1")
        dev = x.device
        w64 = torch.empty((nop, nnz), dtype=torch.float64, device=dev)
        status = torch.empty(n, dtype=torch.int8, device=dev)
        resid = torch.empty(n, dtype=torch.float32, device=dev)
        iters = torch.empty(n, dtype=torch.int8, device=dev)
        o = WOpts(ABF_HERMITE, int(rbf), float(sigma), int(ops), PREC_FP64, float(tol_stop), float(tol_pass),
                  int(max_iters), None)
        dom = make_domain3(domain)
        _check(self.lib.labfm_weights3(self.h, _ptr(x), _ptr(y), _ptr(z), n, C.byref(dom), _ptr(R), int(k),
                                       _ptr(row_ptr), _ptr(col), nnz, C.byref(o), _ptr(w64), _ptr(status),
                                       _ptr(resid), _ptr(iters), _stream(torch)), "labfm_weights3")
        return w64, status, resid, iters

    # ------------------------------------------------------------------ weights
    def weights(self, x, y, R, order, row_ptr, col, domain, ops=OP_DX | OP_DY | OP_LAP, abf=ABF_HERMITE,
                rbf=RBF_WENDLAND_C2, sigma=1.0, prec=PREC_FP64, tol_stop=1e-13, tol_pass=1e-10, max_iters=5,
                want64=True, want32=False, out=None, mlp=None, noalloc=False):
        """Weights [nops, nnz] (FP64 and/or FP32), status[n] int8, resid[n] f32, iters[n] int8.

        prec=PREC_MLP starts the refinement of the network's order from
        `mlp` (an MLP) instead of from a first solve; PREC_MLP_NOLU takes the
        network's coefficients without a factorisation and solves the nodes
        they leave above tol_pass on the FP64 path.  noalloc=True calls
        labfm_weights_noalloc (no library allocation; the outputs are still
        allocated here unless `out` is given)."""
        torch = self.torch
        n = x.numel()
        nnz = col.numel()
        for nm, t in (("x", x), ("y", y), ("R", R)):
            _need(nm, t, torch.float64, n)
        _need("order", order, torch.int8, n)
        _need_csr(torch, row_ptr, col, n)
        k = nops_of(ops)
        dev = x.device
        if out is None:
            w64 = torch.empty((k, nnz), dtype=torch.float64, device=dev) if want64 else None
            w32 = torch.empty((k, nnz), dtype=torch.float32, device=dev) if want32 else None
            status = torch.empty(n, dtype=torch.int8, device=dev)
            resid = torch.empty(n, dtype=torch.float32, device=dev)
            iters = torch.empty(n, dtype=torch.int8, device=dev)
        else:
            w64, w32, status, resid, iters = out
        _need("w64", w64, torch.float64, k * nnz)
        _need("w32", w32, torch.float32, k * nnz)
        _need("status", status, torch.int8, n)
        _need("resid", resid, torch.float32, n)
        _need("iters", iters, torch.int8, n)
        o = WOpts(int(abf), int(rbf), float(sigma), int(ops), int(prec), float(tol_stop), float(tol_pass),
                  int(max_iters), None)
        desc = None
        if prec in (PREC_MLP, PREC_MLP_NOLU):
            if mlp is None:
                raise LabfmError("the warm start needs a network (mlp=...)")
            desc = mlp.desc()
            o.mlp = C.pointer(desc)
        dom = make_domain(domain)
        fn = self.lib.labfm_weights_noalloc if noalloc else self.lib.labfm_weights
        _check(fn(self.h, _ptr(x), _ptr(y), n, C.byref(dom), _ptr(R), _ptr(order), _ptr(row_ptr), _ptr(col), nnz,
                  C.byref(o), _ptr(w64), _ptr(w32), _ptr(status), _ptr(resid), _ptr(iters), _stream(torch)),
               "labfm_weights_noalloc" if noalloc else "labfm_weights")
        return w64, w32, status, resid, iters

    def weights_batched(self, sets, ops=OP_DX | OP_DY | OP_LAP, abf=ABF_HERMITE, rbf=RBF_WENDLAND_C2, sigma=1.0,
                        prec=PREC_MIXED, tol_stop=1e-13, tol_pass=1e-10, max_iters=5, want64=True, want32=False,
                        use_graph=True, outs=None):
        """Weights of many node sets in one launch sequence.

        sets: list of dicts with x, y, R, order, row_ptr, col (device tensors)
        and domain.  Returns a list of (w64, w32, status, resid, iters) per
        set (allocated unless `outs` gives them)."""
        torch = self.torch
        k = nops_of(ops)
        if outs is None:
            outs = []
            for S in sets:
                n, nnz, dev = S["x"].numel(), S["col"].numel(), S["x"].device
                outs.append((torch.empty((k, nnz), dtype=torch.float64, device=dev) if want64 else None,
                             torch.empty((k, nnz), dtype=torch.float32, device=dev) if want32 else None,
                             torch.empty(n, dtype=torch.int8, device=dev),
                             torch.empty(n, dtype=torch.float32, device=dev),
                             torch.empty(n, dtype=torch.int8, device=dev)))
        for S, o in zip(sets, outs):
            n, nnz = S["x"].numel(), S["col"].numel()
            for nm in ("x", "y", "R"):
                _need(nm, S[nm], torch.float64, n)
            _need("order", S["order"], torch.int8, n)
            _need_csr(torch, S["row_ptr"], S["col"], n)
            _need("w64", o[0], torch.float64, k * nnz)
            _need("w32", o[1], torch.float32, k * nnz)
            _need("status", o[2], torch.int8, n)
            _need("resid", o[3], torch.float32, n)
            _need("iters", o[4], torch.int8, n)
        table = (NodeSetDesc * len(sets))()
        for t, (S, o) in enumerate(zip(sets, outs)):
            d = table[t]
            d.x, d.y, d.n = S["x"].data_ptr(), S["y"].data_ptr(), S["x"].numel()
            d.dom = make_domain(S["domain"])
            d.R, d.order = S["R"].data_ptr(), S["order"].data_ptr()
            d.row_ptr, d.col, d.nnz = S["row_ptr"].data_ptr(), S["col"].data_ptr(), S["col"].numel()
            d.w64 = o[0].data_ptr() if o[0] is not None else None
            d.w32 = o[1].data_ptr() if o[1] is not None else None
            d.status, d.resid, d.iters = o[2].data_ptr(), o[3].data_ptr(), o[4].data_ptr()
        o = WOpts(int(abf), int(rbf), float(sigma), int(ops), int(prec), float(tol_stop), float(tol_pass),
                  int(max_iters), None)
        _check(self.lib.labfm_weights_batched(self.h, len(sets), table, C.byref(o), int(bool(use_graph)),
                                              _stream(torch)), "labfm_weights_batched")
        return outs

    def autotune_query(self, order, ops=OP_DX | OP_DY | OP_LAP, abf=ABF_HERMITE, rbf=RBF_WENDLAND_C2):
        """(route, ms_mixed, ms_fp64, sample): route 0 untuned, 1 mixed kernels, 2 FP64 kernels."""
        r = C.c_int(0)
        a, b = C.c_double(0), C.c_double(0)
        ns = C.c_int64(0)
        _check(self.lib.labfm_autotune_query(self.h, int(abf), int(rbf), int(ops), int(order), C.byref(r), C.byref(a),
                                             C.byref(b), C.byref(ns)), "labfm_autotune_query")
        return r.value, a.value, b.value, ns.value

    def combine(self, w64, coef, want64=True, want32=False):
        torch = self.torch
        _need("w64", w64, torch.float64)
        nsets, nnz = w64.shape
        c = (C.c_double * nsets)(*[float(v) for v in coef])
        o64 = torch.empty(nnz, dtype=torch.float64, device=w64.device) if want64 else None
        o32 = torch.empty(nnz, dtype=torch.float32, device=w64.device) if want32 else None
        _check(self.lib.labfm_combine(self.h, _ptr(w64), nsets, c, nnz, _ptr(o64), _ptr(o32), _stream(torch)),
               "labfm_combine")
        return o64, o32

    # ------------------------------------------------------------------ application
    def apply_operator(self, row_ptr, col, w, u, out=None):
        """out[d, i] = sum_j w[d, s] (u[col[s]] - u[i]); w is [nops, nnz] or [nnz]."""
        torch = self.torch
        n = u.numel()
        w2 = w if w.dim() == 2 else w.view(1, -1)
        nops, nnz = w2.shape
        if w2.dtype != u.dtype:
            raise LabfmError("weights and field must have the same dtype")
        _need_csr(torch, row_ptr, col, n)
        _need("w", w2, u.dtype, nops * col.numel())
        _need("u", u, None, n)
        _need("out", out, u.dtype, nops * n)
        dtype = 1 if u.dtype == torch.float64 else 0
        if out is None:
            out = torch.empty((nops, n), dtype=u.dtype, device=u.device)
        _check(self.lib.labfm_apply_operator(self.h, _ptr(row_ptr), _ptr(col), n, nnz, nops, _ptr(w2), dtype,
                                             _ptr(u), _ptr(out), _stream(torch)), "labfm_apply_operator")
        return out if w.dim() == 2 else out[0]

    # ------------------------------------------------------------------ learned warm start
    def mlp_features(self, x, y, R, row_ptr, col, domain, kmax=64, out=None):
        """[n, 3 kmax] FP32 stencil features (nearest kmax neighbours by scaled distance)."""
        torch = self.torch
        n = x.numel()
        for nm, t in (("x", x), ("y", y), ("R", R)):
            _need(nm, t, torch.float64, n)
        _need_csr(torch, row_ptr, col, n)
        _need("out", out, torch.float32, 3 * kmax * n)
        feat = out if out is not None else torch.empty((n, 3 * kmax), dtype=torch.float32, device=x.device)
        dom = make_domain(domain)
        _check(self.lib.labfm_mlp_features(self.h, _ptr(x), _ptr(y), n, C.byref(dom), _ptr(R), _ptr(row_ptr),
                                           _ptr(col), int(kmax), _ptr(feat), _stream(torch)), "labfm_mlp_features")
        return feat

    def moment_systems(self, x, y, R, k, row_ptr, col, domain, ops=OP_DX | OP_DY | OP_LAP, abf=ABF_HERMITE,
                       rbf=RBF_WENDLAND_C2, sigma=1.0):
        """Training data of the warm start for the first n = row_ptr.numel() - 1
        nodes, at order k (x, y hold every node col refers to): moment matrices
        [n, p, p] FP32 (as assembled), coefficients Psi [n, nops p] FP32
        (operator-major) and status [n] int8."""
        torch = self.torch
        n = row_ptr.numel() - 1
        for nm, t in (("x", x), ("y", y), ("R", R)):
            _need(nm, t, torch.float64, n)
        _need_csr(torch, row_ptr, col, n)
        p = (k * k + 3 * k) // 2
        M = torch.empty((n, p, p), dtype=torch.float32, device=x.device)
        psi = torch.empty((n, nops_of(ops) * p), dtype=torch.float32, device=x.device)
        st = torch.empty(n, dtype=torch.int8, device=x.device)
        o = WOpts(int(abf), int(rbf), float(sigma), int(ops), PREC_FP64, 0.0, 0.0, 0, None)
        dom = make_domain(domain)
        _check(self.lib.labfm_moment_systems(self.h, _ptr(x), _ptr(y), n, C.byref(dom), _ptr(R), int(k),
                                             _ptr(row_ptr), _ptr(col), col.numel(), C.byref(o), _ptr(M), _ptr(psi),
                                             _ptr(st), _stream(torch)), "labfm_moment_systems")
        return M, psi, st

    # ------------------------------------------------------------------ time stepping
    def step(self, row_ptr, col, w_lin, w_bh, gamma, dt, u, nsteps, scratch=None, use_graph=True, fixed=None):
        """Advance u in place by nsteps RK4 steps of du/dt = L_lin u - gamma B(B u);
        nodes with fixed != 0 (int8 device tensor [n]) keep their value."""
        torch = self.torch
        n = u.numel()
        if u.dtype not in (torch.float32, torch.float64):
            raise ValueError("u must be float32 or float64")
        if scratch is None:
            scratch = torch.empty(5 * n, dtype=u.dtype, device=u.device)
        _need_csr(torch, row_ptr, col, n)
        _need("w_lin", w_lin, u.dtype, col.numel())
        _need("w_bh", w_bh, u.dtype, col.numel())
        _need("u", u, None, n)
        _need("scratch", scratch, u.dtype, 5 * n)
        dtype = 1 if u.dtype == torch.float64 else 0
        if fixed is not None and (fixed.dtype != torch.int8 or fixed.numel() != n or not fixed.is_contiguous()):
            raise ValueError("fixed must be a contiguous int8 tensor of n entries")
        plan = StepPlan(row_ptr.data_ptr(), col.data_ptr(), n, col.numel(), dtype, w_lin.data_ptr(),
                        w_bh.data_ptr() if w_bh is not None else None, float(gamma), float(dt),
                        fixed.data_ptr() if fixed is not None else None)
        _check(self.lib.labfm_step(self.h, C.byref(plan), _ptr(u), _ptr(scratch), int(nsteps), int(bool(use_graph)),
                                   _stream(torch)), "labfm_step")
        return u

    def burgers_step(self, row_ptr, col, w_x, w_y, w_lap, nu, dt, u, v, nsteps, w_hv=None, scratch=None,
                     use_graph=True, fixed=None, dfix=None):
        """Advance the velocity (u, v) in place by nsteps RK4 steps of the viscous
        Burgers' equation du/dt = -(u d/dx + v d/dy) u + nu lap u + L_hv u (same for v).
        Nodes with fixed != 0 hold their values or, with dfix ([2, 4, n], the
        dtype of u), take dfix[0, q] / dfix[1, q] as their stage-q derivatives."""
        torch = self.torch
        n = u.numel()
        if v.numel() != n or v.dtype != u.dtype:
            raise ValueError("u and v must have the same size and dtype")
        if u.dtype not in (torch.float32, torch.float64):
            raise ValueError("u and v must be float32 or float64")
        if scratch is None:
            scratch = torch.empty(6 * n, dtype=u.dtype, device=u.device)
        _need_csr(torch, row_ptr, col, n)
        for nm, t in (("w_x", w_x), ("w_y", w_y), ("w_lap", w_lap), ("w_hv", w_hv)):
            _need(nm, t, u.dtype, col.numel())
        _need("u", u, None, n)
        _need("v", v, None, n)
        _need("scratch", scratch, u.dtype, 6 * n)
        dtype = 1 if u.dtype == torch.float64 else 0
        if fixed is not None and (fixed.dtype != torch.int8 or fixed.numel() != n or not fixed.is_contiguous()):
            raise ValueError("fixed must be a contiguous int8 tensor of n entries")
        if dfix is not None and (dfix.dtype != u.dtype or dfix.numel() != 8 * n or not dfix.is_contiguous()
                                 or fixed is None):
            raise ValueError("dfix must be a contiguous [2, 4, n] tensor of u's dtype, with a fixed mask")
        plan = BurgersPlan(row_ptr.data_ptr(), col.data_ptr(), n, col.numel(), dtype, w_x.data_ptr(), w_y.data_ptr(),
                           w_lap.data_ptr(), w_hv.data_ptr() if w_hv is not None else None, float(nu), float(dt),
                           fixed.data_ptr() if fixed is not None else None,
                           dfix.data_ptr() if dfix is not None else None)
        _check(self.lib.labfm_burgers_step(self.h, C.byref(plan), _ptr(u), _ptr(v), _ptr(scratch), int(nsteps),
                                           int(bool(use_graph)), _stream(torch)), "labfm_burgers_step")
        return u, v

    def neumann_rows(self, row_ptr, col, w_x, w_y, w_lap, parent, nx, ny):
        """Rows of the global system with Neumann ghost rows (Sec. 5.2): a node
        with parent[g] = b >= 0 gets b's normal-derivative row along (nx[g],
        ny[g]), every other node its Laplacian row.  Returns (row_ptr, col, w,
        center) for poisson_solve(..., center=center)."""
        torch = self.torch
        n = row_ptr.numel() - 1
        _need_csr(torch, row_ptr, col, n)
        for nm, t in (("w_x", w_x), ("w_y", w_y), ("w_lap", w_lap)):
            _need(nm, t, torch.float64, col.numel())
        _need("parent", parent, torch.int32, n)
        _need("nx", nx, torch.float64, n)
        _need("ny", ny, torch.float64, n)
        dev = row_ptr.device
        orp = torch.empty(n + 1, dtype=torch.int64, device=dev)
        nnz = C.c_int64(0)
        st = _stream(torch)
        args = (self.h, _ptr(row_ptr), _ptr(col), n, col.numel(), _ptr(w_x), _ptr(w_y), _ptr(w_lap), _ptr(parent),
                _ptr(nx), _ptr(ny), _ptr(orp))
        _check(self.lib.labfm_neumann_rows(*args, None, None, None, C.byref(nnz), st), "labfm_neumann_rows(count)")
        ocol = torch.empty(max(nnz.value, 1), dtype=torch.int32, device=dev)
        ow = torch.empty(max(nnz.value, 1), dtype=torch.float64, device=dev)
        ocen = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
        _check(self.lib.labfm_neumann_rows(*args, _ptr(ocol), _ptr(ow), _ptr(ocen), None, st),
               "labfm_neumann_rows(fill)")
        return orp, ocol[:nnz.value], ow[:nnz.value], ocen[:n]

    def poisson_solve(self, row_ptr, col, w_lap, F, phi=None, fixed=None, tol=1e-10, max_iters=10000,
                      check_every=16, scratch=None, center=None):
        """Solve A^L phi = F (FP64, Jacobi-BiCGStab on the GPU); rows with
        fixed != 0 are identity rows; with center (from neumann_rows) row i
        takes its differences about node center[i].  Returns (phi,
        iterations, relative residual, converged)."""
        torch = self.torch
        n = F.numel()
        if F.dtype != torch.float64 or w_lap.dtype != torch.float64:
            raise ValueError("the Poisson solve is FP64: F and w_lap must be float64")
        if phi is None:
            phi = torch.zeros_like(F)
        if scratch is None:
            scratch = torch.empty(8 * n, dtype=torch.float64, device=F.device)
        _need_csr(torch, row_ptr, col, n)
        _need("w_lap", w_lap, torch.float64, col.numel())
        _need("F", F, torch.float64, n)
        _need("phi", phi, torch.float64, n)
        _need("scratch", scratch, torch.float64, 8 * n)
        if fixed is not None and (fixed.dtype != torch.int8 or fixed.numel() != n or not fixed.is_contiguous()):
            raise ValueError("fixed must be a contiguous int8 tensor of n entries")
        if center is not None:
            _need("center", center, torch.int32, n)
        plan = PoissonPlan(row_ptr.data_ptr(), col.data_ptr(), n, col.numel(), w_lap.data_ptr(),
                           fixed.data_ptr() if fixed is not None else None, float(tol), int(max_iters),
                           int(check_every), center.data_ptr() if center is not None else None)
        it, res, conv = C.c_int(0), C.c_double(0.0), C.c_int(0)
        _check(self.lib.labfm_poisson_solve(self.h, C.byref(plan), _ptr(F), _ptr(phi), _ptr(scratch), C.byref(it),
                                            C.byref(res), C.byref(conv), _stream(torch)), "labfm_poisson_solve")
        return phi, it.value, res.value, bool(conv.value)

    def ns_step(self, row_ptr, col, w_x, w_y, w_lap, nu, dt, omega, nsteps, psi=None, psi_fixed=None, tol=1e-10,
                max_iters=10000, check_every=8, scratch=None):
        """Advance the vorticity in place by nsteps RK4 steps of the vorticity-
        streamfunction Navier-Stokes equations (FP64).  Returns (omega, psi,
        BiCGStab iterations over all solves, all solves converged)."""
        torch = self.torch
        n = omega.numel()
        for t in (w_x, w_y, w_lap, omega):
            if t.dtype != torch.float64:
                raise ValueError("the vorticity-streamfunction step is FP64")
        if psi is None:
            psi = torch.zeros_like(omega)
        if scratch is None:
            scratch = torch.empty(14 * n, dtype=torch.float64, device=omega.device)
        _need_csr(torch, row_ptr, col, n)
        for nm, t in (("w_x", w_x), ("w_y", w_y), ("w_lap", w_lap)):
            _need(nm, t, torch.float64, col.numel())
        _need("omega", omega, torch.float64, n)
        _need("psi", psi, torch.float64, n)
        _need("psi_fixed", psi_fixed, torch.int8, n)
        _need("scratch", scratch, torch.float64, 14 * n)
        if psi_fixed is not None and (psi_fixed.dtype != torch.int8 or psi_fixed.numel() != n):
            raise ValueError("psi_fixed must be an int8 tensor of n entries")
        plan = NSPlan(row_ptr.data_ptr(), col.data_ptr(), n, col.numel(), w_x.data_ptr(), w_y.data_ptr(),
                      w_lap.data_ptr(), psi_fixed.data_ptr() if psi_fixed is not None else None, float(nu), float(dt),
                      float(tol), int(max_iters), int(check_every))
        it, conv = C.c_int(0), C.c_int(0)
        _check(self.lib.labfm_ns_step(self.h, C.byref(plan), _ptr(omega), _ptr(psi), _ptr(scratch), int(nsteps),
                                      C.byref(it), C.byref(conv), _stream(torch)), "labfm_ns_step")
        return omega, psi, it.value, bool(conv.value)


class MLP:
    """Warm-start network for the weight solve (parameters as device tensors).

    dims = (3 kmax, hidden..., nops * p(order)); SiLU between layers.  FP32
    master weights with BF16 copies for the matrix cores, FP32 biases, Adam
    moments, and the output de-normalisation Psi = mu + sd * y.  Every step
    (forward, backward, loss, Adam, cast) runs in liblabfm.so."""

    def __init__(self, ctx, dims=(192, 256, 256, 256, 132), order=8, ops=OP_DX | OP_DY | OP_LAP, kmax=64, seed=0,
                 out_scale=0.01):
        torch = ctx.torch
        self.ctx = ctx
        self.dims = tuple(int(d) for d in dims)
        self.L = len(self.dims) - 1
        if self.L < 1 or self.L > MLP_MAX_LAYERS:
            raise LabfmError("1..8 layers")
        self.order, self.ops, self.kmax = int(order), int(ops), int(kmax)
        dev = torch.device("cuda", ctx.device)
        g = torch.Generator().manual_seed(int(seed))
        # He-normal initial weights (the last layer scaled by out_scale, so that
        # an untrained network starts near Psi = mu), zero biases
        self.W = [(torch.randn((self.dims[l + 1], self.dims[l]), generator=g, dtype=torch.float64) *
                   (2.0 / self.dims[l]) ** 0.5 * (out_scale if l == self.L - 1 else 1.0)).to(torch.float32).to(dev)
                  for l in range(self.L)]
        self.b = [torch.zeros(self.dims[l + 1], dtype=torch.float32, device=dev) for l in range(self.L)]
        self.Wb = [torch.empty(w.shape, dtype=torch.bfloat16, device=dev) for w in self.W]
        self.mu = torch.zeros(self.dims[-1], dtype=torch.float32, device=dev)
        self.sd = torch.ones(self.dims[-1], dtype=torch.float32, device=dev)
        self.mW = [torch.zeros_like(w) for w in self.W]
        self.vW = [torch.zeros_like(w) for w in self.W]
        self.mb = [torch.zeros_like(b) for b in self.b]
        self.vb = [torch.zeros_like(b) for b in self.b]
        self.gW = [torch.empty_like(w) for w in self.W]
        self.gb = [torch.empty_like(b) for b in self.b]
        self.t = 0
        self.sync_bf16()

    def sync_bf16(self):
        """BF16 copies of the FP32 master weights."""
        for w, wb in zip(self.W, self.Wb):
            _check(self.ctx.lib.labfm_mlp_cast_bf16(self.ctx.h, _ptr(w), _ptr(wb), w.numel(),
                                                    _stream(self.ctx.torch)), "labfm_mlp_cast_bf16")

    def set_output_scaling(self, mu, sd):
        torch = self.ctx.torch
        self.mu.copy_(torch.as_tensor(mu, dtype=torch.float32))
        self.sd.copy_(torch.as_tensor(sd, dtype=torch.float32))

    def desc(self):
        d = MLPDesc()
        d.n_layers = self.L
        for l, v in enumerate(self.dims):
            d.dims[l] = v
        for l in range(self.L):
            d.W[l] = self.Wb[l].data_ptr()
            d.b[l] = self.b[l].data_ptr()
        d.mu, d.sd = self.mu.data_ptr(), self.sd.data_ptr()
        d.order, d.ops, d.kmax = self.order, self.ops, self.kmax
        self._desc = d  # keep alive while the call is enqueued
        return d

    def cache_for(self, B):
        torch = self.ctx.torch
        d = self.desc()
        nf = self.ctx.lib.labfm_mlp_cache_floats(C.byref(d), int(B))
        return torch.empty(max(nf, 1), dtype=torch.float32, device=self.W[0].device)

    def forward(self, X, cache=None, denorm=False, out=None):
        torch = self.ctx.torch
        B = X.shape[0]
        if out is None:
            out = torch.empty((B, self.dims[-1]), dtype=torch.float32, device=X.device)
        d = self.desc()
        _check(self.ctx.lib.labfm_mlp_forward(self.ctx.h, C.byref(d), _ptr(X), B, _ptr(out), _ptr(cache),
                                              int(bool(denorm)), _stream(torch)), "labfm_mlp_forward")
        return out

    def backward(self, X, cache, dout):
        """Fills self.gW / self.gb with dLoss/dW, dLoss/db."""
        d = self.desc()
        gr = MLPGrads()
        for l in range(self.L):
            gr.W[l] = self.gW[l].data_ptr()
            gr.b[l] = self.gb[l].data_ptr()
        _check(self.ctx.lib.labfm_mlp_backward(self.ctx.h, C.byref(d), _ptr(X), _ptr(cache), _ptr(dout), X.shape[0],
                                               C.byref(gr), _stream(self.ctx.torch)), "labfm_mlp_backward")
        return self.gW, self.gb

    def moment_loss(self, y, M, loss=None, dy=None):
        """Per-sample moment residual |M (mu + sd y) - C|^2 (FP64 [B]) and d(mean)/dy."""
        torch = self.ctx.torch
        B = y.shape[0]
        if loss is None:
            loss = torch.empty(B, dtype=torch.float64, device=y.device)
        if dy is None:
            dy = torch.empty_like(y)
        _check(self.ctx.lib.labfm_mlp_moment_loss(self.ctx.h, _ptr(y), _ptr(M), _ptr(self.mu), _ptr(self.sd),
                                                  self.order, self.ops, B, _ptr(dy), _ptr(loss), _stream(torch)),
               "labfm_mlp_moment_loss")
        return loss, dy

    def adam(self, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        """One Adam step on every parameter (gradients from the last backward)."""
        self.t += 1
        hp = Adam(float(lr), float(beta1), float(beta2), float(eps))
        st = _stream(self.ctx.torch)
        for l in range(self.L):
            _check(self.ctx.lib.labfm_mlp_adam(self.ctx.h, _ptr(self.W[l]), _ptr(self.gW[l]), _ptr(self.mW[l]),
                                               _ptr(self.vW[l]), _ptr(self.Wb[l]), self.W[l].numel(), C.byref(hp),
                                               self.t, st), "labfm_mlp_adam")
            _check(self.ctx.lib.labfm_mlp_adam(self.ctx.h, _ptr(self.b[l]), _ptr(self.gb[l]), _ptr(self.mb[l]),
                                               _ptr(self.vb[l]), None, self.b[l].numel(), C.byref(hp), self.t, st),
                   "labfm_mlp_adam")

    def train_step(self, X, M, lr, cache=None):
        """forward -> moment loss -> backward -> Adam on one batch; returns the per-sample losses."""
        if cache is None:
            cache = self.cache_for(X.shape[0])
        y = self.forward(X, cache=cache)
        loss, dy = self.moment_loss(y, M)
        self.backward(X, cache, dy)
        self.adam(lr)
        return loss
