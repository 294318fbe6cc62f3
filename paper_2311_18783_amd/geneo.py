"""Thin ctypes binding of libgeneo (include/geneo.h).

Argument marshalling only: every step of assembly, partitioning, setup,
apply and solve runs inside the library.  Device vectors are torch float64
tensors on the context's device, passed by data_ptr(); the library orders
its work on the given HIP stream (torch's current stream by default).
Importing this module fails loudly if libgeneo.so has not been built.
"""
from __future__ import annotations

import ctypes as C
import os
import re

import numpy as np
# torch's ROCm libraries must be loaded before libgeneo: the two HIP runtimes
# then share torch's HSA runtime; loading libgeneo first leaves the library's
# runtime without a device once torch initialises.
import torch  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgeneo.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "geneo.h")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2311_18783_amd.build`")
lib = C.CDLL(LIB_PATH)

STATUS = {0: "OK", -1: "EINVAL", -2: "ENOTSPD", -3: "ENOCONV", -4: "EOOM", -5: "EHIP", -6: "EUNSUPPORTED",
          -7: "ESYNC"}
FP64, FP32_REFINE1 = 0, 1
COARSE_SNK_GENEO, COARSE_SNK, COARSE_NONE, COARSE_NK, COARSE_NK_GENEO = 0, 1, 2, 3, 4
WEIGHT_IDENTITY, WEIGHT_POU = 0, 1
PCG, GMRES = 0, 1
PCG_DEFLATED, PCG_BALANCED = 0, 1
ORDER_NATURAL, ORDER_NESTED_DISSECTION, ORDER_AUTO = 0, 1, 2
SCHEDULE_AUTO, SCHEDULE_STEPS, SCHEDULE_LEVELS = 0, 1, 2
PART_BOX, PART_RCB, PART_EXPLICIT = 0, 1, 2


class GeneoError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code
        self.status = STATUS.get(code, str(code))


class Mesh(C.Structure):
    _fields_ = [("n_nodes", C.c_int64), ("xyz", C.POINTER(C.c_double)), ("n_tets", C.c_int64),
                ("tets", C.POINTER(C.c_int32)), ("cell_of_tet", C.POINTER(C.c_int32)),
                ("n_bfaces", C.c_int64), ("bfaces", C.POINTER(C.c_int32)),
                ("bface_dirichlet", C.POINTER(C.c_int8))]


class SystemInfo(C.Structure):
    _fields_ = [("n", C.c_int64), ("nnz", C.c_int64), ("n_edges", C.c_int64), ("n_free_nodes", C.c_int64),
                ("n_cells", C.c_int64), ("assemble_ms", C.c_double)]


class PartitionOpts(C.Structure):
    _fields_ = [("kind", C.c_int32), ("box", C.c_int32 * 3), ("nparts", C.c_int32),
                ("rcb_jitter", C.POINTER(C.c_double)), ("part_of_cell", C.POINTER(C.c_int32)),
                ("overlap", C.c_int32)]


class DecompInfo(C.Structure):
    _fields_ = [("n_sub", C.c_int32), ("n_min", C.c_int32), ("n_max", C.c_int32), ("sum_n", C.c_int64),
                ("sum_p", C.c_int64), ("n_floating", C.c_int32), ("sum_n3_over_3", C.c_double)]


class SetupOpts(C.Structure):
    _fields_ = [("tau", C.c_double), ("nev_max", C.c_int32), ("coarse", C.c_int32),
                ("local_precision", C.c_int32), ("lobpcg_tol", C.c_double), ("lobpcg_maxit", C.c_int32),
                ("lobpcg_guard", C.c_int32), ("seed", C.c_uint64), ("coarse_drop_tol", C.c_double),
                ("warm_start", C.POINTER(C.c_double)), ("fp32_rho_max", C.c_double),
                ("model", C.c_void_p), ("keep_ritz", C.c_int32), ("coarse_order", C.c_int32),
                ("one_level_weight", C.c_int32), ("classical", C.c_int32), ("coarse_schedule", C.c_int32)]


class PrecondInfo(C.Structure):
    _fields_ = [("n0", C.c_int32), ("n0_rank", C.c_int32), ("n0_local_dropped", C.c_int32),
                ("n_snk", C.c_int32), ("n_geneo", C.c_int32),
                ("lobpcg_iters", C.c_int32), ("lobpcg_unconverged", C.c_int32), ("fp64_fallbacks", C.c_int32),
                ("min_kept_pivot", C.c_double), ("max_dropped_pivot", C.c_double),
                ("t_extract_ms", C.c_double), ("t_factor_ms", C.c_double), ("t_gevp_ms", C.c_double),
                ("t_coarse_build_ms", C.c_double), ("t_coarse_factor_ms", C.c_double),
                ("local_factor_flops", C.c_double), ("fp32_rho_est", C.c_double),
                ("coarse_factor_flops", C.c_double), ("coarse_fill", C.c_double),
                ("learned_starts", C.c_int32), ("start_residual", C.c_double),
                ("fp32_prechecked", C.c_int32), ("fp32_kappa_lb", C.c_double),
                ("learned_candidates", C.c_int32), ("coarse_nd_levels", C.c_int32),
                ("coarse_nd_predicted_depth", C.c_int32),
                ("coarse_solve_depth", C.c_int32), ("coarse_levels", C.c_int32),
                ("coarse_schedule_used", C.c_int32), ("t_factor_fp32_ms", C.c_double),
                ("coarse_lambda_min", C.c_double), ("coarse_drop_tol_used", C.c_double),
                ("coarse_refactors", C.c_int32), ("t_coarse_refactor_ms", C.c_double),
                ("coarse_solve_bytes", C.c_double), ("t_lobpcg_loop_ms", C.c_double),
                ("lobpcg_solve_ms", C.c_double), ("lobpcg_solve_bytes", C.c_double)]


class ModelOpts(C.Structure):
    _fields_ = [("canvas", C.c_int32), ("hidden", C.c_int32), ("k", C.c_int32), ("seed", C.c_uint64)]


class ModelInfo(C.Structure):
    _fields_ = [("in_dim", C.c_int32), ("rows", C.c_int32), ("k", C.c_int32), ("hidden", C.c_int32),
                ("canvas", C.c_int32), ("n_params", C.c_int64), ("n_train", C.c_int32), ("n_holdout", C.c_int32)]


class TrainOpts(C.Structure):
    _fields_ = [("epochs", C.c_int32), ("batch", C.c_int32), ("lr", C.c_double), ("seed", C.c_uint64)]


class TrainInfo(C.Structure):
    _fields_ = [("loss_first", C.c_double), ("loss_last", C.c_double), ("holdout_loss", C.c_double),
                ("train_ms", C.c_double)]


class FactorSchedule(C.Structure):
    _fields_ = [("mode", C.c_int32), ("group", C.c_int32), ("potrf", C.c_int32), ("ms", C.c_double)]


class SolveOpts(C.Structure):
    _fields_ = [("rtol", C.c_double), ("maxit", C.c_int32), ("graph", C.c_int32), ("method", C.c_int32),
                ("restart", C.c_int32), ("true_residual", C.c_int32), ("pcg_form", C.c_int32)]


class SolveInfo(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("rel_residual", C.c_double), ("solve_ms", C.c_double),
                ("graph_replays", C.c_int32), ("residual_replacements", C.c_int32),
                ("true_rel_residual", C.c_double), ("residual_floor", C.c_double),
                ("coarse_solve_ms", C.c_double), ("coarse_solves", C.c_int64)]


_vp = C.c_void_p
_P = C.POINTER
_sigs = {
    "geneo_create": (C.c_int, [_P(_vp), C.c_int, _vp]),
    "geneo_destroy": (None, [_vp]),
    "geneo_last_error": (C.c_char_p, [_vp]),
    "geneo_assemble": (C.c_int, [_vp, _P(Mesh), _P(C.c_double), _P(C.c_double), C.c_double, _P(_vp)]),
    "geneo_system_info_get": (C.c_int, [_vp, _P(SystemInfo)]),
    "geneo_system_export": (C.c_int, [_vp, _vp, _P(C.c_int32), _P(C.c_int32), _P(C.c_double), _P(C.c_int32)]),
    "geneo_spmv": (C.c_int, [_vp, _vp, _vp, _vp]),
    "geneo_partition": (C.c_int, [_vp, _vp, _P(PartitionOpts), _P(_vp)]),
    "geneo_decomp_info_get": (C.c_int, [_vp, _P(DecompInfo)]),
    "geneo_decomp_subdomain": (C.c_int, [_vp, C.c_int32, _P(C.c_int32), _P(C.c_int32), _P(C.c_double),
                                         _P(C.c_int32), _P(C.c_int32)]),
    "geneo_setup_opts_default": (None, [_P(SetupOpts)]),
    "geneo_setup": (C.c_int, [_vp, _vp, _vp, _P(SetupOpts), _P(_vp)]),
    "geneo_precond_info_get": (C.c_int, [_vp, _P(PrecondInfo)]),
    "geneo_precond_eigs": (C.c_int, [_vp, C.c_int32, _P(C.c_double), C.c_int32, _P(C.c_int32), _P(C.c_int32)]),
    "geneo_precond_ritz": (C.c_int, [_vp, _vp, C.c_int32, _P(C.c_double), C.c_int32, _P(C.c_int32)]),
    "geneo_apply": (C.c_int, [_vp, _vp, _vp, _vp]),
    "geneo_solve": (C.c_int, [_vp, _vp, _vp, _vp, _vp, _P(SolveOpts), _P(SolveInfo)]),
    "geneo_potrf_batched": (C.c_int, [_vp, C.c_int32, _P(C.c_int32), _P(C.c_int64), _vp, C.c_int32,
                                      _P(C.c_double)]),
    "geneo_potrf_batched_noalloc": (C.c_int, [_vp, C.c_int32, _P(C.c_int32), _P(C.c_int64), _vp, C.c_int32,
                                              _P(C.c_double)]),
    "geneo_tune_factor": (C.c_int, [_vp, C.c_int32, _P(C.c_int32), C.c_int32, C.c_int32, _P(FactorSchedule),
                                    _P(C.c_int32)]),
    "geneo_tune_lookup": (C.c_int, [C.c_int32, _P(C.c_int32), C.c_int32, _P(FactorSchedule)]),
    "geneo_tune_save": (C.c_int, [C.c_char_p]),
    "geneo_tune_load": (C.c_int, [C.c_char_p]),
    "geneo_model_opts_default": (None, [_P(ModelOpts)]),
    "geneo_model_create": (C.c_int, [_vp, _P(ModelOpts), _P(_vp)]),
    "geneo_model_info_get": (C.c_int, [_vp, _P(ModelInfo)]),
    "geneo_model_collect": (C.c_int, [_vp, _vp, _vp, _vp, _vp, C.c_int32]),
    "geneo_model_train": (C.c_int, [_vp, _vp, _P(TrainOpts), _P(TrainInfo)]),
    "geneo_model_predict": (C.c_int, [_vp, _vp, C.c_int32, _P(C.c_float), _P(C.c_float)]),
    "geneo_model_loss_grad": (C.c_int, [_vp, _vp, C.c_int32, _P(C.c_float), _P(C.c_float), _P(C.c_uint8),
                                        _P(C.c_double), _P(C.c_float)]),
    "geneo_model_get_params": (C.c_int, [_vp, _P(C.c_float)]),
    "geneo_model_set_params": (C.c_int, [_vp, _vp, _P(C.c_float)]),
    "geneo_model_save": (C.c_int, [_vp, C.c_char_p]),
    "geneo_model_load": (C.c_int, [_vp, C.c_char_p, _P(_vp)]),
    "geneo_free_model": (None, [_vp]),
    "geneo_free_system": (None, [_vp]),
    "geneo_free_decomp": (None, [_vp]),
    "geneo_free_precond": (None, [_vp]),
}
for _name, (_res, _args) in _sigs.items():
    _f = getattr(lib, _name)
    _f.restype = _res
    _f.argtypes = _args


def header_symbols(path=HEADER):
    """Function names declared in include/geneo.h."""
    txt = open(path).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(geneo_[a-z0-9_]+)\s*\(", txt)))


def _ptr(a, ct):
    return a.ctypes.data_as(C.POINTER(ct)) if a is not None else None


def _dptr(t):
    return C.c_void_p(t.data_ptr())


def check_vector(t, n, device, name="vector"):
    """Reject a tensor the library cannot take as a device vector of length
    n: it must be a contiguous torch float64 tensor on HIP device `device`
    with exactly n elements.  Raises ValueError before any library call, so
    a wrong dtype, length or device never reaches a kernel."""
    import torch
    if not isinstance(t, torch.Tensor):
        raise ValueError(f"{name}: expected a torch tensor, got {type(t).__name__}")
    if t.dtype != torch.float64:
        raise ValueError(f"{name}: dtype {t.dtype}, expected torch.float64")
    if not t.is_contiguous():
        raise ValueError(f"{name}: not contiguous")
    if t.numel() != n:
        raise ValueError(f"{name}: {t.numel()} elements, expected n = {n}")
    if t.device.type != "cuda" or (t.device.index if t.device.index is not None else 0) != device:
        raise ValueError(f"{name}: on {t.device}, expected cuda:{device}")


def tune_lookup(sizes, precision=FP64):
    """geneo_tune_lookup: the factorisation schedule (mode, group, potrf) a
    batch of these matrix sizes gets from the process-wide table (host only)."""
    n = np.ascontiguousarray(sizes, dtype=np.int32)
    out = FactorSchedule()
    rc = lib.geneo_tune_lookup(len(n), _ptr(n, C.c_int32), int(precision), C.byref(out))
    if rc != 0:
        raise GeneoError(rc, "bad sizes or precision")
    return out.mode, out.group, out.potrf


def tune_save(path):
    """geneo_tune_save: write the schedule table to a text file."""
    rc = lib.geneo_tune_save(str(path).encode())
    if rc != 0:
        raise GeneoError(rc, f"cannot write {path}")


def tune_load(path):
    """geneo_tune_load: merge a schedule table from a text file."""
    rc = lib.geneo_tune_load(str(path).encode())
    if rc != 0:
        raise GeneoError(rc, f"cannot read or parse {path}")


class Context:
    """A library context bound to one device and one HIP stream."""

    def __init__(self, device=0, stream=None):
        import torch
        self.device = device
        if stream is None:
            stream = torch.cuda.current_stream(device).cuda_stream
        self.h = C.c_void_p()
        self._check(lib.geneo_create(C.byref(self.h), device, C.c_void_p(stream)))

    def _check(self, rc):
        if rc != 0:
            msg = lib.geneo_last_error(self.h if self.h else None).decode()
            raise GeneoError(rc, msg)

    def close(self):
        if self.h:
            lib.geneo_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -------------------------------------------------------------- assemble
    def assemble(self, mesh, mu, eps, gamma, dirichlet):
        xyz = np.ascontiguousarray(mesh["xyz"], dtype=np.float64)
        tets = np.ascontiguousarray(mesh["tets"], dtype=np.int32)
        cot = np.ascontiguousarray(mesh["hex_of_tet"], dtype=np.int32) if "hex_of_tet" in mesh else None
        bf = np.ascontiguousarray(mesh["bfaces"], dtype=np.int32)
        bd = np.ascontiguousarray(dirichlet, dtype=np.int8)
        mu = np.ascontiguousarray(mu, dtype=np.float64)
        eps = np.ascontiguousarray(eps, dtype=np.float64)
        m = Mesh(xyz.shape[0], _ptr(xyz, C.c_double), tets.shape[0], _ptr(tets, C.c_int32),
                 _ptr(cot, C.c_int32) if cot is not None else None, bf.shape[0], _ptr(bf, C.c_int32),
                 _ptr(bd, C.c_int8))
        h = C.c_void_p()
        self._check(lib.geneo_assemble(self.h, C.byref(m), _ptr(mu, C.c_double), _ptr(eps, C.c_double),
                                       float(gamma), C.byref(h)))
        return System(self, h)

    def partition(self, system, kind="box", box=(1, 1, 1), nparts=0, jitter=None, part_of_cell=None, overlap=1):
        o = PartitionOpts()
        o.kind = {"box": PART_BOX, "rcb": PART_RCB, "explicit": PART_EXPLICIT}[kind]
        o.box = (C.c_int32 * 3)(*box)
        o.nparts = int(nparts)
        jit = np.ascontiguousarray(jitter, dtype=np.float64) if jitter is not None else None
        poc = np.ascontiguousarray(part_of_cell, dtype=np.int32) if part_of_cell is not None else None
        o.rcb_jitter = _ptr(jit, C.c_double) if jit is not None else None
        o.part_of_cell = _ptr(poc, C.c_int32) if poc is not None else None
        o.overlap = int(overlap)
        h = C.c_void_p()
        self._check(lib.geneo_partition(self.h, system.h, C.byref(o), C.byref(h)))
        return Decomp(self, h)

    def setup(self, system, decomp, **kw):
        o = SetupOpts()
        lib.geneo_setup_opts_default(C.byref(o))
        ws = kw.pop("warm_start", None)
        model = kw.pop("model", None)
        for k, v in kw.items():
            setattr(o, k, v)
        if model is not None:
            o.model = model.h
        if ws is not None:
            ws = np.ascontiguousarray(ws, dtype=np.float64)
            o.warm_start = _ptr(ws, C.c_double)
        h = C.c_void_p()
        self._check(lib.geneo_setup(self.h, system.h, decomp.h, C.byref(o), C.byref(h)))
        pc = Precond(self, h)
        pc.system, pc.n = system, system.info().n
        return pc

    def apply(self, pc, r, z):
        check_vector(r, pc.n, self.device, "r")
        check_vector(z, pc.n, self.device, "z")
        self._check(lib.geneo_apply(self.h, pc.h, _dptr(r), _dptr(z)))

    def spmv(self, system, x, y):
        n = system.info().n
        check_vector(x, n, self.device, "x")
        check_vector(y, n, self.device, "y")
        self._check(lib.geneo_spmv(self.h, system.h, _dptr(x), _dptr(y)))

    def solve(self, system, pc, b, x, rtol=1e-8, maxit=1000, allow_noconv=False, graph=True, method=PCG,
              restart=0, true_residual=False, pcg_form=None):
        """geneo_solve: PCG (method=PCG) or right-preconditioned GMRES
        (method=GMRES, restart length `restart`, 0 = none) from x = 0 (b, x:
        float64 device tensors of length n).  graph=True replays one captured
        PCG iteration as a HIP graph from the second iteration on;
        graph=False launches kernel by kernel (same kernels, bitwise equal
        iterates).  allow_noconv returns the info of a run stopped by maxit
        instead of raising.  true_residual=True: PCG continues from the true
        residual while it misses rtol (at most two restarts).  pcg_form:
        PCG_DEFLATED (default: from x0 = Q b with (I - Q A) M_AS + Q, one
        coarse solve per iteration) or PCG_BALANCED (M_AS,2 from x0 = 0)."""
        n = system.info().n
        if pc is not None and pc.system is not system:
            raise ValueError("the preconditioner was built on another system")
        check_vector(b, n, self.device, "b")
        check_vector(x, n, self.device, "x")
        o = SolveOpts(float(rtol), int(maxit), 1 if graph else 0, int(method), int(restart),
                      1 if true_residual else 0, PCG_DEFLATED if pcg_form is None else int(pcg_form))
        info = SolveInfo()
        rc = lib.geneo_solve(self.h, system.h, pc.h if pc is not None else None, _dptr(b), _dptr(x),
                             C.byref(o), C.byref(info))
        if rc == -3 and allow_noconv:
            return info
        self._check(rc)
        return info

    def potrf_batched(self, A, sizes, offsets, precision=FP64, noalloc=False):
        """geneo_potrf_batched (noalloc=True: geneo_potrf_batched_noalloc, which
        allocates no device memory and takes batches up to its scratch limit)."""
        import torch
        n = np.ascontiguousarray(sizes, dtype=np.int32)
        off = np.ascontiguousarray(offsets, dtype=np.int64)
        want = torch.float64 if precision == FP64 else torch.float32
        if not isinstance(A, torch.Tensor) or A.dtype != want or not A.is_contiguous() \
                or A.device.type != "cuda":
            raise ValueError(f"A: expected a contiguous {want} device tensor")
        ld = (n.astype(np.int64) + 127) // 128 * 128
        if n.size == 0 or (n < 1).any() or (off < 0).any() or int((off + ld * ld).max()) > A.numel():
            raise ValueError("A: matrix sizes / offsets run past the buffer")
        ms = C.c_double()
        fn = lib.geneo_potrf_batched_noalloc if noalloc else lib.geneo_potrf_batched
        self._check(fn(self.h, len(n), _ptr(n, C.c_int32), _ptr(off, C.c_int64), _dptr(A), int(precision),
                       C.byref(ms)))
        return ms.value


    def tune_factor(self, sizes, precision=FP64, reps=2):
        """geneo_tune_factor: time the candidate schedules on synthetic SPD
        matrices of these sizes, record the fastest for the batch's key and
        return (mode, group, potrf, ms, candidates timed)."""
        n = np.ascontiguousarray(sizes, dtype=np.int32)
        best = FactorSchedule()
        tried = C.c_int32()
        self._check(lib.geneo_tune_factor(self.h, len(n), _ptr(n, C.c_int32), int(precision), int(reps),
                                          C.byref(best), C.byref(tried)))
        return best.mode, best.group, best.potrf, best.ms, tried.value

    # -------------------------------------------------------------- learned warm start
    def model_create(self, canvas=12, hidden=256, k=20, seed=2311):
        o = ModelOpts(int(canvas), int(hidden), int(k), int(seed))
        h = C.c_void_p()
        self._check(lib.geneo_model_create(self.h, C.byref(o), C.byref(h)))
        return Model(self, h)

    def model_load(self, path):
        h = C.c_void_p()
        self._check(lib.geneo_model_load(self.h, str(path).encode(), C.byref(h)))
        return Model(self, h)


class _Handle:
    _free = None

    def __init__(self, ctx, h):
        self.ctx = ctx
        self.h = h

    def __del__(self):
        try:
            if self.h and self._free is not None:
                getattr(lib, self._free)(self.h)
                self.h = None
        except Exception:
            pass


class System(_Handle):
    _free = "geneo_free_system"

    def info(self):
        i = SystemInfo()
        self.ctx._check(lib.geneo_system_info_get(self.h, C.byref(i)))
        return i

    def export(self):
        """Host copy of A (scipy CSR) and the global edge id of each free edge."""
        import scipy.sparse as sp
        i = self.info()
        rp = np.empty(i.n + 1, np.int32)
        ci = np.empty(i.nnz, np.int32)
        v = np.empty(i.nnz, np.float64)
        fe = np.empty(i.n, np.int32)
        self.ctx._check(lib.geneo_system_export(self.ctx.h, self.h, _ptr(rp, C.c_int32), _ptr(ci, C.c_int32),
                                                _ptr(v, C.c_double), _ptr(fe, C.c_int32)))
        return sp.csr_matrix((v, ci, rp), shape=(i.n, i.n)), fe


class Decomp(_Handle):
    _free = "geneo_free_decomp"

    def info(self):
        i = DecompInfo()
        self.ctx._check(lib.geneo_decomp_info_get(self.h, C.byref(i)))
        return i

    def subdomain(self, i):
        ni, pi = C.c_int32(), C.c_int32()
        self.ctx._check(lib.geneo_decomp_subdomain(self.h, i, C.byref(ni), None, None, C.byref(pi), None))
        dofs = np.empty(ni.value, np.int32)
        pou = np.empty(ni.value, np.float64)
        gn = np.empty(pi.value, np.int32)
        self.ctx._check(lib.geneo_decomp_subdomain(self.h, i, None, _ptr(dofs, C.c_int32), _ptr(pou, C.c_double),
                                                   None, _ptr(gn, C.c_int32)))
        return dofs, pou, gn


class Precond(_Handle):
    _free = "geneo_free_precond"

    def info(self):
        i = PrecondInfo()
        self.ctx._check(lib.geneo_precond_info_get(self.h, C.byref(i)))
        return i

    def ritz(self, i, n_i, cap=64):
        kk = C.c_int32()
        self.ctx._check(lib.geneo_precond_ritz(self.ctx.h, self.h, i, None, cap, C.byref(kk)))
        V = np.empty((kk.value, n_i), np.float64)
        self.ctx._check(lib.geneo_precond_ritz(self.ctx.h, self.h, i, _ptr(V, C.c_double), cap, C.byref(kk)))
        return V.T.copy()

    def eigs(self, i, cap=64):
        lam = np.empty(cap, np.float64)
        cnt, sel = C.c_int32(), C.c_int32()
        self.ctx._check(lib.geneo_precond_eigs(self.h, i, _ptr(lam, C.c_double), cap, C.byref(cnt), C.byref(sel)))
        return lam[:cnt.value].copy(), sel.value


class Model(_Handle):
    """Learned warm start of the eigensolver (see include/geneo.h)."""
    _free = "geneo_free_model"

    def info(self):
        i = ModelInfo()
        self.ctx._check(lib.geneo_model_info_get(self.h, C.byref(i)))
        return i

    def collect(self, system, decomp, precond, holdout=False):
        self.ctx._check(lib.geneo_model_collect(self.ctx.h, self.h, system.h, decomp.h, precond.h, int(holdout)))

    def train(self, epochs=20, batch=32, lr=1e-3, seed=0):
        o = TrainOpts(int(epochs), int(batch), float(lr), int(seed))
        i = TrainInfo()
        self.ctx._check(lib.geneo_model_train(self.ctx.h, self.h, C.byref(o), C.byref(i)))
        return i

    def predict(self, X):
        X = np.ascontiguousarray(X, dtype=np.float32)
        inf = self.info()
        Y = np.empty((X.shape[0], inf.rows * inf.k), np.float32)
        self.ctx._check(lib.geneo_model_predict(self.ctx.h, self.h, X.shape[0], _ptr(X, C.c_float),
                                                _ptr(Y, C.c_float)))
        return Y

    def loss_grad(self, X, V, mask, with_grad=True):
        X = np.ascontiguousarray(X, dtype=np.float32)
        V = np.ascontiguousarray(V, dtype=np.float32)
        mask = np.ascontiguousarray(mask, dtype=np.uint8)
        loss = C.c_double()
        g = np.empty(self.info().n_params, np.float32) if with_grad else None
        self.ctx._check(lib.geneo_model_loss_grad(self.ctx.h, self.h, X.shape[0], _ptr(X, C.c_float),
                                                  _ptr(V, C.c_float), _ptr(mask, C.c_uint8), C.byref(loss),
                                                  _ptr(g, C.c_float) if g is not None else None))
        return loss.value, g

    def get_params(self):
        p = np.empty(self.info().n_params, np.float32)
        self.ctx._check(lib.geneo_model_get_params(self.h, _ptr(p, C.c_float)))
        return p

    def set_params(self, p):
        p = np.ascontiguousarray(p, dtype=np.float32)
        self.ctx._check(lib.geneo_model_set_params(self.ctx.h, self.h, _ptr(p, C.c_float)))

    def save(self, path):
        self.ctx._check(lib.geneo_model_save(self.h, str(path).encode()))
