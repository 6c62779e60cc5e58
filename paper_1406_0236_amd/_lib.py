"""ctypes binding of libaxs.so (include/axs.h).  Argument marshalling only: every
step of the computation runs in the HIP library.  Device vectors are torch
complex128 tensors of shape (nrhs, N); PyTorch supplies device memory (through
its caching allocator) and the stream."""
from __future__ import annotations

import atexit
import ctypes
import os
import weakref

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libaxs.so")

AXS_OK, AXS_NOT_CONVERGED = 0, 1
FP64, FP32 = 0, 1
SOLVE_FP64, SOLVE_MIXED = 0, 1
SOLVE_CERTIFY = 16   # flag: recompute the final residual with one more FP64 application
SOLVE_UNPRECONDITIONED = 32   # flag (FP64 mode): GMRES on (D + B) sigma = -v
SOLVE_RESTART_INNER = 64   # flag (mixed mode): inner GMRES runs start from scratch
_STATUS = {0: "AXS_OK", 1: "AXS_NOT_CONVERGED", -1: "AXS_EINVAL", -2: "AXS_EHIP", -3: "AXS_ENOMEM",
           -4: "AXS_ESTATE", -5: "AXS_ENONFINITE"}

_lib = None

# Live contexts and networks, in creation order (weak references).  They are
# closed in reverse order at interpreter exit, while torch (whose allocator
# frees their device memory) is still loaded: a network before the context it
# lives on.
_LIVE = []


def _register(obj):
    _LIVE.append(weakref.ref(obj))


@atexit.register
def _close_all():
    for ref in reversed(_LIVE):
        obj = ref()
        if obj is not None:
            try:
                obj.close()
            except Exception:
                pass


class AxsError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


class SolveInfo(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("inner_iterations", ctypes.c_int32),
                ("rel_residual", ctypes.c_double), ("seconds", ctypes.c_double),
                ("used_warm_start", ctypes.c_int32), ("converged", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)

EXPORTS = {
    # name: (restype, argtypes)
    "axs_create": (ctypes.c_int32, [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int, ctypes.c_void_p, ALLOC_FN,
                                    FREE_FN, ctypes.c_void_p]),
    "axs_destroy": (ctypes.c_int32, [ctypes.c_void_p]),
    "axs_last_error": (ctypes.c_char_p, [ctypes.c_void_p]),
    "axs_build_body": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                        ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ctypes.c_int)]),
    "axs_precompute_scattering": (ctypes.c_int32, [ctypes.c_void_p]),
    "axs_num_unknowns": (ctypes.c_int32, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64)]),
    "axs_node_geometry": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p]),
    "axs_modal_matrices": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_void_p]),
    "axs_apply_matvec": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                          ctypes.c_int]),
    "axs_apply_matvec_noalloc": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                                  ctypes.c_int]),
    "axs_apply_interbody": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                             ctypes.c_int]),
    "axs_apply_precond": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                           ctypes.c_int]),
    "axs_solve": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                   ctypes.c_int, ctypes.c_double, ctypes.c_int, ctypes.POINTER(SolveInfo)]),
    "axs_incident_plane_waves": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p]),
    "axs_incident_point_sources": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                                    ctypes.c_void_p]),
    "axs_eval_field": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                                        ctypes.c_int, ctypes.c_void_p]),
    "axs_far_field": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                                       ctypes.c_int, ctypes.c_void_p]),
    "axs_set_timing": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int]),
    "axs_last_timing": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p]),
    "axs_skeletonize": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_double, ctypes.c_double,
                                         ctypes.POINTER(ctypes.c_int64)]),
    "axs_skeletonize_points": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                                ctypes.c_uint64, ctypes.POINTER(ctypes.c_int64)]),
    "axs_skeleton_rank": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                                           ctypes.POINTER(ctypes.c_int)]),
    "axs_skeleton_nodes": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                                            ctypes.c_void_p]),
    "axs_skeleton_interp": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p]),
    "axs_solve_skeleton": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                            ctypes.c_int, ctypes.c_double, ctypes.c_int, ctypes.POINTER(SolveInfo)]),
    "axs_interbody_launch_shape": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                                                    ctypes.POINTER(ctypes.c_int)]),
    "axs_set_interbody_config": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                                  ctypes.c_int, ctypes.c_int]),
    "axs_set_target_bodies": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int]),
    "axs_mlp_create": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                        ctypes.POINTER(ctypes.c_void_p)]),
    "axs_mlp_destroy": (ctypes.c_int32, [ctypes.c_void_p]),
    "axs_mlp_num_params": (ctypes.c_int32, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64)]),
    "axs_mlp_set_params": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p]),
    "axs_mlp_get_params": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p]),
    "axs_mlp_forward": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int]),
    "axs_mlp_gradient": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                          ctypes.POINTER(ctypes.c_double), ctypes.c_void_p]),
    "axs_mlp_adam_step": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                           ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                           ctypes.POINTER(ctypes.c_double)]),
    "axs_mlp_train_epoch": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                             ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                                             ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                             ctypes.POINTER(ctypes.c_double)]),
    "axs_warm_start_size": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_int64)]),
    "axs_warm_start_encode": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                               ctypes.c_int, ctypes.c_void_p]),
    "axs_warm_start_decode": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                               ctypes.c_int, ctypes.c_void_p]),
    "axs_mlp_train": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                       ctypes.c_char_p, ctypes.c_void_p]),
    "axs_mlp_predict": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]),
}


def load():
    """Load libaxs.so; raises if it is missing (there is no fallback path)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                              "(the HIP library is required, there is no CPU fallback)")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in EXPORTS.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


class Context:
    """One solver context on one GPU (see include/axs.h for the semantics)."""

    def __init__(self, device: int = 0, use_torch_allocator: bool = True):
        import torch
        self._torch = torch
        self.lib = load()
        self.device = device
        self.stream = torch.cuda.current_stream(device)
        self._cb = None
        alloc, free = ALLOC_FN(0), FREE_FN(0)
        if use_torch_allocator:
            stream = self.stream

            def _alloc(nbytes, _user):
                try:
                    return torch.cuda.caching_allocator_alloc(int(nbytes), device, stream)
                except Exception:
                    return None

            delete = torch.cuda.caching_allocator_delete

            def _free(p, _user):
                try:
                    delete(p)
                except Exception:   # torch already torn down at interpreter exit
                    pass
            alloc, free = ALLOC_FN(_alloc), FREE_FN(_free)
            self._cb = (alloc, free)
        h = ctypes.c_void_p()
        st = self.lib.axs_create(ctypes.byref(h), device, ctypes.c_void_p(self.stream.cuda_stream), alloc, free, None)
        if st != AXS_OK:
            raise AxsError(st, "axs_create failed")
        self.h = h
        _register(self)
        self.N = 0
        self.max_nf = 0
        self.kappa = None

    def close(self):
        if getattr(self, "h", None):
            self.lib.axs_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st, soft_ok=False):
        if st == AXS_OK or (soft_ok and st == AXS_NOT_CONVERGED):
            return st
        raise AxsError(st, self.lib.axs_last_error(self.h).decode())

    def _vec(self, t, nrhs=None):
        torch = self._torch
        assert t.dtype == torch.complex128 and t.is_cuda and t.is_contiguous(), "complex128 contiguous cuda tensor"
        assert t.dim() == 2 and t.shape[1] == self.N, f"expected (nrhs, {self.N})"
        return ctypes.c_void_p(t.data_ptr()), t.shape[0]

    def _empty(self, nrhs, n=None):
        torch = self._torch
        return torch.empty((nrhs, self.N if n is None else n), dtype=torch.complex128, device=f"cuda:{self.device}")

    # -- setup ------------------------------------------------------------------
    def build_body(self, rz, drz, gw, n_panels, p, kappa, eta, M, centre, rot) -> int:
        rz = np.ascontiguousarray(rz, dtype=np.float64)
        drz = np.ascontiguousarray(drz, dtype=np.float64)
        gw = np.ascontiguousarray(gw, dtype=np.float64)
        centre = np.ascontiguousarray(centre, dtype=np.float64)
        rot = np.ascontiguousarray(rot, dtype=np.float64)
        bid = ctypes.c_int()
        self._check(self.lib.axs_build_body(self.h, _ptr(rz), _ptr(drz), _ptr(gw), int(n_panels), int(p),
                                            float(kappa), float(eta), int(M), _ptr(centre), _ptr(rot),
                                            ctypes.byref(bid)))
        n = ctypes.c_int64()
        self.lib.axs_num_unknowns(self.h, ctypes.byref(n))
        self.N = n.value
        self.max_nf = max(self.max_nf, 2 * int(M) + 1)
        self.kappa = float(kappa)
        return bid.value

    def add_workload(self, wl):
        for b in wl.bodies:
            c = b.contour
            self.build_body(c.rz, c.drz, c.gw, c.n_panels, c.p, wl.kappa, wl.eta, b.M, b.centre, b.rot)
        return self

    def precompute_scattering(self):
        self._check(self.lib.axs_precompute_scattering(self.h))

    def node_geometry(self) -> np.ndarray:
        out = np.empty((self.N, 7))
        self._check(self.lib.axs_node_geometry(self.h, _ptr(out)))
        return out

    def modal_matrices(self, body: int, which: int = 1, M: int = None, NG: int = None):
        """A~_m (which=0) or S_m (which=1) of body's shape as complex128 (M+1, NG, NG)."""
        out = self._torch.empty((M + 1, NG, NG), dtype=self._torch.complex128, device=f"cuda:{self.device}")
        self._check(self.lib.axs_modal_matrices(self.h, int(body), int(which), ctypes.c_void_p(out.data_ptr())))
        return out

    # -- operators ----------------------------------------------------------------
    def _apply(self, fn, x, precision, out):
        px, nrhs = self._vec(x)
        y = self._empty(nrhs) if out is None else out
        py, _ = self._vec(y)
        self._check(fn(self.h, px, py, nrhs, precision))
        return y

    def apply_matvec(self, sigma, precision=FP64, out=None):
        return self._apply(self.lib.axs_apply_matvec, sigma, precision, out)

    def apply_matvec_noalloc(self, sigma, precision=FP64, out=None):
        """axs_apply_matvec_noalloc: the operator with the library's static scratch (out is
        allocated here by torch unless given)."""
        return self._apply(self.lib.axs_apply_matvec_noalloc, sigma, precision, out)

    def apply_interbody(self, sigma, precision=FP64, out=None):
        return self._apply(self.lib.axs_apply_interbody, sigma, precision, out)

    def apply_precond(self, x, precision=FP64, out=None):
        return self._apply(self.lib.axs_apply_precond, x, precision, out)

    def solve(self, incident, sigma0=None, mode=SOLVE_FP64, tol=1e-7, max_iters=200, out=None, certify=False,
              precondition=True):
        """axs_solve; certify=True ORs AXS_SOLVE_CERTIFY into the mode, precondition=False
        AXS_SOLVE_UNPRECONDITIONED."""
        if certify:
            mode = int(mode) | SOLVE_CERTIFY
        if not precondition:
            mode = int(mode) | SOLVE_UNPRECONDITIONED
        pv, nrhs = self._vec(incident)
        p0 = self._vec(sigma0)[0] if sigma0 is not None else None
        sig = self._empty(nrhs) if out is None else out
        ps, _ = self._vec(sig)
        info = (SolveInfo * nrhs)()
        st = self.lib.axs_solve(self.h, pv, p0, ps, nrhs, int(mode), float(tol), int(max_iters), info)
        self._check(st, soft_ok=True)
        return sig, [i.as_dict() for i in info]

    # -- skeletonization (Sec. 5) ----------------------------------------------------
    def skeletonize(self, eps=1e-8, proxy_factor=2.0):
        """axs_skeletonize; returns the number of skeleton nodes."""
        n = ctypes.c_int64()
        self._check(self.lib.axs_skeletonize(self.h, float(eps), float(proxy_factor), ctypes.byref(n)))
        return n.value

    def skeletonize_points(self, eps=1e-8, proxy_factor=2.0, n_proxy=0, seed=1):
        """axs_skeletonize_points; returns the number of skeleton nodes."""
        n = ctypes.c_int64()
        self._check(self.lib.axs_skeletonize_points(self.h, float(eps), float(proxy_factor), int(n_proxy),
                                                    int(seed) & ((1 << 64) - 1), ctypes.byref(n)))
        return n.value

    def skeleton_nodes(self, body_id):
        """Ascending local node indices of a body's skeleton (numpy int32)."""
        cnt = ctypes.c_int(0)
        self._check(self.lib.axs_skeleton_nodes(self.h, int(body_id), ctypes.byref(cnt), None))
        out = np.zeros(max(cnt.value, 1), dtype=np.int32)
        self._check(self.lib.axs_skeleton_nodes(self.h, int(body_id), ctypes.byref(cnt), _ptr(out)))
        return out[:cnt.value]

    def skeleton_interp(self, body_id):
        """X^T of a body's point skeleton: complex128 tensor (k, N_G N_F) on the device
        (the transpose of the column-major k x n matrix the library returns)."""
        k, n = self.skeleton_rank(body_id)
        xt = self._torch.empty((n, k), dtype=self._torch.complex128, device=f"cuda:{self.device}")
        self._check(self.lib.axs_skeleton_interp(self.h, int(body_id), ctypes.c_void_p(xt.data_ptr())))
        return xt.T

    def skeleton_rank(self, body_id):
        """(skeleton rings, contour nodes) of a body's shape; for point skeletons
        (skeleton nodes, nodes)."""
        k, ng = ctypes.c_int(), ctypes.c_int()
        self._check(self.lib.axs_skeleton_rank(self.h, int(body_id), ctypes.byref(k), ctypes.byref(ng)))
        return k.value, ng.value

    def solve_skeleton(self, incident, mode=SOLVE_FP64, tol=1e-7, max_iters=200, out=None, certify=False):
        """axs_solve_skeleton; certify=True reports the full-system residual of the lifted sigma."""
        if certify:
            mode = int(mode) | SOLVE_CERTIFY
        pv, nrhs = self._vec(incident)
        sig = self._empty(nrhs) if out is None else out
        ps, _ = self._vec(sig)
        info = (SolveInfo * nrhs)()
        st = self.lib.axs_solve_skeleton(self.h, pv, ps, nrhs, int(mode), float(tol), int(max_iters), info)
        self._check(st, soft_ok=True)
        return sig, [i.as_dict() for i in info]

    # -- fields ---------------------------------------------------------------------
    def incident_plane_waves(self, dirs):
        d = np.ascontiguousarray(np.atleast_2d(dirs), dtype=np.float64)
        v = self._empty(d.shape[0])
        self._check(self.lib.axs_incident_plane_waves(self.h, _ptr(d), d.shape[0], ctypes.c_void_p(v.data_ptr())))
        return v

    def incident_point_sources(self, src, amp):
        s = np.ascontiguousarray(np.atleast_2d(src), dtype=np.float64)
        a = np.asarray(amp, dtype=np.complex128).reshape(-1)
        ab = np.ascontiguousarray(np.stack([a.real, a.imag], axis=1))
        v = self._empty(1)
        self._check(self.lib.axs_incident_point_sources(self.h, _ptr(s), _ptr(ab), s.shape[0],
                                                        ctypes.c_void_p(v.data_ptr())))
        return v

    def eval_field(self, sigma, targets):
        t = np.ascontiguousarray(np.atleast_2d(targets), dtype=np.float64)
        ps, nrhs = self._vec(sigma)
        u = self._empty(nrhs, t.shape[0])
        self._check(self.lib.axs_eval_field(self.h, ps, nrhs, _ptr(t), t.shape[0], ctypes.c_void_p(u.data_ptr())))
        return u

    def far_field(self, sigma, xhat):
        t = np.ascontiguousarray(np.atleast_2d(xhat), dtype=np.float64)
        ps, nrhs = self._vec(sigma)
        u = self._empty(nrhs, t.shape[0])
        self._check(self.lib.axs_far_field(self.h, ps, nrhs, _ptr(t), t.shape[0], ctypes.c_void_p(u.data_ptr())))
        return u

    # -- instrumentation --------------------------------------------------------------
    def set_timing(self, enable=True):
        self._check(self.lib.axs_set_timing(self.h, int(bool(enable))))

    def last_timing(self):
        ms = np.zeros(5)
        self._check(self.lib.axs_last_timing(self.h, _ptr(ms)))
        return {"interbody": ms[0], "dft_forward": ms[1], "modal_apply": ms[2], "dft_inverse": ms[3],
                "total": ms[4]}

    def set_interbody_config(self, precision, variant=0, targets_per_thread=0, block=0, splits=0):
        """Launch shape of the inter-body sum (0 = default): variant 1 = points, 2 = rings,
        3 = MFMA order, 4 = MFMA order with the FP16 multiply-accumulate (FP32 only; for both,
        targets_per_thread = groups of 16 targets per wavefront)."""
        self._check(self.lib.axs_set_interbody_config(self.h, int(precision), int(variant), int(targets_per_thread),
                                                      int(block), int(splits)))

    def set_target_bodies(self, first_body=0, count=0):
        """axs_set_target_bodies: the inter-body sum computes the rows of bodies
        [first_body, first_body + count) only (one GPU's share); (0, 0) = all."""
        self._check(self.lib.axs_set_target_bodies(self.h, int(first_body), int(count)))

    def interbody_launch_shape(self, precision, nrhs=1):
        """The resolved launch shape (variant, targets_per_thread, block, splits) for nrhs."""
        out = (ctypes.c_int * 4)()
        self._check(self.lib.axs_interbody_launch_shape(self.h, int(precision), int(nrhs), out))
        return tuple(int(v) for v in out)


class Mlp:
    """The warm-start network (include/axs.h, axs_mlp_*): FP32, on a context's
    device and stream.  X, T, Y are float32 cuda tensors [batch][n]."""

    def __init__(self, ctx: Context, n_in: int, width: int, depth: int, n_out: int):
        self.ctx = ctx
        self.lib = ctx.lib
        self.sizes = [n_in] + [width] * depth + [n_out]
        h = ctypes.c_void_p()
        st = self.lib.axs_mlp_create(ctx.h, n_in, width, depth, n_out, ctypes.byref(h))
        ctx._check(st)
        self.h = h
        _register(self)
        n = ctypes.c_int64()
        self.lib.axs_mlp_num_params(self.h, ctypes.byref(n))
        self.nparams = n.value

    def close(self):
        if getattr(self, "h", None):
            self.lib.axs_mlp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _f32(self, t, ncol):
        torch = self.ctx._torch
        assert t.dtype == torch.float32 and t.is_cuda and t.is_contiguous() and t.dim() == 2 and t.shape[1] == ncol
        return ctypes.c_void_p(t.data_ptr()), t.shape[0]

    def set_params(self, params):
        p = np.ascontiguousarray(params, dtype=np.float32)
        assert p.size == self.nparams
        self.ctx._check(self.lib.axs_mlp_set_params(self.h, _ptr(p)))

    def get_params(self):
        p = np.empty(self.nparams, dtype=np.float32)
        self.ctx._check(self.lib.axs_mlp_get_params(self.h, _ptr(p)))
        return p

    def forward(self, X):
        px, b = self._f32(X, self.sizes[0])
        Y = self.ctx._torch.empty((b, self.sizes[-1]), dtype=self.ctx._torch.float32, device=X.device)
        self.ctx._check(self.lib.axs_mlp_forward(self.h, px, ctypes.c_void_p(Y.data_ptr()), b))
        return Y

    def gradient(self, X, T):
        px, b = self._f32(X, self.sizes[0])
        pt, _ = self._f32(T, self.sizes[-1])
        g = self.ctx._torch.empty(self.nparams, dtype=self.ctx._torch.float32, device=X.device)
        loss = ctypes.c_double()
        self.ctx._check(self.lib.axs_mlp_gradient(self.h, px, pt, b, ctypes.byref(loss), ctypes.c_void_p(g.data_ptr())))
        return loss.value, g

    def adam_step(self, X, T, lr, beta1=0.9, beta2=0.999, eps=1e-8, want_loss=True):
        px, b = self._f32(X, self.sizes[0])
        pt, _ = self._f32(T, self.sizes[-1])
        loss = ctypes.c_double()
        self.ctx._check(self.lib.axs_mlp_adam_step(self.h, px, pt, b, float(lr), float(beta1), float(beta2),
                                                   float(eps), ctypes.byref(loss) if want_loss else None))
        return loss.value if want_loss else None

    def train_epoch(self, X, T, order, batch, lrs, beta1=0.9, beta2=0.999, eps=1e-8, want_loss=True):
        """len(lrs) Adam steps; step s trains on rows order[s*batch:(s+1)*batch] of X and T."""
        px, rows = self._f32(X, self.sizes[0])
        pt, rows_t = self._f32(T, self.sizes[-1])
        assert rows == rows_t
        o = np.ascontiguousarray(order, dtype=np.int32)
        lr = np.ascontiguousarray(lrs, dtype=np.float64)
        assert o.size == batch * lr.size
        loss = ctypes.c_double()
        self.ctx._check(self.lib.axs_mlp_train_epoch(self.h, px, pt, rows, _ptr(o), int(batch), int(lr.size),
                                                     _ptr(lr), float(beta1), float(beta2), float(eps),
                                                     ctypes.byref(loss) if want_loss else None))
        return loss.value if want_loss else None


def warm_start_size(ctx: Context, mmax: int) -> int:
    """axs_warm_start_size: floats per right-hand side of the warm-start layout."""
    n = ctypes.c_int64()
    ctx._check(ctx.lib.axs_warm_start_size(ctx.h, int(mmax), ctypes.byref(n)))
    return n.value


def _dirs(dirs, nrhs=None):
    d = np.ascontiguousarray(np.atleast_2d(dirs), dtype=np.float64)
    assert d.ndim == 2 and d.shape[1] == 3 and (nrhs is None or d.shape[0] == nrhs)
    return d


def warm_start_encode(ctx: Context, sigma, dirs, mmax: int):
    """axs_warm_start_encode: training targets (float32 [nrhs][P]) of densities sigma."""
    torch = ctx._torch
    ps, nrhs = ctx._vec(sigma)
    d = _dirs(dirs, nrhs)
    out = torch.empty((nrhs, warm_start_size(ctx, mmax)), dtype=torch.float32, device=sigma.device)
    ctx._check(ctx.lib.axs_warm_start_encode(ctx.h, ps, _ptr(d), nrhs, int(mmax), ctypes.c_void_p(out.data_ptr())))
    return out


def warm_start_decode(ctx: Context, Y, dirs, mmax: int):
    """axs_warm_start_decode: densities (complex128 [nrhs][N]) of the layout Y."""
    torch = ctx._torch
    d = _dirs(dirs)
    nrhs = d.shape[0]
    assert Y.dtype == torch.float32 and Y.is_cuda and Y.is_contiguous() and Y.shape == (nrhs, warm_start_size(ctx, mmax))
    out = ctx._empty(nrhs)
    ctx._check(ctx.lib.axs_warm_start_decode(ctx.h, ctypes.c_void_p(Y.data_ptr()), _ptr(d), nrhs, int(mmax),
                                             ctypes.c_void_p(out.data_ptr())))
    return out


def mlp_train(net: Mlp, X, Y, hparams: dict):
    """axs_mlp_train; X float32 cuda [S][4] = (d, k), Y float32 cuda [S][n_out];
    hparams as in include/axs.h.  Returns the per-epoch losses."""
    import json
    px, S = net._f32(X, net.sizes[0])
    py, S2 = net._f32(Y, net.sizes[-1])
    assert S == S2
    epochs = int(hparams.get("epochs", 200))
    losses = np.zeros(epochs, dtype=np.float64)
    text = json.dumps({k: float(v) for k, v in hparams.items()}).encode()
    net.ctx._check(net.lib.axs_mlp_train(net.h, px, py, S, text, _ptr(losses)))
    return losses


def mlp_predict(net: Mlp, ctx: Context, dirs, k_range, kappas=None):
    """axs_mlp_predict: the initial guess (complex128 [nrhs][N]) on ctx for plane waves dirs."""
    d = _dirs(dirs)
    nrhs = d.shape[0]
    kr = np.ascontiguousarray(k_range, dtype=np.float64)
    assert kr.shape == (2,)
    kp = None
    if kappas is not None:
        kp = np.ascontiguousarray(np.broadcast_to(np.asarray(kappas, dtype=np.float64), (nrhs,)))
    out = ctx._empty(nrhs)
    ctx._check(net.lib.axs_mlp_predict(net.h, ctx.h, _ptr(d), _ptr(kp) if kp is not None else None, nrhs, _ptr(kr),
                                       ctypes.c_void_p(out.data_ptr())))
    return out
