"""Thin ctypes binding of ``liblgf.so`` (C ABI in ``include/lgf.h``).

Argument marshalling only: every step of a solve runs in the library's HIP kernels.  Torch is
used for device memory (tensors passed by ``data_ptr()``) and streams.  Loading fails loudly if
the library has not been built; there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblgf.so")

LGF_FP64_PLAIN = 0
LGF_FP32_REFINE = 1
LGF_BASE_SUPER = 0
LGF_BASE_BLOCK = 1
# forward operators of Plan.apply (lgf_op)
LAPLACIAN = 0
GRADIENT = 1
CURL = 2

EXPORTS = ["lgf_init", "lgf_plan", "lgf_plan_check", "lgf_solve", "lgf_apply", "lgf_solve_batch", "lgf_plan_get_info",
           "lgf_plan_destroy", "lgf_status_string", "lgf_green_eval", "lgf_green_table",
           "lgf_kernel_spectrum", "lgf_profile", "lgf_profile_read", "lgf_server_create", "lgf_server_submit", "lgf_server_poll",
           "lgf_server_wait_all", "lgf_server_stats", "lgf_server_destroy", "lgf_plan_set_mac_shape",
           "lgf_plan_set_near_shape", "lgf_server_submit_layout", "lgf_server_info", "lgf_workspace_poison", "lgf_layout_adapt",
           "lgf_solve_noalloc", "lgf_server_reset_stats"]
SCRATCH_BYTES = 64 << 20       # LGF_SCRATCH_BYTES: the allocation-free solve's workspace


class LgfError(RuntimeError):
    def __init__(self, code: int, what: str):
        self.code = code
        super().__init__(f"{what}: {status_string(code)} ({code})")


class Options(C.Structure):
    _fields_ = [("precision", C.c_int32), ("dc_iters", C.c_int32), ("autotune", C.c_int32),
                ("base_level", C.c_int32), ("hbm_budget", C.c_uint64)]


class PlanInfo(C.Structure):
    _fields_ = [("blocks", C.c_int64), ("unknowns", C.c_int64), ("refinement_levels", C.c_int32),
                ("max_octree_levels", C.c_int32), ("interactions", C.c_int64),
                ("fft_forward", C.c_int64), ("fft_inverse", C.c_int64), ("mac_rows", C.c_int64),
                ("workspace_bytes", C.c_int64), ("spectra", C.c_int64),
                ("super_forward", C.c_int64), ("super_inverse", C.c_int64),
                ("near_rows", C.c_int64), ("near_pairs", C.c_int64),
                ("mac_lds_tiles", C.c_int64), ("mac_lds_inner", C.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def load() -> C.CDLL:
    """Load the built library (raises if it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run paper_1911_10228_amd/build.py "
                          "(or __graft_entry__.build())")
    lib = C.CDLL(LIB_PATH)
    P, I32, I64, U64 = C.c_void_p, C.c_int32, C.c_int64, C.c_uint64
    sig = {
        "lgf_init": ([], I32),
        "lgf_plan": ([P, P, I64, I32, I32, P, P], I32),
        "lgf_plan_check": ([P, P, I64, I32, I32, P, P], I32),
        "lgf_solve": ([P, P, P, P], I32),
        "lgf_apply": ([P, I32, P, P, P], I32),
        "lgf_solve_batch": ([P, P, P, I32, P], I32),
        "lgf_plan_get_info": ([P, P], I32),
        "lgf_plan_destroy": ([P], I32),
        "lgf_status_string": ([I32], C.c_char_p),
        "lgf_green_eval": ([P, I64, P, P], I32),
        "lgf_green_table": ([P, P], I32),
        "lgf_kernel_spectrum": ([I32, I32, I32, I32, I32, P, P], I32),
        "lgf_profile": ([I32], I32),
        "lgf_profile_read": ([P, I32, P], I32),
        "lgf_server_create": ([U64, P, P], I32),
        "lgf_server_submit": ([P, P, P, P, P], I32),
        "lgf_server_poll": ([P, I64, P], I32),
        "lgf_server_wait_all": ([P], I32),
        "lgf_server_stats": ([P, P, P, P, P], I32),
        "lgf_server_destroy": ([P], I32),
        "lgf_plan_set_mac_shape": ([P, I32], I32),
        "lgf_plan_set_near_shape": ([P, I32], I32),
        "lgf_server_submit_layout": ([P, P, P, I64, I32, I32, P, P, P, P], I32),
        "lgf_server_info": ([P, P], I32),
        "lgf_workspace_poison": ([I32], I32),
        "lgf_layout_adapt": ([P, P, I64, I32, P, I32, C.c_double, P, P, I64, P, P], I32),
        "lgf_solve_noalloc": ([P, P, P, P], I32),
        "lgf_server_reset_stats": ([P], I32),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def status_string(code: int) -> str:
    return load().lgf_status_string(code).decode()


def _check(code: int, what: str):
    if code != 0:
        raise LgfError(code, what)


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr())


def init():
    _check(load().lgf_init(), "lgf_init")


class Plan:
    """A planned solve for a block layout (see include/lgf.h for the conventions)."""

    def __init__(self, blocks, levels, n_b: int, interp_order: int,
                 precision: int = LGF_FP64_PLAIN, dc_iters: int = 0, hbm_budget: int = 0,
                 base_level: int = 0, autotune: int = 0):
        lib = load()
        b = np.ascontiguousarray(np.asarray(blocks, dtype=np.int32).reshape(-1, 3))
        lv = np.ascontiguousarray(np.zeros(len(b), np.int32) if levels is None
                                  else np.asarray(levels, dtype=np.int32).reshape(-1))
        opt = Options(precision, dc_iters, autotune, base_level, hbm_budget)
        h = C.c_void_p()
        _check(lib.lgf_plan(b.ctypes.data, lv.ctypes.data, len(b), n_b, interp_order,
                            C.byref(opt), C.byref(h)), "lgf_plan")
        self._h = h
        self.n_b = n_b
        self.nblocks = len(b)
        self.precision = precision

    @property
    def handle(self):
        return self._h

    def info(self) -> dict:
        inf = PlanInfo()
        _check(load().lgf_plan_get_info(self._h, C.byref(inf)), "lgf_plan_get_info")
        return inf.as_dict()

    def solve(self, f, u, stream=None):
        """u <- solution for source f; both float64 CUDA tensors [n, N_b, N_b, N_b]."""
        self._check_field(f)
        self._check_field(u)
        _check(load().lgf_solve(self._h, _ptr(f), _ptr(u), _stream(stream)), "lgf_solve")

    def solve_noalloc(self, f, u, stream=None):
        """As solve, on the library's static workspace: allocates nothing (lgf_solve_noalloc)."""
        self._check_field(f)
        self._check_field(u)
        _check(load().lgf_solve_noalloc(self._h, _ptr(f), _ptr(u), _stream(stream)), "lgf_solve_noalloc")

    def apply(self, op: int, u, out, stream=None):
        """out <- op(u) on the layout's per-level lattice (LAPLACIAN, GRADIENT or CURL; float64
        CUDA tensors, [n, N_b, N_b, N_b] per component, 3 components where the op has them)."""
        import torch
        nin = 3 if op == CURL else 1
        nout = 1 if op == LAPLACIAN else 3
        m = self.nblocks * self.n_b ** 3
        for t, c in ((u, nin), (out, nout)):
            if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous() and t.numel() == c * m):
                raise ValueError(f"op {op}: fields must be contiguous float64 CUDA tensors of {c} x "
                                 "[n, N_b, N_b, N_b]")
        _check(load().lgf_apply(self._h, int(op), _ptr(u), _ptr(out), _stream(stream)), "lgf_apply")

    def set_mac_shape(self, shape: int):
        """Force the coarse-level MAC launch shape (diagnostics; 0 restores the chosen one)."""
        _check(load().lgf_plan_set_mac_shape(self._h, shape), "lgf_plan_set_mac_shape")

    def set_near_shape(self, shape: int):
        """Force the base-level super-block MAC launch shape (diagnostics; autotuned plans)."""
        _check(load().lgf_plan_set_near_shape(self._h, shape), "lgf_plan_set_near_shape")

    def _check_field(self, t):
        import torch
        if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()
                and t.numel() == self.nblocks * self.n_b ** 3):
            raise ValueError("fields must be contiguous float64 CUDA tensors [n, N_b, N_b, N_b]")

    def close(self):
        if getattr(self, "_h", None):
            _check(load().lgf_plan_destroy(self._h), "lgf_plan_destroy")
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def plan_check(blocks, levels, n_b: int, interp_order: int, precision: int = LGF_FP64_PLAIN,
               dc_iters: int = 0, base_level: int = 0, autotune: int = 0) -> dict:
    """Host-only plan build with validation of every kernel work item, including the launch-shape
    alternatives the autotuner would time (no GPU needed)."""
    b = np.ascontiguousarray(np.asarray(blocks, dtype=np.int32).reshape(-1, 3))
    lv = np.ascontiguousarray(np.zeros(len(b), np.int32) if levels is None
                              else np.asarray(levels, dtype=np.int32).reshape(-1))
    opt = Options(precision, dc_iters, autotune, base_level, 0)
    inf = PlanInfo()
    _check(load().lgf_plan_check(b.ctypes.data, lv.ctypes.data, len(b), n_b, interp_order,
                                 C.byref(opt), C.byref(inf)), "lgf_plan_check")
    return inf.as_dict()


class VectorPlan:
    """Vector Poisson problem L u_c = f_c, c < components, on one block layout through one plan:
    every solve advances all components together in shared launches (lgf_solve_batch with the
    plan once per component; each occurrence runs on a workspace of its own)."""

    def __init__(self, blocks, levels, n_b: int, interp_order: int, components: int = 3, **kw):
        self.plan = Plan(blocks, levels, n_b, interp_order, **kw)
        self.components = components

    def solve(self, f, u, stream=None):
        """u <- solution for f; both float64 CUDA tensors [components, n, N_b, N_b, N_b]."""
        if len(f) != self.components or len(u) != self.components:
            raise ValueError("one source and one solution field per component")
        solve_batch([self.plan] * self.components, [f[c] for c in range(len(f))],
                    [u[c] for c in range(len(u))], stream)

    def close(self):
        self.plan.close()


def solve_batch(plans, fs, us, stream=None):
    n = len(plans)
    for p, f, u in zip(plans, fs, us):
        p._check_field(f)
        p._check_field(u)
    hp = (C.c_void_p * n)(*[p.handle.value for p in plans])
    fp = (C.c_void_p * n)(*[f.data_ptr() for f in fs])
    up = (C.c_void_p * n)(*[u.data_ptr() for u in us])
    _check(load().lgf_solve_batch(hp, fp, up, n, _stream(stream)), "lgf_solve_batch")


def adapt_layout(blocks, levels, n_b: int, field, n_levels: int, alpha: float = 1.0 / 32,
                 stream=None):
    """One adaptation step of the refinement criterion on the GPU (lgf_layout_adapt): field is a
    float64 CUDA tensor [n, N_b, N_b, N_b] on the layout (blocks, levels).  Returns the new
    layout as numpy arrays (blocks [m, 3] int32, levels [m] int32)."""
    import torch
    b = torch.as_tensor(np.ascontiguousarray(np.asarray(blocks, np.int32).reshape(-1, 3))).cuda()
    lv = torch.as_tensor(np.ascontiguousarray(np.asarray(levels, np.int32).reshape(-1))).cuda()
    n = b.shape[0]
    if not (field.is_cuda and field.dtype == torch.float64 and field.is_contiguous()
            and field.numel() == n * n_b ** 3):
        raise ValueError("field must be a contiguous float64 CUDA tensor [n, N_b, N_b, N_b]")
    cap = 8 * n + 8
    while True:
        ob = torch.empty((cap, 3), dtype=torch.int32, device="cuda")
        ol = torch.empty((cap,), dtype=torch.int32, device="cuda")
        m = C.c_int64()
        code = load().lgf_layout_adapt(_ptr(b), _ptr(lv), n, n_b, _ptr(field), n_levels, alpha,
                                       _ptr(ob), _ptr(ol), cap, C.byref(m), _stream(stream))
        if code == -3 and m.value > cap:
            cap = m.value
            continue
        _check(code, "lgf_layout_adapt")
        return ob[:m.value].cpu().numpy(), ol[:m.value].cpu().numpy()


def green_eval(n_dev, out_dev, stream=None):
    """out[i] = G(n[i]) on the device: n int32 CUDA tensor [m, 3], out float64 [m]."""
    _check(load().lgf_green_eval(_ptr(n_dev), n_dev.shape[0], _ptr(out_dev), _stream(stream)),
           "lgf_green_eval")


def green_table(out_dev, stream=None):
    """Copy the dense FP64 table cube [101, 101, 101] into out (float64 CUDA tensor)."""
    _check(load().lgf_green_table(_ptr(out_dev), _stream(stream)), "lgf_green_table")


def kernel_spectrum(n_b, s, d, out_dev, stream=None):
    """FP64 half spectrum [2N_b, 2N_b, N_b+1] complex of G(s (d N_b + r)) into out (float64
    CUDA tensor [2N_b, 2N_b, N_b+1, 2]).  s = 0: the base-level super-block kernel of block
    side B = 2 N_b, G(d B + r) with |d| <= 1, into a tensor [2B, 2B, B+1, 2]."""
    _check(load().lgf_kernel_spectrum(n_b, s, int(d[0]), int(d[1]), int(d[2]), _ptr(out_dev),
                                      _stream(stream)), "lgf_kernel_spectrum")


class ProfileEntry(C.Structure):
    _fields_ = [("kind", C.c_int32), ("precision", C.c_int32), ("n_b", C.c_int32),
                ("mode", C.c_int32), ("launches", C.c_int64), ("ms", C.c_double),
                ("work", C.c_int64)]


KIND_NAMES = ["coarsen", "convert", "refine", "correct", "anterp", "fft_fwd", "mac", "fft_inv",
              "interp", "combine", "residual", "super_fwd", "near_mac", "super_inv"]


def profile(enable: bool):
    _check(load().lgf_profile(1 if enable else 0), "lgf_profile")


def profile_read() -> list:
    """Per (kernel, precision, N_b): launches, summed ms (HIP events), summed work."""
    arr = (ProfileEntry * 64)()
    n = C.c_int32()
    _check(load().lgf_profile_read(arr, 64, C.byref(n)), "lgf_profile_read")
    return [{"kernel": KIND_NAMES[e.kind], "precision": ["fp32", "fp64", "fp32/fp64"][e.precision],
             "n_b": e.n_b, "mode": e.mode, "launches": e.launches, "ms": e.ms, "work": e.work}
            for e in arr[:min(n.value, 64)]]


class ServerMemory(C.Structure):
    _fields_ = [("reserved_bytes", C.c_int64), ("in_use_bytes", C.c_int64),
                ("peak_in_use_bytes", C.c_int64), ("slots", C.c_int64), ("peak_slots", C.c_int64),
                ("binds", C.c_int64), ("plans_cached", C.c_int64), ("plan_hits", C.c_int64),
                ("plan_misses", C.c_int64), ("plan_ms_total", C.c_double), ("plan_ms_max", C.c_double)]


def workspace_poison(enable: bool):
    """Diagnostics: fill every workspace with NaN bytes when a plan's items are placed in it."""
    _check(load().lgf_workspace_poison(1 if enable else 0), "lgf_workspace_poison")


class Server:
    """Continuous-batching solve server (lgf_server_* in include/lgf.h)."""

    def __init__(self, hbm_budget: int = 0, stream=None):
        h = C.c_void_p()
        _check(load().lgf_server_create(hbm_budget, _stream(stream), C.byref(h)), "lgf_server_create")
        self._h = h

    def submit(self, plan: Plan, f, u) -> int:
        plan._check_field(f)
        plan._check_field(u)
        rid = C.c_int64()
        _check(load().lgf_server_submit(self._h, plan.handle, _ptr(f), _ptr(u), C.byref(rid)),
               "lgf_server_submit")
        return rid.value

    def submit_layout(self, blocks, levels, n_b: int, interp_order: int, f, u,
                      precision: int = LGF_FP64_PLAIN, dc_iters: int = 0, autotune: int = 0,
                      base_level: int = 0) -> int:
        """Submit by layout: the server takes the plan from its layout-keyed cache or builds it."""
        b = np.ascontiguousarray(np.asarray(blocks, dtype=np.int32).reshape(-1, 3))
        lv = np.ascontiguousarray(np.zeros(len(b), np.int32) if levels is None
                                  else np.asarray(levels, dtype=np.int32).reshape(-1))
        import torch
        m = len(b) * n_b ** 3
        for t in (f, u):
            if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous() and t.numel() == m):
                raise ValueError("fields must be contiguous float64 CUDA tensors [n, N_b, N_b, N_b]")
        opt = Options(precision, dc_iters, autotune, base_level, 0)
        rid = C.c_int64()
        _check(load().lgf_server_submit_layout(self._h, b.ctypes.data, lv.ctypes.data, len(b), n_b,
                                               interp_order, C.byref(opt), _ptr(f), _ptr(u),
                                               C.byref(rid)), "lgf_server_submit_layout")
        return rid.value

    def info(self) -> dict:
        m = ServerMemory()
        _check(load().lgf_server_info(self._h, C.byref(m)), "lgf_server_info")
        return {k: getattr(m, k) for k, _ in m._fields_}

    def reset_stats(self):
        """Start latency, throughput and memory statistics afresh (plans and memory stay)."""
        _check(load().lgf_server_reset_stats(self._h), "lgf_server_reset_stats")

    def poll(self, rid: int) -> bool:
        done = C.c_int32()
        _check(load().lgf_server_poll(self._h, rid, C.byref(done)), "lgf_server_poll")
        return bool(done.value)

    def wait_all(self):
        _check(load().lgf_server_wait_all(self._h), "lgf_server_wait_all")

    def stats(self) -> dict:
        p50, p99, pts = C.c_double(), C.c_double(), C.c_double()
        n = C.c_int64()
        _check(load().lgf_server_stats(self._h, C.byref(p50), C.byref(p99), C.byref(pts), C.byref(n)),
               "lgf_server_stats")
        return {"p50_us": p50.value, "p99_us": p99.value, "points_per_s": pts.value,
                "completed": n.value}

    def close(self):
        if getattr(self, "_h", None):
            _check(load().lgf_server_destroy(self._h), "lgf_server_destroy")
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
