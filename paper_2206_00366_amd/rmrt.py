"""ctypes binding of librmrt.so (argument marshalling only).

Every step of the method runs inside the library's HIP kernels; this module
only converts Python values to the C structures of include/rmrt.h, passes
device pointers of torch tensors and the current HIP stream, and turns error
codes into exceptions.  It raises ImportError when the library is not built:
there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
# RMRT_LIBRARY selects another build of the library (the index-checked
# librmrt_checked.so); the default is the in-tree production build
LIB_PATH = os.environ.get("RMRT_LIBRARY") or os.path.join(_HERE, "librmrt.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: run `python -m paper_2206_00366_amd.build` first")

# One HIP runtime per process: torch bundles its own libamdhip64.so.7, so it is
# loaded first and librmrt.so binds to that same runtime (loading the library
# first would pull a second runtime from /opt/rocm into the process).
import torch  # noqa: E402,F401

_lib = C.CDLL(LIB_PATH)

# ---- constants (include/rmrt.h) ----
OK, EINVAL, EUNSUPPORTED, EHIP, ENONFINITE, ENOMEM = 0, -1, -2, -3, -4, -5
Q9, Q19, Q27, Q5, Q7 = 0, 1, 2, 3, 4
NSE, NCDE = 0, 1
F64, F32DEV, F16DEV = 0, 1, 2
AB, AA = 0, 1
OUT_F64, OUT_F32 = 0, 1
LAUNCH_XCD_ORDER, LAUNCH_PERSISTENT, LAUNCH_WIDE_TILES, LAUNCH_BUFFER_OFFSETS = 1, 2, 4, 8
LAUNCH_ALTERNATE_ORDER = 16
LAUNCH_XCD_CHUNKS = 32
GRAD_STRAIN, GRAD_STRESS, GRAD_PHI = 0, 1, 2
WALL_XM, WALL_XP, WALL_YM, WALL_YP, WALL_ZM, WALL_ZP = 1, 2, 4, 8, 16, 32

LATTICES = {"Q9": Q9, "Q19": Q19, "Q27": Q27, "Q5": Q5, "Q7": Q7}
EQUATIONS = {"NSE": NSE, "NCDE": NCDE}
STORAGES = {"f64": F64, "f32dev": F32DEV, "f16dev": F16DEV}
PATTERNS = {"AB": AB, "AA": AA}
Q_OF = {Q9: 9, Q19: 19, Q27: 27, Q5: 5, Q7: 7}
DIM_OF = {Q9: 2, Q19: 3, Q27: 3, Q5: 2, Q7: 3}


class Params(C.Structure):
    _fields_ = [
        ("lattice", C.c_int), ("equation", C.c_int), ("storage", C.c_int), ("pattern", C.c_int),
        ("n", C.c_int * 3), ("dx", C.c_double * 3), ("dt", C.c_double), ("cs2", C.c_double),
        ("nu", C.c_double), ("nu_b", C.c_double), ("s_hi", C.c_double), ("w_corner", C.c_double),
        ("D0", C.c_double), ("D2", C.c_double), ("adv", C.c_double * 3), ("force", C.c_double * 3),
        ("source", C.c_double), ("rho0", C.c_double), ("wall_faces", C.c_uint), ("check_every", C.c_int),
        ("incompressible", C.c_int), ("nu_tensor", C.c_double * 6), ("nu_b_axis", C.c_double * 3),
        ("gamma0", C.c_int), ("diffusive", C.c_int), ("c_zero", C.c_int), ("central", C.c_int), ("hermite", C.c_int),
        ("bhll", C.c_int),
    ]


class Derived(C.Structure):
    _fields_ = [
        ("q", C.c_int), ("d", C.c_int), ("c", C.c_double * 3), ("cs2", C.c_double),
        ("w", C.c_double * 27), ("s_nu", C.c_double), ("s_s", C.c_double * 3), ("s_b", C.c_double * 3),
        ("s_hi", C.c_double), ("Sbar2", (C.c_double * 3) * 3), ("nu_b", C.c_double),
        ("s_pair", C.c_double * 3),
    ]


_vp = C.c_void_p
_sig = {
    "rmrt_last_error": (C.c_char_p, []),
    "rmrt_version": (C.c_char_p, []),
    "rmrt_stream_copy": (C.c_int, [_vp, _vp, C.c_size_t, _vp]),
    "rmrt_derive": (C.c_int, [C.POINTER(Params), C.POINTER(Derived)]),
    "rmrt_population_bytes": (C.c_int, [C.POINTER(Params), C.POINTER(C.c_size_t)]),
    "rmrt_init": (C.c_int, [C.POINTER(_vp), C.POINTER(Params), _vp, _vp, _vp, _vp, _vp, C.c_int, _vp]),
    "rmrt_set_fields": (C.c_int, [_vp, _vp, _vp, C.c_int, _vp]),
    "rmrt_set_source_fields": (C.c_int, [_vp, _vp, _vp, _vp]),
    "rmrt_step": (C.c_int, [_vp, C.c_int, _vp]),
    "rmrt_step_prepare": (C.c_int, [_vp, C.c_int, _vp]),
    "rmrt_moments": (C.c_int, [_vp, _vp, _vp, C.c_int, _vp]),
    "rmrt_populations": (C.c_int, [_vp, _vp, _vp]),
    "rmrt_reduce": (C.c_int, [_vp, C.POINTER(C.c_double), _vp]),
    "rmrt_reduce_noalloc": (C.c_int, [_vp, _vp, _vp]),
    "rmrt_residual": (C.c_int, [_vp, C.POINTER(C.c_double), _vp]),
    "rmrt_steps_taken": (C.c_int, [_vp, C.POINTER(C.c_longlong)]),
    "rmrt_checkpoint_bytes": (C.c_int, [_vp, C.POINTER(C.c_size_t)]),
    "rmrt_checkpoint_save": (C.c_int, [_vp, _vp, _vp]),
    "rmrt_checkpoint_restore": (C.c_int, [_vp, _vp, _vp]),
    "rmrt_set_launch": (C.c_int, [_vp, C.c_int, C.c_int]),
    "rmrt_get_launch": (C.c_int, [_vp, C.POINTER(C.c_int), C.POINTER(C.c_int)]),
    "rmrt_tune": (C.c_int, [_vp, C.c_int, _vp, C.POINTER(C.c_int)]),
    "rmrt_free": (C.c_int, [_vp]),
    "rmrt_batch_create": (C.c_int, [C.POINTER(_vp), C.c_int, C.POINTER(Params), C.POINTER(_vp),
                                     C.POINTER(_vp), C.POINTER(_vp), _vp]),
    "rmrt_batch_domain": (C.c_int, [_vp, C.c_int, C.POINTER(_vp)]),
    "rmrt_batch_autotune": (C.c_int, [_vp, C.c_int, _vp, C.POINTER(C.c_int)]),
    "rmrt_batch_set_config": (C.c_int, [_vp, C.c_int]),
    "rmrt_batch_set_group_bytes": (C.c_int, [_vp, C.c_size_t]),
    "rmrt_batch_get_group_bytes": (C.c_int, [_vp, C.POINTER(C.c_size_t), C.POINTER(C.c_int)]),
    "rmrt_preflight": (C.c_int, [_vp, C.POINTER(C.c_double), C.c_int, C.POINTER(C.c_double), _vp]),
    "rmrt_checked_build": (C.c_int, []),
    "rmrt_checked_violations": (C.c_int, [_vp, C.POINTER(C.c_uint), _vp]),
    "rmrt_checked_set_limit": (C.c_int, [_vp, C.c_uint, _vp]),
    "rmrt_batch_set_xcd_chunks": (C.c_int, [_vp, C.c_int]),
    "rmrt_batch_get_xcd_chunks": (C.c_int, [_vp, C.POINTER(C.c_int), C.POINTER(C.c_int)]),
    "rmrt_batch_num_configs": (C.c_int, []),
    "rmrt_batch_config_info": (C.c_int, [C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int),
                                          C.POINTER(C.c_int), C.POINTER(C.c_int)]),
    "rmrt_local_gradients": (C.c_int, [_vp, C.c_int, _vp, C.c_int, _vp]),
    "rmrt_step_local": (C.c_int, [_vp, C.c_int, _vp, C.c_int, _vp]),
    "rmrt_batch_step": (C.c_int, [_vp, C.c_int, _vp]),
    "rmrt_batch_step_prepare": (C.c_int, [_vp, C.c_int, _vp]),
    "rmrt_batch_residual": (C.c_int, [_vp, C.POINTER(C.c_double), _vp]),
    "rmrt_batch_free": (C.c_int, [_vp]),
    "rmrt_nn_conv_forward": (C.c_int, [_vp, _vp, _vp, _vp, _vp, _vp, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int,
                                       C.c_int, C.c_int, _vp]),
    "rmrt_nn_flip_weights": (C.c_int, [_vp, _vp, C.c_int, C.c_int, _vp]),
    "rmrt_nn_wgrad_scratch_floats": (C.c_size_t, [C.c_int, C.c_int, C.c_int, C.c_int, C.c_int]),
    "rmrt_nn_conv_backward_weight": (C.c_int, [_vp, _vp, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, _vp,
                                               _vp, _vp, C.c_size_t, _vp]),
    "rmrt_nn_masked_mse": (C.c_int, [_vp, C.c_int, _vp, _vp, C.c_long, C.c_int, _vp, _vp, _vp, _vp, _vp]),
    "rmrt_nn_adam": (C.c_int, [_vp, _vp, _vp, _vp, _vp, C.c_long, C.c_float, C.c_float, C.c_float, C.c_float,
                               C.c_int, _vp]),
    "rmrt_nn_to_bf16": (C.c_int, [_vp, _vp, C.c_long, _vp]),
    "rmrt_nn_features": (C.c_int, [_vp, _vp, C.c_int, C.c_int, C.c_int, C.c_int, C.c_float, C.c_float, _vp,
                                   C.c_int, _vp, _vp]),
    "rmrt_nn_targets": (C.c_int, [_vp, _vp, _vp, C.c_int, C.c_int, C.c_int, C.c_int, C.c_float, C.c_float,
                                  C.c_float, _vp, _vp, _vp]),
    "rmrt_nn_warm_fields": (C.c_int, [_vp, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_float, C.c_float,
                                      C.c_float, _vp, _vp, _vp, _vp]),
}
for _name, (_res, _args) in _sig.items():
    _fn = getattr(_lib, _name)
    _fn.restype = _res
    _fn.argtypes = _args

EXPORTED = tuple(_sig)


class RMRTError(RuntimeError):
    def __init__(self, code, where):
        msg = _lib.rmrt_last_error().decode()
        super().__init__(f"{where} returned {code}: {msg}")
        self.code = code


def _check(code, where):
    if code != OK:
        raise RMRTError(code, where)


def lib():
    return _lib


def checked_build() -> bool:
    """True when the loaded library tests every neighbour index (librmrt_checked.so)."""
    return bool(_lib.rmrt_checked_build())


def version() -> str:
    return _lib.rmrt_version().decode()


def stream_copy(dst, src):
    """HBM probe: copy src into dst (torch tensors of equal byte size) on the current stream."""
    nbytes = src.numel() * src.element_size()
    _check(_lib.rmrt_stream_copy(_ptr(dst), _ptr(src), nbytes, _stream()), "rmrt_stream_copy")


def make_params(lattice="Q9", equation="NSE", storage="f64", pattern="AB", n=(8, 8, 1),
                dx=(1.0, 1.0, 1.0), dt=1.0, cs2=-1.0, nu=0.1, nu_b=-1.0, s_hi=-1.0, w_corner=-1.0,
                D0=0.0, D2=0.0, adv=(0.0, 0.0, 0.0), force=(0.0, 0.0, 0.0), source=0.0, rho0=1.0,
                wall_faces=0, check_every=0, incompressible=False, nu_tensor=None, nu_b_axis=None,
                gamma0=False, diffusive=False, c_zero=False, central=False, hermite=False, bhll=False, **_ignored) -> Params:
    def pad3(v, fill):
        v = list(v) + [fill] * 3
        return v[:3]

    p = Params()
    p.lattice = LATTICES[lattice] if isinstance(lattice, str) else int(lattice)
    p.equation = EQUATIONS[equation] if isinstance(equation, str) else int(equation)
    p.storage = STORAGES[storage] if isinstance(storage, str) else int(storage)
    p.pattern = PATTERNS[pattern] if isinstance(pattern, str) else int(pattern)
    p.n[:] = [int(v) for v in pad3(n, 1)]
    p.dx[:] = [float(v) for v in pad3(dx, 1.0)]
    p.dt, p.cs2, p.nu, p.nu_b, p.s_hi, p.w_corner = float(dt), float(cs2), float(nu), float(nu_b), float(s_hi), float(w_corner)
    p.D0, p.D2 = float(D0), float(D2)
    p.adv[:] = [float(v) for v in pad3(adv, 0.0)]
    p.force[:] = [float(v) for v in pad3(force, 0.0)]
    p.source, p.rho0 = float(source), float(rho0)
    p.wall_faces = int(wall_faces)
    p.check_every = int(check_every)
    p.incompressible = int(bool(incompressible))
    p.gamma0 = int(bool(gamma0))
    p.diffusive = int(bool(diffusive))
    p.c_zero = int(bool(c_zero))
    p.central = int(bool(central))
    p.hermite = int(bool(hermite))
    p.bhll = int(bool(bhll))
    p.nu_tensor[:] = [float(v) for v in (nu_tensor if nu_tensor is not None else [-1.0] * 6)]
    p.nu_b_axis[:] = [float(v) for v in (nu_b_axis if nu_b_axis is not None else [-1.0] * 3)]
    return p


def derive(params: Params) -> Derived:
    out = Derived()
    _check(_lib.rmrt_derive(C.byref(params), C.byref(out)), "rmrt_derive")
    return out


def population_bytes(params: Params) -> int:
    b = C.c_size_t()
    _check(_lib.rmrt_population_bytes(C.byref(params), C.byref(b)), "rmrt_population_bytes")
    return b.value


def preflight(params: Params, u0=None, steps=400) -> float:
    """Largest per-step growth of a small perturbation of the uniform state
    (rho0, u0) under the parameter set's step (rmrt_preflight); > 1: unstable."""
    g = C.c_double()
    uu = None if u0 is None else (C.c_double * 3)(*[float(x) for x in u0] + [0.0] * (3 - len(u0)))
    _check(_lib.rmrt_preflight(C.byref(params), uu, int(steps), C.byref(g), _stream()), "rmrt_preflight")
    return g.value


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


_STORE_DTYPES = {F64: "float64", F32DEV: "float32", F16DEV: "float16"}


class Domain:
    """One domain: owns torch tensors for its buffers and an rmrt_ctx."""

    def __init__(self, params: Params, rho, u=None, solid=None, with_fne=False, device="cuda"):
        import torch
        self.params = params
        self.q = Q_OF[params.lattice]
        self.d = DIM_OF[params.lattice]
        self.N = params.n[0] * params.n[1] * params.n[2]
        dt = getattr(torch, _STORE_DTYPES[params.storage])
        esize = torch.empty(0, dtype=dt).element_size()
        self.f0 = torch.empty(population_bytes(params) // esize, dtype=dt, device=device)
        self.f1 = torch.empty_like(self.f0) if params.pattern == AB else None
        self.solid = None if solid is None else torch.as_tensor(solid, dtype=torch.uint8, device=device).contiguous()
        rho = torch.as_tensor(rho, dtype=torch.float64, device=device).contiguous()
        u = None if u is None else torch.as_tensor(u, dtype=torch.float64, device=device).contiguous()
        self._ctx = C.c_void_p()
        _check(_lib.rmrt_init(C.byref(self._ctx), C.byref(params), _ptr(self.f0), _ptr(self.f1),
                              _ptr(self.solid), _ptr(rho), _ptr(u), int(with_fne), _stream()), "rmrt_init")
        self._keep = (rho, u)

    @classmethod
    def _borrow(cls, ctx, params, f0, f1, solid):
        self = cls.__new__(cls)
        self.params = params
        self.q = Q_OF[params.lattice]
        self.d = DIM_OF[params.lattice]
        self.N = params.n[0] * params.n[1] * params.n[2]
        self.f0, self.f1, self.solid = f0, f1, solid
        self._ctx = ctx
        self._borrowed = True
        return self

    def set_fields(self, rho, u=None, with_fne=False):
        import torch
        rho = torch.as_tensor(rho, dtype=torch.float64, device=self.f0.device).contiguous()
        u = None if u is None else torch.as_tensor(u, dtype=torch.float64, device=self.f0.device).contiguous()
        _check(_lib.rmrt_set_fields(self._ctx, _ptr(rho), _ptr(u), int(with_fne), _stream()), "rmrt_set_fields")
        self._keep = (rho, u)

    def step(self, n=1):
        _check(_lib.rmrt_step(self._ctx, int(n), _stream()), "rmrt_step")

    def prepare(self, n):
        """Capture the graphs of step(n) now (no steps are taken)."""
        _check(_lib.rmrt_step_prepare(self._ctx, int(n), _stream()), "rmrt_step_prepare")

    def source_dtype(self):
        import torch
        return torch.float64 if self.params.storage == F64 else torch.float32

    def set_source_fields(self, S=None, F=None):
        """Attach per-node source fields (device tensors of source_dtype(); S: N
        values, F: (d, N)) or detach with both None.  The tensors are kept
        referenced; update them in place between steps for time-varying sources."""
        import torch
        dt = self.source_dtype()

        def dev(a, shape):
            if a is None:
                return None
            t = torch.as_tensor(a, device=self.f0.device)
            if t.dtype != dt or not t.is_contiguous():
                raise ValueError(f"source fields must be contiguous {dt} tensors")
            return t.view(shape)
        self._src = (dev(S, (self.N,)), dev(F, (self.d, self.N)))
        _check(_lib.rmrt_set_source_fields(self._ctx, _ptr(self._src[0]), _ptr(self._src[1]), _stream()),
               "rmrt_set_source_fields")

    def moments(self, out_dtype=OUT_F64, with_u=True):
        import torch
        dt = torch.float64 if out_dtype == OUT_F64 else torch.float32
        rho = torch.empty(self.N, dtype=dt, device=self.f0.device)
        u = torch.empty(self.d * self.N, dtype=dt, device=self.f0.device) if with_u else None
        _check(_lib.rmrt_moments(self._ctx, _ptr(rho), _ptr(u), int(out_dtype), _stream()), "rmrt_moments")
        return rho, (u.view(self.d, self.N) if u is not None else None)

    def local_gradients(self, kind=GRAD_STRAIN, out_dtype=OUT_F64):
        """Strain rate / stress components (xx, yy, [zz,] xy, [xz, yz]) or grad phi, shape (ncomp, N)."""
        import torch
        dt = torch.float64 if out_dtype == OUT_F64 else torch.float32
        nc = self.d if kind == GRAD_PHI else self.d * (self.d + 1) // 2
        out = torch.empty(nc * self.N, dtype=dt, device=self.f0.device)
        _check(_lib.rmrt_local_gradients(self._ctx, int(kind), _ptr(out), int(out_dtype), _stream()),
               "rmrt_local_gradients")
        return out.view(nc, self.N)

    def step_local(self, kind=GRAD_STRAIN, out_dtype=OUT_F32):
        """One step fused with the local outputs of the state it starts from, shape (ncomp, N)."""
        import torch
        dt = torch.float64 if out_dtype == OUT_F64 else torch.float32
        nc = self.d if kind == GRAD_PHI else self.d * (self.d + 1) // 2
        out = torch.empty(nc * self.N, dtype=dt, device=self.f0.device)
        _check(_lib.rmrt_step_local(self._ctx, int(kind), _ptr(out), int(out_dtype), _stream()), "rmrt_step_local")
        return out.view(nc, self.N)

    def populations(self):
        import torch
        out = torch.empty(self.q * self.N, dtype=torch.float64, device=self.f0.device)
        _check(_lib.rmrt_populations(self._ctx, _ptr(out), _stream()), "rmrt_populations")
        return out.view(self.q, self.N)

    def reduce(self):
        out = (C.c_double * 4)()
        _check(_lib.rmrt_reduce(self._ctx, out, _stream()), "rmrt_reduce")
        return list(out)

    def residual(self):
        r = C.c_double()
        _check(_lib.rmrt_residual(self._ctx, C.byref(r), _stream()), "rmrt_residual")
        return r.value

    def checkpoint(self, device="cuda"):
        """The context's checkpoint in a new uint8 tensor (device or "cpu")."""
        import torch
        n = C.c_size_t()
        _check(_lib.rmrt_checkpoint_bytes(self._ctx, C.byref(n)), "rmrt_checkpoint_bytes")
        buf = torch.empty(n.value, dtype=torch.uint8, device=device)
        _check(_lib.rmrt_checkpoint_save(self._ctx, _ptr(buf), _stream()), "rmrt_checkpoint_save")
        return buf

    def restore(self, buf):
        _check(_lib.rmrt_checkpoint_restore(self._ctx, _ptr(buf), _stream()), "rmrt_checkpoint_restore")

    def checked_violations(self):
        """Neighbour indices found out of range so far (checked builds only)."""
        n = C.c_uint()
        _check(_lib.rmrt_checked_violations(self._ctx, C.byref(n), _stream()), "rmrt_checked_violations")
        return n.value

    def checked_set_limit(self, limit):
        """Lower the node bound of the index checks (a test of the checks; checked builds only)."""
        _check(_lib.rmrt_checked_set_limit(self._ctx, int(limit), _stream()), "rmrt_checked_set_limit")

    def steps_taken(self):
        s = C.c_longlong()
        _check(_lib.rmrt_steps_taken(self._ctx, C.byref(s)), "rmrt_steps_taken")
        return s.value

    def set_launch(self, blocks_per_cu, flags=0):
        _check(_lib.rmrt_set_launch(self._ctx, int(blocks_per_cu), int(flags)), "rmrt_set_launch")

    def get_launch(self):
        b, x = C.c_int(), C.c_int()
        _check(_lib.rmrt_get_launch(self._ctx, C.byref(b), C.byref(x)), "rmrt_get_launch")
        return b.value, x.value

    def tune(self, steps=20):
        b = C.c_int()
        _check(_lib.rmrt_tune(self._ctx, int(steps), _stream(), C.byref(b)), "rmrt_tune")
        return b.value

    def close(self):
        if getattr(self, "_borrowed", False):
            return
        if self._ctx:
            _lib.rmrt_free(self._ctx)
            self._ctx = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Many domains stepped through one tile list: one launch per step, or one per domain group
    and step (rmrt_batch_set_group_bytes), graph-replayed."""

    def __init__(self, params_list, solids=None, device="cuda"):
        import torch
        nd = len(params_list)
        self.params = list(params_list)
        arr = (Params * nd)(*self.params)
        self.f0, self.f1, self.solids = [], [], []
        for k, p in enumerate(self.params):
            dt = getattr(torch, _STORE_DTYPES[p.storage])
            esize = torch.empty(0, dtype=dt).element_size()
            self.f0.append(torch.empty(population_bytes(p) // esize, dtype=dt, device=device))
            self.f1.append(torch.empty_like(self.f0[-1]) if p.pattern == AB else None)
            s = None if solids is None or solids[k] is None else torch.as_tensor(
                solids[k], dtype=torch.uint8, device=device).contiguous()
            self.solids.append(s)
        f0 = (C.c_void_p * nd)(*[t.data_ptr() for t in self.f0])
        f1 = (C.c_void_p * nd)(*[t.data_ptr() for t in self.f1]) if self.params[0].pattern == AB else None
        sol = (C.c_void_p * nd)(*[0 if s is None else s.data_ptr() for s in self.solids])
        self._b = C.c_void_p()
        _check(_lib.rmrt_batch_create(C.byref(self._b), nd, arr, f0, f1, sol, _stream()), "rmrt_batch_create")
        self.domains = []
        for k in range(nd):
            ctx = C.c_void_p()
            _check(_lib.rmrt_batch_domain(self._b, k, C.byref(ctx)), "rmrt_batch_domain")
            self.domains.append(Domain._borrow(ctx, self.params[k], self.f0[k], self.f1[k], self.solids[k]))

    def step(self, n=1):
        _check(_lib.rmrt_batch_step(self._b, int(n), _stream()), "rmrt_batch_step")

    def prepare(self, n):
        """Capture the graphs of step(n) now (no steps are taken)."""
        _check(_lib.rmrt_batch_step_prepare(self._b, int(n), _stream()), "rmrt_batch_step_prepare")

    def autotune(self, steps=10):
        ch = C.c_int()
        _check(_lib.rmrt_batch_autotune(self._b, int(steps), _stream(), C.byref(ch)), "rmrt_batch_autotune")
        return ch.value

    def set_config(self, cfg):
        _check(_lib.rmrt_batch_set_config(self._b, int(cfg)), "rmrt_batch_set_config")

    def set_group_bytes(self, nbytes):
        """Domain groups of at most nbytes of populations stepped one after the other (0: one group)."""
        _check(_lib.rmrt_batch_set_group_bytes(self._b, C.c_size_t(int(nbytes))), "rmrt_batch_set_group_bytes")

    def group_bytes(self):
        """(group size limit in bytes, number of groups)."""
        nb, ng = C.c_size_t(), C.c_int()
        _check(_lib.rmrt_batch_get_group_bytes(self._b, C.byref(nb), C.byref(ng)), "rmrt_batch_get_group_bytes")
        return nb.value, ng.value

    def set_xcd_chunks(self, mode):
        """1: XCD chunks for the groups whose rows straddle cache lines; 0: never."""
        _check(_lib.rmrt_batch_set_xcd_chunks(self._b, int(mode)), "rmrt_batch_set_xcd_chunks")

    def xcd_chunks(self):
        """(mode, number of groups launched with XCD chunks under mode 1)."""
        m, g = C.c_int(), C.c_int()
        _check(_lib.rmrt_batch_get_xcd_chunks(self._b, C.byref(m), C.byref(g)), "rmrt_batch_get_xcd_chunks")
        return m.value, g.value

    def residuals(self):
        n = len(self.domains)
        out = (C.c_double * n)()
        code = _lib.rmrt_batch_residual(self._b, out, _stream())
        if code not in (OK, ENONFINITE):
            _check(code, "rmrt_batch_residual")
        return list(out)

    @staticmethod
    def configs():
        out = []
        for k in range(_lib.rmrt_batch_num_configs()):
            t, n, b, p, w = C.c_int(), C.c_int(), C.c_int(), C.c_int(), C.c_int()
            _check(_lib.rmrt_batch_config_info(k, C.byref(t), C.byref(n), C.byref(b), C.byref(p), C.byref(w)),
                   "rmrt_batch_config_info")
            out.append((t.value, n.value, b.value, p.value, w.value))
        return out

    def close(self):
        if self._b:
            _lib.rmrt_batch_free(self._b)
            self._b = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------------------
# Surrogate kernels (bf16 tensors are torch.bfloat16 / int16 views)
# ---------------------------------------------------------------------------
NN_EPI_NONE, NN_EPI_SILU, NN_EPI_SILU_GRAD = 0, 1, 2


def nn_conv_forward(x, w, bias, y_pre, a_out, aux, dil, epilogue):
    B, H, W, Cin = x.shape
    Cout = w.shape[0]
    _check(_lib.rmrt_nn_conv_forward(_ptr(x), _ptr(w), _ptr(bias), _ptr(y_pre), _ptr(a_out), _ptr(aux),
                                     B, H, W, Cin, Cout, int(dil), int(epilogue), _stream()), "rmrt_nn_conv_forward")


def nn_flip_weights(w, wt):
    _check(_lib.rmrt_nn_flip_weights(_ptr(w), _ptr(wt), w.shape[0], w.shape[3], _stream()), "rmrt_nn_flip_weights")


def nn_wgrad_scratch_floats(B, H, W, Cin, Cout):
    return _lib.rmrt_nn_wgrad_scratch_floats(B, H, W, Cin, Cout)


def nn_conv_backward_weight(x, dy, dil, dw, db, scratch):
    B, H, W, Cin = x.shape
    Cout = dy.shape[3]
    _check(_lib.rmrt_nn_conv_backward_weight(_ptr(x), _ptr(dy), B, H, W, Cin, Cout, int(dil), _ptr(dw), _ptr(db),
                                             _ptr(scratch), scratch.numel(), _stream()),
           "rmrt_nn_conv_backward_weight")


def nn_masked_mse(out, target, weight, dout, scratch, inv_den, loss):
    Cs = out.shape[-1]
    P = out.numel() // Cs
    C_used = target.shape[-1]
    _check(_lib.rmrt_nn_masked_mse(_ptr(out), Cs, _ptr(target), _ptr(weight), P, C_used, _ptr(dout), _ptr(scratch),
                                   _ptr(inv_den), _ptr(loss), _stream()), "rmrt_nn_masked_mse")


def nn_adam(w, w_bf16, g, m, v, lr, t, b1=0.9, b2=0.999, eps=1e-8):
    _check(_lib.rmrt_nn_adam(_ptr(w), _ptr(w_bf16), _ptr(g), _ptr(m), _ptr(v), w.numel(), float(lr), float(b1),
                             float(b2), float(eps), int(t), _stream()), "rmrt_nn_adam")


def nn_to_bf16(src, dst):
    _check(_lib.rmrt_nn_to_bf16(_ptr(src), _ptr(dst), src.numel(), _stream()), "rmrt_nn_to_bf16")


def nn_features(solid, re, B, nx, ny, k, dy, re_scale, x0):
    import torch
    scratch = torch.empty(B * (nx + 1), dtype=torch.float32, device=x0.device)
    _check(_lib.rmrt_nn_features(_ptr(solid), _ptr(re), B, nx, ny, k, float(dy), float(re_scale), _ptr(x0),
                                 x0.shape[-1], _ptr(scratch), _stream()), "rmrt_nn_features")


def nn_targets(rho, u, solid, B, nx, ny, k, dy, Ut, rho_scale, tgt, wgt):
    _check(_lib.rmrt_nn_targets(_ptr(rho), _ptr(u), _ptr(solid), B, nx, ny, k, float(dy), float(Ut),
                                float(rho_scale), _ptr(tgt), _ptr(wgt), _stream()), "rmrt_nn_targets")


def nn_warm_fields(out, B, nx, ny, k, dy, Ut, rho_scale, solid, rho, u):
    _check(_lib.rmrt_nn_warm_fields(_ptr(out), out.shape[-1], B, nx, ny, k, float(dy), float(Ut), float(rho_scale),
                                    _ptr(solid), _ptr(rho), _ptr(u), _stream()), "rmrt_nn_warm_fields")
