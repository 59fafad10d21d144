"""ctypes binding of libpinmpc (argument marshalling only).

Every step of the solve runs in the HIP library; this module only fills the
C structs with device pointers of torch tensors and passes the caller's HIP
stream.  It fails loudly when the library is missing: there is no host
fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpinmpc.so")

NX, NU, NRES = 13, 12, 5
ST_OK, ST_MAXITER, ST_UNPOLISHED, ST_NONFINITE, ST_BADINPUT = range(5)
E_TOOBIG = -6                  # PINMPC_ETOOBIG
NOALLOC_SCRATCH_BYTES = 256 << 20   # PINMPC_NOALLOC_SCRATCH_BYTES


class Settings(ctypes.Structure):
    _fields_ = [
        ("rho", ctypes.c_float),
        ("iters", ctypes.c_int32),
        ("accel", ctypes.c_int32),
        ("restart_eta", ctypes.c_float),
        ("scaling", ctypes.c_int32),
        ("refine", ctypes.c_int32),
        ("refine_passes", ctypes.c_int32),
        ("ipm_iters", ctypes.c_int32),
        ("polish_passes", ctypes.c_int32),
        ("kkt_tol", ctypes.c_double),
        ("precision", ctypes.c_int32),
        ("form", ctypes.c_int32),
        ("graph", ctypes.c_int32),
        ("first_passes", ctypes.c_int32),
        ("group", ctypes.c_int32),
        ("scan", ctypes.c_int32),
    ]


class Batch(ctypes.Structure):
    _fields_ = [
        ("batch", ctypes.c_int32),
        ("n_max", ctypes.c_int32),
        ("N", ctypes.c_void_p),
        ("A", ctypes.c_void_p),
        ("Bu", ctypes.c_void_p),
        ("e", ctypes.c_void_p),
        ("x0", ctypes.c_void_p),
        ("u_prev", ctypes.c_void_p),
        ("x_ref", ctypes.c_void_p),
        ("u_ref", ctypes.c_void_p),
        ("Q", ctypes.c_void_p),
        ("R", ctypes.c_void_p),
        ("contact", ctypes.c_void_p),
        ("mu", ctypes.c_void_p),
        ("fz_max", ctypes.c_void_p),
        ("tau_max", ctypes.c_void_p),
        ("weight", ctypes.c_void_p),
        ("contacts", ctypes.c_int32),
    ]


class Out(ctypes.Structure):
    _fields_ = [
        ("u", ctypes.c_void_p),
        ("x", ctypes.c_void_p),
        ("res", ctypes.c_void_p),
        ("iters", ctypes.c_void_p),
        ("status", ctypes.c_void_p),
        ("detail", ctypes.c_void_p),
    ]


class Physics(ctypes.Structure):
    _fields_ = [
        ("batch", ctypes.c_int32),
        ("n_max", ctypes.c_int32),
        ("model", ctypes.c_int32),
        ("N", ctypes.c_void_p),
        ("yaw", ctypes.c_void_p),
        ("c_ref", ctypes.c_void_p),
        ("feet", ctypes.c_void_p),
        ("mass", ctypes.c_void_p),
        ("inertia", ctypes.c_void_p),
        ("dt", ctypes.c_void_p),
    ]


class Landmarks(ctypes.Structure):
    _fields_ = [
        ("envs", ctypes.c_int32),
        ("n_landmarks", ctypes.c_int32),
        ("ring", ctypes.c_int32),
        ("ticks_per_step", ctypes.c_int32),
        ("com", ctypes.c_void_p),
        ("tag", ctypes.c_void_p),
    ]


EXPORTS = {
    "pinmpc_default_settings": (None, [ctypes.POINTER(Settings)]),
    "pinmpc_create": (ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int,
                                     ctypes.c_size_t, ctypes.POINTER(Settings)]),
    "pinmpc_set_settings": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Settings)]),
    "pinmpc_workspace_bytes": (ctypes.c_int, [ctypes.POINTER(Settings), ctypes.c_int32,
                                              ctypes.c_int32, ctypes.POINTER(ctypes.c_size_t)]),
    "pinmpc_workspace_bytes_contacts": (ctypes.c_int, [ctypes.POINTER(Settings), ctypes.c_int32,
                                                       ctypes.c_int32, ctypes.c_int32,
                                                       ctypes.POINTER(ctypes.c_size_t)]),
    "pinmpc_solve": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Batch), ctypes.POINTER(Out),
                                    ctypes.c_void_p]),
    "pinmpc_solve_noalloc": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Batch),
                                            ctypes.POINTER(Out), ctypes.c_void_p]),
    "pinmpc_admm": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Batch), ctypes.c_int32,
                                   ctypes.c_void_p, ctypes.c_void_p]),
    "pinmpc_stats": (ctypes.c_int, [ctypes.c_void_p] + [ctypes.POINTER(ctypes.c_double)] * 4),
    "pinmpc_stats_back": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32] +
                          [ctypes.POINTER(ctypes.c_double)] * 4),
    "pinmpc_stats_traffic": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double),
                                            ctypes.POINTER(ctypes.c_double)]),
    "pinmpc_build_dynamics": (ctypes.c_int, [ctypes.POINTER(Physics), ctypes.c_void_p,
                                             ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "pinmpc_server_export_state": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                                  ctypes.c_void_p, ctypes.c_size_t]),
    "pinmpc_server_import_state": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                                  ctypes.c_void_p, ctypes.c_size_t]),
    "pinmpc_landmarks_clear": (ctypes.c_int, [ctypes.POINTER(Landmarks), ctypes.c_void_p,
                                              ctypes.c_void_p]),
    "pinmpc_landmarks_push": (ctypes.c_int, [ctypes.POINTER(Landmarks), ctypes.c_int32,
                                             ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                             ctypes.c_void_p]),
    "pinmpc_landmark_reward": (ctypes.c_int, [ctypes.POINTER(Landmarks), ctypes.c_void_p,
                                              ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                              ctypes.c_float, ctypes.c_void_p, ctypes.c_void_p,
                                              ctypes.c_void_p]),
    "pinmpc_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "pinmpc_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "pinmpc_server_create": (ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int,
                                            ctypes.POINTER(Settings), ctypes.c_int, ctypes.c_int32,
                                            ctypes.c_int32, ctypes.c_size_t]),
    "pinmpc_submit": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Batch), ctypes.POINTER(Out),
                                     ctypes.c_int32, ctypes.POINTER(ctypes.c_int64)]),
    "pinmpc_poll": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.POINTER(ctypes.c_int),
                                   ctypes.POINTER(ctypes.c_double)]),
    "pinmpc_wait": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.POINTER(ctypes.c_double)]),
    "pinmpc_server_stats": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64),
                                           ctypes.POINTER(ctypes.c_int64)]),
    "pinmpc_server_destroy": (ctypes.c_int, [ctypes.c_void_p]),
}

_lib = None


STATS_RING = 64   # PINMPC_STATS_RING
NMAX = 64         # PINMPC_NMAX
NMAX_LONG = 512   # PINMPC_NMAX_LONG
WARM_SLOT_BYTES = NMAX * 5 * 25 * 4   # PINMPC_WARM_SLOT_BYTES
E_BUSY = -5       # PINMPC_EBUSY


def warm_image_bytes(count: int) -> int:
    """PINMPC_WARM_IMAGE_BYTES(count)."""
    return 16 + count * WARM_SLOT_BYTES


def load(path: str = LIB_PATH):
    """Load libpinmpc.so (raises if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libpinmpc.so not built at {path}; run __graft_entry__.build()")
    # torch ships its own HIP runtime; load it first so that the library binds
    # to the same runtime instance torch's tensors and streams live in
    import torch  # noqa: F401
    lib = ctypes.CDLL(path)
    for name, (res, args) in EXPORTS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class PinmpcError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(msg)
        self.code = code


def _check(rc):
    if rc != 0:
        raise PinmpcError(rc, f"pinmpc error {rc}: {load().pinmpc_strerror(rc).decode()}")


def default_settings(**over) -> Settings:
    s = Settings()
    load().pinmpc_default_settings(ctypes.byref(s))
    for k, v in over.items():
        if not hasattr(s, k):
            raise KeyError(k)
        setattr(s, k, v)
    return s


FIELDS = ("N", "A", "B", "e", "x0", "u_prev", "x_ref", "u_ref", "Q", "R", "contact",
          "mu", "fz_max", "tau_max", "weight")


def to_device(batch: dict, device="cuda"):
    """Copy a generator batch (numpy) to device tensors (torch)."""
    import torch
    out = {}
    for k in FIELDS:
        if k in batch and batch[k] is not None:
            out[k] = torch.from_numpy(np.ascontiguousarray(batch[k])).to(device)
    return out


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def n_inputs(dev: dict) -> int:
    """Inputs per stage of a batch (12: two contacts; 24: feet and hands)."""
    return int(dev["B"].shape[-1])


def make_batch_struct(dev: dict) -> Batch:
    import torch
    A = dev["A"]
    assert A.dtype == torch.float32 and A.is_contiguous()
    b = Batch()
    b.batch, b.n_max = int(A.shape[0]), int(A.shape[1])
    b.contacts = n_inputs(dev) // 6
    for k in FIELDS:
        t = dev.get(k)
        if t is not None:
            assert t.is_contiguous() and t.shape[0] == b.batch, k
        setattr(b, "Bu" if k == "B" else k, None if t is None else t.data_ptr())
    return b


class Solver:
    """One library context on one GPU."""

    def __init__(self, device: int = 0, hbm_budget: int = 0, **settings):
        lib = load()
        self.settings = default_settings(**settings)
        h = ctypes.c_void_p()
        _check(lib.pinmpc_create(ctypes.byref(h), int(device), int(hbm_budget),
                                 ctypes.byref(self.settings)))
        self._h = h
        self.device = device

    def close(self):
        if getattr(self, "_h", None):
            load().pinmpc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set(self, **over):
        for k, v in over.items():
            setattr(self.settings, k, v)
        _check(load().pinmpc_set_settings(self._h, ctypes.byref(self.settings)))

    def alloc_out(self, dev):
        import torch
        Bn, n = int(dev["A"].shape[0]), int(dev["A"].shape[1])
        d = dev["A"].device
        return {
            "u": torch.empty((Bn, n, n_inputs(dev)), dtype=torch.float32, device=d),
            "x": torch.empty((Bn, n + 1, NX), dtype=torch.float32, device=d),
            "res": torch.empty((Bn, NRES), dtype=torch.float32, device=d),
            "iters": torch.empty((Bn,), dtype=torch.int32, device=d),
            "status": torch.empty((Bn,), dtype=torch.int32, device=d),
            "detail": torch.empty((Bn, 4), dtype=torch.int32, device=d),
        }

    def solve(self, dev: dict, out: dict | None = None, stream=None, batch_struct=None):
        """Solve the batch held in device tensors; returns the output tensors."""
        import torch
        if out is None:
            out = self.alloc_out(dev)
        b = batch_struct if batch_struct is not None else make_batch_struct(dev)
        o = _out_struct(out)
        st = stream if stream is not None else torch.cuda.current_stream()
        _check(load().pinmpc_solve(self._h, ctypes.byref(b), ctypes.byref(o),
                                   ctypes.c_void_p(st.cuda_stream)))
        return out

    def solve_noalloc(self, dev: dict, out: dict, stream=None):
        """pinmpc_solve_noalloc: the same solve with the library's static
        device scratch as workspace (no device allocation by the library);
        `out` must be preallocated."""
        import torch
        b = make_batch_struct(dev)
        o = _out_struct(out)
        st = stream if stream is not None else torch.cuda.current_stream()
        _check(load().pinmpc_solve_noalloc(self._h, ctypes.byref(b), ctypes.byref(o),
                                           ctypes.c_void_p(st.cuda_stream)))
        return out

    def admm(self, dev: dict, iters: int, stream=None):
        """ADMM only: final z iterates [B][n][13 + inputs] (unscaled)."""
        import torch
        Bn, n = int(dev["A"].shape[0]), int(dev["A"].shape[1])
        z = torch.empty((Bn, n, NX + n_inputs(dev)), dtype=torch.float32, device=dev["A"].device)
        b = make_batch_struct(dev)
        st = stream if stream is not None else torch.cuda.current_stream()
        _check(load().pinmpc_admm(self._h, ctypes.byref(b), int(iters),
                                  ctypes.c_void_p(z.data_ptr()), ctypes.c_void_p(st.cuda_stream)))
        return z

    def traffic(self):
        """Algorithmic HBM bytes of the last solve and their rate (GB/s)."""
        b, g = ctypes.c_double(), ctypes.c_double()
        _check(load().pinmpc_stats_traffic(self._h, ctypes.byref(b), ctypes.byref(g)))
        return {"bytes": b.value, "gbs": g.value}

    def stats(self, back: int = 0):
        """Phase times (ms) of the last solve, or of the solve `back` solves
        before it (up to STATS_RING - 1)."""
        vals = [ctypes.c_double() for _ in range(4)]
        _check(load().pinmpc_stats_back(self._h, int(back), *[ctypes.byref(v) for v in vals]))
        return dict(zip(("total_ms", "setup_ms", "admm_ms", "refine_ms"), [v.value for v in vals]))


def _out_struct(out):
    def opt(k):
        return None if out.get(k) is None else out[k].data_ptr()
    return Out(out["u"].data_ptr(), out["x"].data_ptr(), opt("res"), opt("iters"),
               opt("status"), opt("detail"))


class Server:
    """Continuous-batching server (pinmpc_server_*) on one GPU."""

    def __init__(self, device=0, lanes=3, capacity=4096, warm_slots=0, hbm_budget=0,
                 **settings):
        lib = load()
        self.settings = default_settings(**settings)
        h = ctypes.c_void_p()
        _check(lib.pinmpc_server_create(ctypes.byref(h), int(device), ctypes.byref(self.settings),
                                        int(lanes), int(capacity), int(warm_slots),
                                        int(hbm_budget)))
        self._h = h
        self._keep = {}

    def submit(self, dev, out, warm_base=-1):
        """Queue a request (device tensors stay referenced until it is done)."""
        b = make_batch_struct(dev)
        o = _out_struct(out)
        t = ctypes.c_int64()
        _check(load().pinmpc_submit(self._h, ctypes.byref(b), ctypes.byref(o), int(warm_base),
                                    ctypes.byref(t)))
        self._keep[t.value] = (dev, out)
        return t.value

    def poll(self, ticket):
        done = ctypes.c_int()
        lat = ctypes.c_double()
        _check(load().pinmpc_poll(self._h, int(ticket), ctypes.byref(done), ctypes.byref(lat)))
        if done.value:
            self._keep.pop(ticket, None)
            return lat.value
        return None

    def wait(self, ticket):
        lat = ctypes.c_double()
        _check(load().pinmpc_wait(self._h, int(ticket), ctypes.byref(lat)))
        self._keep.pop(ticket, None)
        return lat.value

    def export_state(self, slot_base: int, count: int) -> bytes:
        """Host image of warm slots [slot_base, slot_base + count)."""
        buf = ctypes.create_string_buffer(warm_image_bytes(count))
        _check(load().pinmpc_server_export_state(self._h, int(slot_base), int(count), buf,
                                                 len(buf)))
        return buf.raw

    def import_state(self, slot_base: int, count: int, image: bytes):
        """Write a host image back into warm slots [slot_base, slot_base + count)."""
        buf = ctypes.create_string_buffer(bytes(image), len(image))
        _check(load().pinmpc_server_import_state(self._h, int(slot_base), int(count), buf,
                                                 len(image)))

    def stats(self):
        a, b = ctypes.c_int64(), ctypes.c_int64()
        _check(load().pinmpc_server_stats(self._h, ctypes.byref(a), ctypes.byref(b)))
        return {"launches": a.value, "problems": b.value}

    def close(self):
        if getattr(self, "_h", None):
            _check(load().pinmpc_server_destroy(self._h))
            self._h = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


PHYSICS_FIELDS = ("N", "yaw_k", "c_ref", "feet", "mass", "inertia", "dt")
MODELS = {"srb": 0, "momentum": 1}


def build_dynamics(phys: dict, A=None, B=None, e=None, model="srb", stream=None):
    """pinmpc_build_dynamics: stage matrices [B][n][13][13], [B][n][13][12]
    and affine terms [B][n][13] from compact physics held in device tensors
    (keys of PHYSICS_FIELDS); model "srb" (13-state single rigid body) or
    "momentum" (the 9-state momentum model, e required)."""
    import torch
    ref = phys["c_ref"]
    assert ref.dtype == torch.float32 and ref.is_contiguous()
    Bn, n = int(ref.shape[0]), int(ref.shape[1])
    if A is None:
        A = torch.empty((Bn, n, NX, NX), dtype=torch.float32, device=ref.device)
    if B is None:
        B = torch.empty((Bn, n, NX, NU), dtype=torch.float32, device=ref.device)
    if e is None and model == "momentum":
        e = torch.empty((Bn, n, NX), dtype=torch.float32, device=ref.device)
    ph = Physics()
    ph.batch, ph.n_max, ph.model = Bn, n, MODELS[model]
    for f, k in (("N", "N"), ("yaw", "yaw_k"), ("c_ref", "c_ref"), ("feet", "feet"),
                 ("mass", "mass"), ("inertia", "inertia"), ("dt", "dt")):
        t = phys.get(k)
        if t is not None:
            assert t.is_contiguous() and t.shape[0] == Bn, k
        setattr(ph, f, None if t is None else t.data_ptr())
    st = stream if stream is not None else torch.cuda.current_stream()
    _check(load().pinmpc_build_dynamics(ctypes.byref(ph), ctypes.c_void_p(A.data_ptr()),
                                        ctypes.c_void_p(B.data_ptr()), _ptr(e),
                                        ctypes.c_void_p(st.cuda_stream)))
    return A, B, e


class LandmarkRing:
    """Device landmark store of Sec. II-C's guidance reward (pinmpc_landmarks_*)."""

    def __init__(self, envs, n_landmarks, ring, ticks_per_step=1, device="cuda"):
        import torch
        self.com = torch.zeros((envs, ring, n_landmarks, 3), dtype=torch.float32, device=device)
        self.tag = torch.full((envs, ring, n_landmarks), -1, dtype=torch.int32, device=device)
        self.st = Landmarks(int(envs), int(n_landmarks), int(ring), int(ticks_per_step),
                            self.com.data_ptr(), self.tag.data_ptr())

    @staticmethod
    def _stream(stream):
        import torch
        st = stream if stream is not None else torch.cuda.current_stream()
        return ctypes.c_void_p(st.cuda_stream)

    def clear(self, env_mask=None, stream=None):
        _check(load().pinmpc_landmarks_clear(ctypes.byref(self.st), _ptr(env_mask),
                                             self._stream(stream)))

    def push(self, x, N, tick, stream=None):
        n_max = int(x.shape[1]) - 1
        _check(load().pinmpc_landmarks_push(ctypes.byref(self.st), n_max, _ptr(N), _ptr(x),
                                            int(tick), self._stream(stream)))

    def reward(self, com, tick, alpha, qc, sigma, stream=None):
        import torch
        envs = self.st.envs
        r = torch.empty(envs, dtype=torch.float32, device=com.device)
        used = torch.empty(envs, dtype=torch.int32, device=com.device)
        _check(load().pinmpc_landmark_reward(ctypes.byref(self.st), _ptr(com), int(tick),
                                             _ptr(alpha), _ptr(qc), float(sigma), _ptr(r),
                                             _ptr(used), self._stream(stream)))
        return r, used
