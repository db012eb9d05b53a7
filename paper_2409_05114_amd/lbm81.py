"""Python binding of the RD3Q81 HIP library (include/lbm81.h).

Argument marshalling only: every step of the method runs in the HIP kernels
of liblbm81.so.  PyTorch provides device memory and streams.  There is no
fallback: if the library is missing or no GPU is present, the calls raise.

The functions below mirror the C ABI one to one (same names, same argument
order); ``Sim`` is a small convenience owner of the device buffers.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbm81.so")

LBM_OK = 0
STATUS = {0: "LBM_OK", -1: "LBM_E_ARG", -2: "LBM_E_HIP", -3: "LBM_E_STATE",
          -4: "LBM_E_UNREALIZABLE", -5: "LBM_E_NEWTON"}
STORAGE = {"f64": 0, "f32": 1, "f16": 2, "bf16": 3}
STORAGE_BYTES = {"f64": 8, "f32": 4, "f16": 2, "bf16": 2}
FLAG_UNREALIZABLE = 0x1
FLAG_NEWTON = 0x2
FLAG_NONFINITE = 0x4
FLAG_NEGATIVE = 0x8
COLLISIONS = {"bgk": 0, "entropic": 1, "series": 2}
BATCH_MAX = 64
Q = 81

_lib = None


class LbmError(RuntimeError):
    def __init__(self, status, where):
        msg = _load().lbm_last_error().decode(errors="replace")
        super().__init__(f"{where}: {STATUS.get(status, status)}: {msg}")
        self.status = status


def _load():
    global _lib
    if _lib is None:
        # torch first: its bundled HIP runtime then satisfies the library's
        # libamdhip64.so.7 dependency, so both share one runtime (and one
        # view of devices, memory and streams)
        import torch  # noqa: F401

        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with "
                "`python -m paper_2409_05114_amd.build` (hipcc, gfx950)")
        lib = ctypes.CDLL(LIB_PATH)
        vp, i, d = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
        sz = ctypes.c_size_t
        lib.lbm_population_bytes.argtypes = [i, i, i, i]
        lib.lbm_population_bytes.restype = sz
        lib.lbm_workspace_bytes.argtypes = [i, i, i]
        lib.lbm_workspace_bytes.restype = sz
        lib.lbm_create.argtypes = [i, i, i, i, vp, vp, vp,
                                   ctypes.POINTER(vp)]
        lib.lbm_create_static.argtypes = [i, i, i, i, vp, vp,
                                          ctypes.POINTER(vp)]
        lib.lbm_destroy.argtypes = [vp]
        lib.lbm_init.argtypes = [vp, vp, vp, vp]
        lib.lbm_step.argtypes = [vp, i, d]
        lib.lbm_moments.argtypes = [vp, vp, vp, vp]
        lib.lbm_populations.argtypes = [vp, vp]
        lib.lbm_velocities.argtypes = [vp, vp]
        lib.lbm_totals.argtypes = [vp, vp, vp]
        lib.lbm_diagnostics.argtypes = [vp, vp, vp]
        lib.lbm_flags.argtypes = [vp, vp, i]
        lib.lbm_flags_async.argtypes = [vp, vp]
        lib.lbm_flags_batch.argtypes = [vp, i, vp, vp]
        lib.lbm_step_batch.argtypes = [vp, vp, vp, i, vp]
        lib.lbm_step_count.argtypes = [vp]
        lib.lbm_step_count.restype = ctypes.c_longlong
        lib.lbm_set_step_count.argtypes = [vp, ctypes.c_longlong]
        lib.lbm_set_collision.argtypes = [vp, i]
        lib.lbm_warm_bytes.argtypes = [i, i, i]
        lib.lbm_warm_bytes.restype = sz
        lib.lbm_set_warm_start.argtypes = [vp, vp]
        lib.lbm_probe_placement.argtypes = [vp, i, ctypes.POINTER(ctypes.c_float)]
        lib.lbm_status_string.argtypes = [i]
        lib.lbm_status_string.restype = ctypes.c_char_p
        lib.lbm_last_error.restype = ctypes.c_char_p
        lib.lbm_version.restype = i
        for name in ("lbm_create", "lbm_create_static", "lbm_destroy", "lbm_init", "lbm_step",
                     "lbm_moments", "lbm_populations", "lbm_totals",
                     "lbm_flags", "lbm_flags_async", "lbm_flags_batch",
                     "lbm_step_batch",
                     "lbm_set_step_count", "lbm_diagnostics",
                     "lbm_set_collision", "lbm_set_warm_start",
                     "lbm_probe_placement"):
            getattr(lib, name).restype = i
        _lib = lib
    return _lib


def library():
    """The loaded ctypes library (loads it on first use)."""
    return _load()


def _check(status, where):
    if status != LBM_OK:
        raise LbmError(status, where)


def _dptr(t):
    """Device pointer of a contiguous CUDA/HIP tensor."""
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return ctypes.c_void_p(t.data_ptr())


# ------------------------------------------------------------ C ABI mirror

# Placement probing (Sim(placement=k)): timed passes per candidate buffer,
# and the device memory left free beside the candidates.
PLACEMENT_REPS = 3
PLACEMENT_RESERVE = 4 << 30


def lbm_population_bytes(nx, ny, nz, storage):
    return int(_load().lbm_population_bytes(nx, ny, nz, STORAGE[storage]))


def lbm_workspace_bytes(nx, ny, nz):
    return int(_load().lbm_workspace_bytes(nx, ny, nz))


def lbm_warm_bytes(nx, ny, nz):
    return int(_load().lbm_warm_bytes(nx, ny, nz))


def lbm_velocities():
    """(c[81, 3] as float64, w[81]) in the library's direction order."""
    c2 = (ctypes.c_int * (3 * Q))()
    w = (ctypes.c_double * Q)()
    n = _load().lbm_velocities(c2, w)
    assert n == Q
    return (np.array(c2[:], dtype=np.float64).reshape(Q, 3) / 2.0,
            np.array(w[:]))


def lbm_version():
    return int(_load().lbm_version())


class Sim:
    """One simulation: caller-owned device buffers + a library handle.

    shape = (nx, ny, nz) cubic cells; 2 nx ny nz sites (cube corners and
    centres).  storage in {"f64", "f32", "f16", "bf16"}.  All work is
    enqueued on ``stream`` (default: torch's current stream at creation).
    static_workspace: create with lbm_create_static (the library's static
    per-device workspace instead of a workspace tensor; one such simulation
    at a time per device).
    placement: number of candidate population buffers (1: a plain
    allocation).  With k > 1, up to k buffers are allocated while at least
    PLACEMENT_RESERVE bytes of device memory stay free, each is timed with
    lbm_probe_placement, the fastest is kept and the others are released
    (torch.cuda.empty_cache()).  The probe times are kept in
    ``placement_ms`` and the index of the kept buffer in
    ``placement_choice``.
    """

    def __init__(self, shape, storage="f64", stream=None, device=None,
                 static_workspace=False, placement=1):
        import torch

        if not torch.cuda.is_available():
            raise RuntimeError("no GPU: the RD3Q81 library runs on HIP only")
        self.torch = torch
        self.shape = tuple(int(v) for v in shape)
        self.storage = storage
        nx, ny, nz = self.shape
        self.n_sites = 2 * nx * ny * nz
        self.device = torch.device(device or f"cuda:{torch.cuda.current_device()}")
        pb = lbm_population_bytes(nx, ny, nz, storage)
        if pb == 0:
            raise ValueError(f"invalid grid {self.shape} or storage {storage}")
        wb = lbm_workspace_bytes(nx, ny, nz)
        self.stream = stream or torch.cuda.current_stream(self.device)
        self.placement_ms = None
        self.placement_choice = 0
        # torch allocations are 256-byte aligned
        if int(placement) > 1:
            self.populations = self._placed(pb, wb, int(placement))
        else:
            self.populations = torch.empty(pb, dtype=torch.uint8,
                                           device=self.device)
        h = ctypes.c_void_p()
        if static_workspace:
            self.workspace = None
            with torch.cuda.device(self.device):
                _check(_load().lbm_create_static(
                    nx, ny, nz, STORAGE[storage], _dptr(self.populations),
                    ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)),
                    "lbm_create_static")
        else:
            self.workspace = torch.empty(wb, dtype=torch.uint8,
                                         device=self.device)
            _check(_load().lbm_create(nx, ny, nz, STORAGE[storage],
                                      _dptr(self.populations),
                                      _dptr(self.workspace),
                                      ctypes.c_void_p(self.stream.cuda_stream),
                                      ctypes.byref(h)), "lbm_create")
        self.handle = h

    def _placed(self, pb, wb, k):
        """The fastest of up to k candidate population buffers."""
        t = self.torch
        nx, ny, nz = self.shape
        lib = _load()
        ws = t.empty(wb, dtype=t.uint8, device=self.device)
        cands = []
        ms = ctypes.c_float()
        with t.cuda.device(self.device):
            for j in range(k):
                if j and t.cuda.mem_get_info(self.device)[0] < pb + PLACEMENT_RESERVE:
                    break
                try:
                    buf = t.empty(pb, dtype=t.uint8, device=self.device)
                except t.cuda.OutOfMemoryError:
                    if not j:
                        raise
                    break  # the candidates found so far will do
                h = ctypes.c_void_p()
                _check(lib.lbm_create(nx, ny, nz, STORAGE[self.storage],
                                      _dptr(buf), _dptr(ws),
                                      ctypes.c_void_p(self.stream.cuda_stream),
                                      ctypes.byref(h)), "lbm_create")
                try:
                    # waits for its passes: the candidate is idle afterwards
                    _check(lib.lbm_probe_placement(h, PLACEMENT_REPS,
                                                   ctypes.byref(ms)),
                           "lbm_probe_placement")
                finally:
                    lib.lbm_destroy(h)
                cands.append((ms.value, j, buf))
        best = min(cands, key=lambda c: (c[0], c[1]))
        self.placement_ms = [c[0] for c in cands]
        self.placement_choice = best[1]
        buf = best[2]
        del cands, best
        t.cuda.empty_cache()
        return buf

    # -- lifetime
    def close(self):
        if getattr(self, "handle", None):
            _load().lbm_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- fields
    def _field(self, a, n):
        t = self.torch
        if isinstance(a, np.ndarray):
            a = t.from_numpy(np.ascontiguousarray(a, dtype=np.float64))
        a = a.to(device=self.device, dtype=t.float64).contiguous()
        if a.numel() != n:
            raise ValueError(f"field has {a.numel()} values, expected {n}")
        return a

    def init(self, rho, u, theta):
        """Populations := f_eq(rho, u, theta); FP64 fields, site order
        [sub][z][y][x], u shaped [3, sites]."""
        n = self.n_sites
        r = self._field(rho, n)
        uu = self._field(u, 3 * n)
        th = self._field(theta, n)
        # the fields were written on torch's current stream
        cur = self.torch.cuda.current_stream(self.device)
        self.stream.wait_stream(cur)
        _check(_load().lbm_init(self.handle, _dptr(r), _dptr(uu), _dptr(th)),
               "lbm_init")
        if self.stream != cur:
            # the caching allocator must not hand the inputs out again before
            # the library's stream has consumed them
            for a in (r, uu, th):
                a.record_stream(self.stream)

    def step(self, nsteps, tau):
        _check(_load().lbm_step(self.handle, int(nsteps), float(tau)),
               "lbm_step")

    def moments(self):
        """(rho[sites], u[3, sites], theta[sites]) as FP64 device tensors."""
        t = self.torch
        n = self.n_sites
        rho = t.empty(n, dtype=t.float64, device=self.device)
        u = t.empty((3, n), dtype=t.float64, device=self.device)
        th = t.empty(n, dtype=t.float64, device=self.device)
        self.stream.wait_stream(t.cuda.current_stream(self.device))
        _check(_load().lbm_moments(self.handle, _dptr(rho), _dptr(u),
                                   _dptr(th)), "lbm_moments")
        t.cuda.current_stream(self.device).wait_stream(self.stream)
        return rho, u, th

    def populations_f64(self):
        """Current f_i as an FP64 device tensor [81, sites] (library
        direction order, see lbm_velocities)."""
        t = self.torch
        f = t.empty((Q, self.n_sites), dtype=t.float64, device=self.device)
        self.stream.wait_stream(t.cuda.current_stream(self.device))
        _check(_load().lbm_populations(self.handle, _dptr(f)),
               "lbm_populations")
        t.cuda.current_stream(self.device).wait_stream(self.stream)
        return f

    def totals(self, check=True):
        """Domain totals [mass, momentum x3, energy moment] and the flag word
        (synchronises).  Raises on a device error flag when check=True."""
        out = (ctypes.c_double * 5)()
        flags = ctypes.c_uint(0)
        st = _load().lbm_totals(self.handle, out, ctypes.byref(flags))
        if check:
            _check(st, "lbm_totals")
        return np.array(out[:]), int(flags.value)

    def diagnostics(self, fields=None):
        """(mean kinetic energy, mean enstrophy) of the current state (the
        Taylor-Green diagnostics; synchronises).  `fields`: optional FP64
        device tensor of at least 4 * sites elements used as the moment
        buffer (allocated per call if None)."""
        t = self.torch
        if fields is None:
            fields = t.empty(4 * self.n_sites, dtype=t.float64, device=self.device)
        if (fields.dtype != t.float64 or not fields.is_contiguous()
                or fields.numel() < 4 * self.n_sites):
            raise ValueError("fields must be a contiguous float64 tensor of "
                             ">= 4 * sites elements")
        self.stream.wait_stream(t.cuda.current_stream(self.device))
        out = (ctypes.c_double * 2)()
        _check(_load().lbm_diagnostics(self.handle, _dptr(fields), out),
               "lbm_diagnostics")
        if self.stream != t.cuda.current_stream(self.device):
            fields.record_stream(self.stream)
        return float(out[0]), float(out[1])

    def flags_async(self, host_u32):
        """Enqueue a copy of the flag word into a pinned torch.int32 host
        tensor of one element (then clear the word); no synchronisation."""
        if host_u32.numel() < 1 or host_u32.is_cuda:
            raise ValueError("expected a host tensor with one element")
        _check(_load().lbm_flags_async(
            self.handle, ctypes.c_void_p(host_u32.data_ptr())), "lbm_flags_async")

    def flags(self, clear=True):
        f = ctypes.c_uint(0)
        _check(_load().lbm_flags(self.handle, ctypes.byref(f), int(clear)),
               "lbm_flags")
        return int(f.value)

    @property
    def step_count(self):
        return int(_load().lbm_step_count(self.handle))

    def set_step_count(self, n):
        _check(_load().lbm_set_step_count(self.handle, int(n)),
               "lbm_set_step_count")

    def set_collision(self, collision):
        """'bgk' (alpha = 2), 'entropic' (alpha from the entropy
        condition, Eq. delH) or 'series' (alpha = 2 towards the series
        equilibrium of Appendix B where it is positive, f_eq elsewhere) for
        the following steps."""
        _check(_load().lbm_set_collision(self.handle, COLLISIONS[collision]),
               "lbm_set_collision")

    def set_warm_start(self, enable=True):
        """Keep the entropic search's alpha per site between steps and start
        the next search there (lbm_set_warm_start; a device buffer of one
        float per site, cleared now).  enable=False detaches it."""
        if enable:
            if getattr(self, "warm", None) is None:
                nx, ny, nz = self.shape
                self.warm = self.torch.empty(lbm_warm_bytes(nx, ny, nz),
                                             dtype=self.torch.uint8,
                                             device=self.device)
            _check(_load().lbm_set_warm_start(self.handle, _dptr(self.warm)),
                   "lbm_set_warm_start")
        else:
            _check(_load().lbm_set_warm_start(self.handle, None),
                   "lbm_set_warm_start")
            if getattr(self, "warm", None) is not None:
                # the library's stream may still use the buffer
                self.warm.record_stream(self.stream)
                self.warm = None

    # -- checkpoint / resume
    def checkpoint(self):
        """Host copy of the state: raw population bytes, step count,
        grid and storage.  Synchronises."""
        self.torch.cuda.synchronize(self.device)
        return {"shape": self.shape, "storage": self.storage,
                "step": self.step_count,
                "populations": self.populations.cpu().numpy().copy()}

    def restore(self, ck):
        if tuple(ck["shape"]) != self.shape or ck["storage"] != self.storage:
            raise ValueError("checkpoint is for another grid or storage")
        src = self.torch.from_numpy(ck["populations"])
        # work still queued on the library's stream must not race the copy
        self.torch.cuda.synchronize(self.device)
        self.populations.copy_(src.to(self.device))
        self.set_step_count(ck["step"])
        self.torch.cuda.synchronize(self.device)


def lbm_step_batch(sims, nsteps, taus, stream=None):
    """Advance sims[k] by nsteps[k] steps with relaxation time taus[k], in
    batched launches on `stream` (default: torch's current stream); an int
    nsteps applies to every simulation.  Simulations created on another
    stream are ordered against it by the library (events)."""
    import torch

    n = len(sims)
    if n == 0:
        return
    if n > BATCH_MAX:
        raise ValueError(f"at most {BATCH_MAX} simulations per batch")
    if isinstance(nsteps, (int, np.integer)):
        nsteps = [int(nsteps)] * n
    if len(nsteps) != n or len(taus) != n:
        raise ValueError("need one step count and one tau per simulation")
    handles = (ctypes.c_void_p * n)(*[s.handle for s in sims])
    ns = (ctypes.c_int * n)(*[int(x) for x in nsteps])
    t = (ctypes.c_double * n)(*[float(x) for x in taus])
    st = stream or torch.cuda.current_stream()
    _check(_load().lbm_step_batch(handles, ns, t, n,
                                  ctypes.c_void_p(st.cuda_stream)),
           "lbm_step_batch")


def lbm_flags_batch(sims, host_u32, stream=None):
    """Enqueue one gather of the flag words of `sims` (at most BATCH_MAX)
    into the pinned torch.int32 host tensor `host_u32` (its first len(sims)
    elements), clearing them; no synchronisation."""
    import torch

    n = len(sims)
    if n == 0:
        return
    if n > BATCH_MAX:
        raise ValueError(f"at most {BATCH_MAX} simulations per call")
    if host_u32.is_cuda or host_u32.numel() < n or host_u32.dtype != torch.int32:
        raise ValueError("expected a host int32 tensor with one slot per simulation")
    handles = (ctypes.c_void_p * n)(*[s.handle for s in sims])
    st = stream or torch.cuda.current_stream()
    _check(_load().lbm_flags_batch(handles, n, ctypes.c_void_p(host_u32.data_ptr()),
                                   ctypes.c_void_p(st.cuda_stream)),
           "lbm_flags_batch")
