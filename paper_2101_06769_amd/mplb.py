"""ctypes binding of libmplb.so (include/mplb.h): argument marshalling only.

Every step of the method runs in the library's HIP kernels; PyTorch (ROCm)
supplies the device arena and the stream.  Importing this module does not
touch the GPU; the first Solver loads the library and raises if it is
missing.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("MPLB_LIBRARY", os.path.join(HERE, "libmplb.so"))

OK, EINVAL, ENOMEM, EDEVICE, EUNSTABLE, ESTATE = 0, -1, -2, -3, -4, -5
BC_PERIODIC, BC_WALL, BC_SYMMETRY = 0, 1, 2
STORE_FP64, STORE_FP32, STORE_FP16S, STORE_FP16S_ALL = 0, 1, 2, 3
COLL_CUMULANT, COLL_SRT = 0, 1
FIELD_PHI, FIELD_RHO, FIELD_UX, FIELD_UY, FIELD_UZ, FIELD_P = range(6)
STORAGE = {"fp64": STORE_FP64, "fp32": STORE_FP32, "fp16s": STORE_FP16S,
           "fp16s_all": STORE_FP16S_ALL}
DTYPE_NAME = {STORE_FP64: "f64", STORE_FP32: "f32", STORE_FP16S: "f16s+f32",
              STORE_FP16S_ALL: "f16s"}


class MplbError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("mplb error %d: %s" % (code, msg))
        self.code = code


class Params(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int32),
        ("n", ctypes.c_int32 * 3),
        ("bc", ctypes.c_int32 * 3),
        ("rho_heavy", ctypes.c_double),
        ("rho_light", ctypes.c_double),
        ("nu_heavy", ctypes.c_double),
        ("nu_light", ctypes.c_double),
        ("W", ctypes.c_double),
        ("mobility", ctypes.c_double),
        ("sigma", ctypes.c_double),
        ("gravity", ctypes.c_double * 3),
        ("storage", ctypes.c_int32),
        ("visc_interp", ctypes.c_int32),
        ("collision", ctypes.c_int32),
        ("cac_edf", ctypes.c_int32),
    ]


_lib = None


def load_library():
    """Load libmplb.so (built in-tree by ``build.build()``); raise if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libmplb.so is not built (run paper_2101_06769_amd.build.build())")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER(Params)
    vp = ctypes.c_void_p
    dp = ctypes.POINTER(ctypes.c_double)
    lib.mplb_version.restype = ctypes.c_int32
    lib.mplb_arch.restype = ctypes.c_char_p
    lib.mplb_last_error.restype = ctypes.c_char_p
    lib.mplb_state_bytes.argtypes = [P]
    lib.mplb_state_bytes.restype = ctypes.c_size_t
    lib.mplb_create.argtypes = [P, vp, ctypes.c_size_t, vp, ctypes.POINTER(vp)]
    lib.mplb_init.argtypes = [vp, dp, dp, dp]
    lib.mplb_step.argtypes = [vp, ctypes.c_int64]
    lib.mplb_step_timed.argtypes = [vp, ctypes.c_int64, dp, dp]
    lib.mplb_sync.argtypes = [vp]
    lib.mplb_steps_done.argtypes = [vp]
    lib.mplb_steps_done.restype = ctypes.c_int64
    lib.mplb_read.argtypes = [vp, ctypes.c_int32, dp]
    lib.mplb_reduce.argtypes = [vp, dp]
    lib.mplb_reduce_noalloc.argtypes = [vp, dp]
    lib.mplb_get_populations.argtypes = [vp, ctypes.c_int32, dp]
    lib.mplb_set_populations.argtypes = [vp, ctypes.c_int32, dp]
    lib.mplb_save_bytes.argtypes = [vp]
    lib.mplb_save_bytes.restype = ctypes.c_size_t
    lib.mplb_save.argtypes = [vp, vp, ctypes.c_size_t]
    lib.mplb_load.argtypes = [vp, vp, ctypes.c_size_t]
    lib.mplb_set_block.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]
    lib.mplb_set_phi_partials.argtypes = [vp, ctypes.c_int32]
    lib.mplb_uses_phi_partials.argtypes = [vp]
    lib.mplb_destroy.argtypes = [vp]
    lib.mplb_destroy.restype = None
    i32p = ctypes.POINTER(ctypes.c_int32)
    lib.mplb_tune_block.argtypes = [vp, ctypes.c_int32, i32p, ctypes.c_int32, i32p, dp]
    lib.mplb_batch_table_bytes.argtypes = [ctypes.c_int32, ctypes.c_int64]
    lib.mplb_batch_table_bytes.restype = ctypes.c_size_t
    lib.mplb_batch_create.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                      ctypes.c_int64, vp, ctypes.c_size_t, vp, ctypes.POINTER(vp)]
    lib.mplb_batch_set_block.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]
    lib.mplb_batch_set_graph_chunk.argtypes = [vp, ctypes.c_int32]
    lib.mplb_batch_tune_block.argtypes = [vp, ctypes.c_int32, i32p, ctypes.c_int32, i32p, dp]
    lib.mplb_batch_attach.argtypes = [vp, vp, ctypes.c_int64, i32p]
    lib.mplb_batch_detach.argtypes = [vp, ctypes.c_int32]
    lib.mplb_batch_step.argtypes = [vp, ctypes.c_int64]
    lib.mplb_batch_remaining.argtypes = [vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64)]
    lib.mplb_batch_status.argtypes = [vp, i32p]
    lib.mplb_batch_set_solo_cells.argtypes = [vp, ctypes.c_int64]
    lib.mplb_batch_is_solo.argtypes = [vp, ctypes.c_int32]
    lib.mplb_batch_steps_done.argtypes = [vp]
    lib.mplb_batch_steps_done.restype = ctypes.c_int64
    lib.mplb_batch_destroy.argtypes = [vp]
    lib.mplb_batch_destroy.restype = None
    _lib = lib
    return lib


def check(rc):
    if rc != OK:
        raise MplbError(rc, load_library().mplb_last_error().decode())
    return rc


def make_params(d: dict, storage="fp32", collision=COLL_CUMULANT) -> Params:
    """Params from a case dictionary (keys of ``inputs``: dim, n, bc, rho_h,
    rho_l, nu_h, nu_l, W, M, sigma, g, optional visc_interp)."""
    p = Params()
    p.dim = int(d["dim"])
    for i in range(3):
        p.n[i] = int(d["n"][i])
        p.bc[i] = int(d["bc"][i])
        p.gravity[i] = float(d["g"][i]) if (i < p.dim) else 0.0
    p.rho_heavy, p.rho_light = float(d["rho_h"]), float(d["rho_l"])
    p.nu_heavy, p.nu_light = float(d["nu_h"]), float(d["nu_l"])
    p.W, p.mobility, p.sigma = float(d["W"]), float(d["M"]), float(d["sigma"])
    p.storage = STORAGE[storage] if isinstance(storage, str) else int(storage)
    p.visc_interp = int(d.get("visc_interp", 0))
    p.collision = int(d.get("collision", collision))
    p.cac_edf = int(d.get("cac_edf", 0))
    return p


def state_bytes(params: Params) -> int:
    n = load_library().mplb_state_bytes(ctypes.byref(params))
    if n == 0:
        raise MplbError(EINVAL, load_library().mplb_last_error().decode())
    return n


def abi_lattice(dim):
    """Velocities (Q, 3) and weights in the library's population order
    a = (cx+1) + 3 (cy+1) [+ 9 (cz+1)]."""
    q = 9 if dim == 2 else 27
    c = np.zeros((q, 3), dtype=np.int64)
    for a in range(q):
        c[a, 0] = a % 3 - 1
        c[a, 1] = (a // 3) % 3 - 1
        if dim == 3:
            c[a, 2] = a // 9 - 1
    w1 = {-1: 1 / 6, 0: 2 / 3, 1: 1 / 6}
    w = np.array([np.prod([w1[int(v)] for v in c[a, :dim]]) for a in range(q)])
    return c, w


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


class Solver:
    """One lattice on one GPU.  ``arena`` and ``stream`` default to a fresh
    torch uint8 tensor on the current device and torch's current stream."""

    def __init__(self, case_params: dict, storage="fp32", collision=COLL_CUMULANT, arena=None,
                 stream=None, device=None):
        import torch

        lib = load_library()
        self.params = make_params(case_params, storage, collision)
        self.dim = self.params.dim
        self.n = tuple(self.params.n)
        self.N = self.n[0] * self.n[1] * self.n[2]
        self.Q = 9 if self.dim == 2 else 27
        self.nbytes = state_bytes(self.params)
        dev = torch.device(device) if device is not None else torch.device("cuda",
                                                                            torch.cuda.current_device())
        if arena is None:
            arena = torch.empty(self.nbytes + 256, dtype=torch.uint8, device=dev)
        self.arena = arena  # keep alive
        base = arena.data_ptr()
        off = (-base) % 256
        if stream is None:
            stream = torch.cuda.current_stream(dev)
        self.stream = stream
        h = ctypes.c_void_p()
        check(lib.mplb_create(ctypes.byref(self.params), ctypes.c_void_p(base + off),
                              arena.numel() - off, ctypes.c_void_p(stream.cuda_stream),
                              ctypes.byref(h)))
        self.h = h
        self._lib = lib

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and h.value:
            self._lib.mplb_destroy(h)
            self.h = None

    def _shape(self):
        return (self.n[2], self.n[1], self.n[0])

    def init(self, phi, u, p=None):
        phi = np.ascontiguousarray(phi, dtype=np.float64).reshape(-1)
        u = np.ascontiguousarray(np.asarray(u, dtype=np.float64)[:self.dim]).reshape(-1)
        assert phi.size == self.N and u.size == self.dim * self.N
        pp = None
        if p is not None:
            pp = np.ascontiguousarray(p, dtype=np.float64).reshape(-1)
            assert pp.size == self.N
        check(self._lib.mplb_init(self.h, _dptr(phi), _dptr(u), _dptr(pp) if pp is not None else None))

    def step(self, n=1):
        check(self._lib.mplb_step(self.h, int(n)))

    def step_timed(self, n):
        """n steps with per-kernel HIP events: (ms_phi, ms_collide) summed."""
        a, b = ctypes.c_double(), ctypes.c_double()
        check(self._lib.mplb_step_timed(self.h, int(n), ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def sync(self):
        check(self._lib.mplb_sync(self.h))

    def steps_done(self):
        return self._lib.mplb_steps_done(self.h)

    def read(self, field):
        out = np.empty(self.N)
        check(self._lib.mplb_read(self.h, int(field), _dptr(out)))
        return out.reshape(self._shape())

    def fields(self):
        u = np.zeros((3,) + self._shape())
        for i in range(self.dim):
            u[i] = self.read(FIELD_UX + i)
        return dict(phi=self.read(FIELD_PHI), rho=self.read(FIELD_RHO), u=u, p=self.read(FIELD_P))

    def reduce(self):
        """(sums[5], status): sum phi, sum rho u (3), max |u|."""
        out = np.zeros(5)
        rc = self._lib.mplb_reduce(self.h, _dptr(out))
        if rc not in (OK, EUNSTABLE):
            check(rc)
        return out, rc

    def reduce_noalloc(self):
        """As reduce(), with the library's static device scratch (no allocation)."""
        out = np.zeros(5)
        rc = self._lib.mplb_reduce_noalloc(self.h, _dptr(out))
        if rc not in (OK, EUNSTABLE):
            check(rc)
        return out, rc

    def get_populations(self, which):
        out = np.empty(self.Q * self.N)
        check(self._lib.mplb_get_populations(self.h, int(which), _dptr(out)))
        return out.reshape((self.Q,) + self._shape())

    def set_populations(self, which, arr):
        a = np.ascontiguousarray(arr, dtype=np.float64).reshape(-1)
        assert a.size == self.Q * self.N
        check(self._lib.mplb_set_populations(self.h, int(which), _dptr(a)))

    def save(self) -> bytes:
        """Checkpoint of the current state (mplb_save) as bytes."""
        n = self._lib.mplb_save_bytes(self.h)
        buf = ctypes.create_string_buffer(n)
        check(self._lib.mplb_save(self.h, buf, n))
        return buf.raw

    def load(self, blob: bytes):
        """Resume from a checkpoint written by save() of a solver with equal
        parameters (mplb_load)."""
        buf = ctypes.create_string_buffer(bytes(blob), len(blob))
        check(self._lib.mplb_load(self.h, buf, len(blob)))

    def set_phi_partials(self, mode=1):
        """0: phi by the pull sum each step; 1: from the partial sums the
        previous update wrote, where that applies."""
        check(self._lib.mplb_set_phi_partials(self.h, int(mode)))

    def uses_phi_partials(self):
        return self.phi_partial_rows() > 0

    def phi_partial_rows(self):
        """Tile rows of the update that sums the next phi; 0 if it does not."""
        r = self._lib.mplb_uses_phi_partials(self.h)
        if r < 0:
            check(r)
        return int(r)

    def set_block(self, bx, by, bz=1):
        check(self._lib.mplb_set_block(self.h, int(bx), int(by), int(bz)))

    def tune_block(self, steps=10, candidates=None):
        """Time candidate block shapes (advances this solver); returns
        ((bx, by, bz), ms_per_step) of the fastest, which is then in use."""
        best = (ctypes.c_int32 * 3)()
        ms = ctypes.c_double()
        if candidates is None:
            cand, nc = None, 0
        else:
            flat = [int(v) for c in candidates for v in c]
            cand, nc = (ctypes.c_int32 * len(flat))(*flat), len(candidates)
        check(self._lib.mplb_tune_block(self.h, int(steps), cand, nc, best, ctypes.byref(ms)))
        return (best[0], best[1], best[2]), ms.value


class Batch:
    """Many solvers of one dimension and storage format stepped together
    (launches over a tile list, one block per tile, hipGraph-replayed chunks)."""

    def __init__(self, dim, storage="fp32", capacity=64, max_tiles=1 << 20, stream=None,
                 device=None):
        import torch

        lib = load_library()
        self._lib = lib
        nbytes = lib.mplb_batch_table_bytes(int(capacity), int(max_tiles))
        if nbytes == 0:
            raise MplbError(EINVAL, "bad batch capacity")
        dev = torch.device(device) if device is not None else torch.device(
            "cuda", torch.cuda.current_device())
        self.table = torch.empty(nbytes + 256, dtype=torch.uint8, device=dev)
        base = self.table.data_ptr()
        off = (-base) % 256
        # a dedicated stream at the default priority: graphs cannot capture the
        # null stream; attached solvers must be created on this stream
        self.stream = stream if stream is not None else torch.cuda.Stream(dev)
        h = ctypes.c_void_p()
        st = STORAGE[storage] if isinstance(storage, str) else int(storage)
        check(lib.mplb_batch_create(int(dim), st, int(capacity), int(max_tiles),
                                    ctypes.c_void_p(base + off), nbytes,
                                    ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)))
        self.h = h
        self.capacity = int(capacity)
        self.members = {}

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and h.value:
            self._lib.mplb_batch_destroy(h)
            self.h = None

    def set_block(self, bx, by, bz=1):
        check(self._lib.mplb_batch_set_block(self.h, int(bx), int(by), int(bz)))

    def set_graph_chunk(self, chunk):
        check(self._lib.mplb_batch_set_graph_chunk(self.h, int(chunk)))

    def tune_block(self, steps=4, candidates=None):
        """Fastest block shape for the attached domains (advances them; tune a copy)."""
        best = (ctypes.c_int32 * 3)()
        ms = ctypes.c_double()
        if candidates:
            arr = (ctypes.c_int32 * (3 * len(candidates)))(*[int(v) for c in candidates for v in c])
            n = len(candidates)
        else:
            arr, n = None, 0
        check(self._lib.mplb_batch_tune_block(self.h, int(steps), arr, n, best, ctypes.byref(ms)))
        return tuple(best), ms.value

    def attach(self, solver, nsteps):
        slot = ctypes.c_int32()
        check(self._lib.mplb_batch_attach(self.h, solver.h, int(nsteps), ctypes.byref(slot)))
        self.members[slot.value] = solver
        return slot.value

    def detach(self, slot):
        check(self._lib.mplb_batch_detach(self.h, int(slot)))
        return self.members.pop(slot)

    def step(self, n):
        check(self._lib.mplb_batch_step(self.h, int(n)))

    def remaining(self, slot):
        r = ctypes.c_int64()
        check(self._lib.mplb_batch_remaining(self.h, int(slot), ctypes.byref(r)))
        return r.value

    def steps_done(self):
        return self._lib.mplb_batch_steps_done(self.h)

    def set_solo_cells(self, min_cells):
        """Domains of at least min_cells cells attached from now on step with
        their own kernels beside the shared batched launches."""
        check(self._lib.mplb_batch_set_solo_cells(self.h, int(min_cells)))

    def is_solo(self, slot):
        r = self._lib.mplb_batch_is_solo(self.h, int(slot))
        if r < 0:
            check(r)
        return bool(r)

    def status(self):
        """{slot: OK or EUNSTABLE} for the attached slots (mplb_batch_status);
        unstable slots are retired by the call."""
        cap = self.capacity
        arr = (ctypes.c_int32 * cap)()
        check(self._lib.mplb_batch_status(self.h, arr))
        return {k: int(arr[k]) for k in range(cap) if arr[k] != ESTATE}
