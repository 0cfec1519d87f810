"""ctypes binding of libtersoff.so (argument marshalling only).

Every step of the evaluation runs in the HIP kernels of the library; this
module only checks tensor shapes, dtypes and devices and passes raw pointers
and the current torch stream.  If the library is missing it raises: there is
no fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtersoff.so")

FP64 = 0
MIXED = 1
SINGLE = 2
PRECISIONS = {"fp64": FP64, "mixed": MIXED, "single": SINGLE}

OK = 0
STATUS = {0: "OK", -1: "E_INVALID", -2: "E_NOMEM", -3: "E_BOX", -4: "E_OVERFLOW", -5: "E_STALE",
          -6: "E_DEVICE", -7: "E_AGAIN", -8: "E_PENDING", -9: "E_STATE"}

# exported symbols (the declarations of include/tersoff.h)
SYMBOLS = ("tersoff_create", "tersoff_destroy", "tersoff_build_neighbors", "tersoff_compute",
           "tersoff_compute_static", "tersoff_set_force_sum", "tersoff_set_mapping", "tersoff_set_packing", "tersoff_check", "tersoff_get_neighbors", "tersoff_get_counts", "tersoff_num_atoms",
           "tersoff_strerror", "tersoff_last_error", "tersoff_profile", "tersoff_profile_read",
           "tersoff_set_batch_atoms", "tersoff_serve_start", "tersoff_serve_stop", "tersoff_submit",
           "tersoff_poll", "tersoff_serve_stats", "tersoff_clock_ns", "tersoff_parse_params",
           "tersoff_md_run")


class ServeConfig(ctypes.Structure):
    _fields_ = [("max_batch_atoms", ctypes.c_int64), ("max_batch_systems", ctypes.c_int32),
                ("max_neighbors", ctypes.c_int32), ("cutoff", ctypes.c_double), ("skin", ctypes.c_double),
                ("max_queued", ctypes.c_int64), ("host_threads", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class Request(ctypes.Structure):
    _fields_ = [("pos", ctypes.c_void_p), ("types", ctypes.c_void_p), ("n", ctypes.c_int64),
                ("box", ctypes.c_double * 3), ("precision", ctypes.c_int32), ("forces", ctypes.c_void_p),
                ("tag", ctypes.c_uint64), ("release_ns", ctypes.c_int64)]


class MDConfig(ctypes.Structure):
    _fields_ = [("dt", ctypes.c_double), ("nsteps", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("mass", ctypes.c_void_p), ("cutoff", ctypes.c_double), ("skin", ctypes.c_double)]


class Result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("batch_systems", ctypes.c_int32), ("n", ctypes.c_int64),
                ("energy", ctypes.c_double), ("virial", ctypes.c_double * 6), ("latency_ms", ctypes.c_double),
                ("tag", ctypes.c_uint64)]

_lib = None


class TersoffError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status


def load():
    """Load libtersoff.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_1710_00882_amd.build` (no CPU fallback exists)")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    i32, i64, f64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    lib.tersoff_create.argtypes = [P, i32, ctypes.POINTER(P)]
    lib.tersoff_create.restype = ctypes.c_int
    lib.tersoff_destroy.argtypes = [P]
    lib.tersoff_destroy.restype = None
    lib.tersoff_build_neighbors.argtypes = [P, P, P, i64, P, f64, f64, P]
    lib.tersoff_build_neighbors.restype = ctypes.c_int
    lib.tersoff_compute.argtypes = [P, P, i32, P, P, P]
    lib.tersoff_compute.restype = ctypes.c_int
    lib.tersoff_compute_static.argtypes = [P, P, i32, P, P, P]
    lib.tersoff_compute_static.restype = ctypes.c_int
    lib.tersoff_set_force_sum.argtypes = [P, i32]
    lib.tersoff_set_force_sum.restype = ctypes.c_int
    lib.tersoff_set_mapping.argtypes = [P, i32]
    lib.tersoff_set_mapping.restype = ctypes.c_int
    lib.tersoff_set_packing.argtypes = [P, i32]
    lib.tersoff_set_packing.restype = ctypes.c_int
    lib.tersoff_check.argtypes = [P, P]
    lib.tersoff_check.restype = ctypes.c_int
    lib.tersoff_get_neighbors.argtypes = [P, P, P, i64, P]
    lib.tersoff_get_neighbors.restype = ctypes.c_int
    lib.tersoff_get_counts.argtypes = [P, P]
    lib.tersoff_get_counts.restype = ctypes.c_int
    lib.tersoff_num_atoms.argtypes = [P]
    lib.tersoff_num_atoms.restype = i64
    lib.tersoff_profile.argtypes = [P, i32]
    lib.tersoff_profile.restype = ctypes.c_int
    lib.tersoff_profile_read.argtypes = [P, P]
    lib.tersoff_profile_read.restype = ctypes.c_int
    lib.tersoff_set_batch_atoms.argtypes = [P, i32]
    lib.tersoff_set_batch_atoms.restype = ctypes.c_int
    lib.tersoff_strerror.argtypes = [ctypes.c_int]
    lib.tersoff_strerror.restype = ctypes.c_char_p
    lib.tersoff_last_error.argtypes = [P]
    lib.tersoff_last_error.restype = ctypes.c_char_p
    lib.tersoff_serve_start.argtypes = [P, ctypes.POINTER(ServeConfig)]
    lib.tersoff_serve_start.restype = ctypes.c_int
    lib.tersoff_serve_stop.argtypes = [P]
    lib.tersoff_serve_stop.restype = ctypes.c_int
    lib.tersoff_submit.argtypes = [P, ctypes.POINTER(Request), ctypes.POINTER(ctypes.c_uint64)]
    lib.tersoff_submit.restype = ctypes.c_int
    lib.tersoff_poll.argtypes = [P, ctypes.c_uint64, f64, ctypes.POINTER(Result)]
    lib.tersoff_poll.restype = ctypes.c_int
    lib.tersoff_serve_stats.argtypes = [P, P]
    lib.tersoff_serve_stats.restype = ctypes.c_int
    lib.tersoff_clock_ns.argtypes = []
    lib.tersoff_clock_ns.restype = i64
    lib.tersoff_parse_params.argtypes = [ctypes.c_char_p, ctypes.POINTER(ctypes.c_char_p), i32, P]
    lib.tersoff_parse_params.restype = ctypes.c_int
    lib.tersoff_md_run.argtypes = [P, P, P, P, P, i64, P, ctypes.POINTER(MDConfig), P, P]
    lib.tersoff_md_run.restype = ctypes.c_int
    _lib = lib
    return lib


def _stream_ptr(torch, device=None) -> int:
    return int(torch.cuda.current_stream(device).cuda_stream)


def _check_dev(t, dtype, shape_tail, name):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape_tail is not None and tuple(t.shape[1:]) != shape_tail:
        raise ValueError(f"{name} must have shape (n, {', '.join(map(str, shape_tail))})")


class Tersoff:
    """One context of libtersoff.so: parameter table, resident neighbour list."""

    def __init__(self, table):
        lib = load()
        tab = np.ascontiguousarray(table, dtype=np.float64)
        nt = int(round((tab.size // 14) ** (1.0 / 3.0)))
        if nt ** 3 * 14 != tab.size:
            raise ValueError("table must hold ntypes^3 entries of 14 values")
        self._table = tab
        self.ntypes = nt
        h = ctypes.c_void_p()
        st = lib.tersoff_create(tab.ctypes.data_as(ctypes.c_void_p), nt, ctypes.byref(h))
        if st != OK:
            raise TersoffError(st, "tersoff_create rejected the parameter table")
        self._h = h
        self._lib = lib
        self.cutoff = float(np.max(tab.reshape(-1, 14)[:, 11] + tab.reshape(-1, 14)[:, 12]))

    def close(self):
        if getattr(self, "_h", None):
            self._lib.tersoff_destroy(self._h)
            self._h = None
            self._held = {}

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _raise(self, st, what):
        msg = self._lib.tersoff_last_error(self._h).decode()
        raise TersoffError(st, f"{what}: {msg}")

    @property
    def n(self) -> int:
        return int(self._lib.tersoff_num_atoms(self._h))

    def build_neighbors(self, pos, types, box, cutoff=None, skin=1.0):
        import torch
        _check_dev(pos, torch.float64, (3,), "pos")
        _check_dev(types, torch.int32, None, "types")
        if types.shape != (pos.shape[0],):
            raise ValueError("types must have shape (n,)")
        b = np.ascontiguousarray(np.asarray(box, dtype=np.float64).reshape(3))
        cut = self.cutoff if cutoff is None else float(cutoff)
        st = self._lib.tersoff_build_neighbors(self._h, pos.data_ptr(), types.data_ptr(), pos.shape[0],
                                               b.ctypes.data_as(ctypes.c_void_p), cut, float(skin),
                                               _stream_ptr(torch, pos.device))
        if st != OK:
            self._raise(st, "tersoff_build_neighbors")

    def compute(self, pos, precision="mixed", forces=None, out=None, want_forces=True, static=False):
        """Returns (out, forces): out = [E, Wxx, Wyy, Wzz, Wxy, Wxz, Wyz] (device).
        static=True calls tersoff_compute_static (no allocation by the library;
        the caller's out and forces tensors are allocated here when not given)."""
        import torch
        _check_dev(pos, torch.float64, (3,), "pos")
        if out is None:
            out = torch.empty(7, dtype=torch.float64, device=pos.device)
        if want_forces and forces is None:
            forces = torch.empty_like(pos)
        if forces is not None:
            _check_dev(forces, torch.float64, (3,), "forces")
        fn = self._lib.tersoff_compute_static if static else self._lib.tersoff_compute
        st = fn(self._h, pos.data_ptr(), PRECISIONS[precision], out.data_ptr(),
                forces.data_ptr() if forces is not None else None, _stream_ptr(torch, pos.device))
        if st != OK:
            self._raise(st, "tersoff_compute_static" if static else "tersoff_compute")
        return out, forces

    def check(self):
        import torch
        st = self._lib.tersoff_check(self._h, _stream_ptr(torch))
        if st != OK:
            self._raise(st, "tersoff_check")

    def check_status(self) -> int:
        import torch
        return int(self._lib.tersoff_check(self._h, _stream_ptr(torch)))

    def neighbors(self):
        n = self.n
        offsets = np.zeros(n + 1, dtype=np.int64)
        total = ctypes.c_int64(0)
        st = self._lib.tersoff_get_neighbors(self._h, offsets.ctypes.data_as(ctypes.c_void_p), None, 0,
                                             ctypes.byref(total))
        if total.value == 0 and st == OK:
            return offsets, np.zeros(0, dtype=np.int32)
        idx = np.zeros(total.value, dtype=np.int32)
        st = self._lib.tersoff_get_neighbors(self._h, offsets.ctypes.data_as(ctypes.c_void_p),
                                             idx.ctypes.data_as(ctypes.c_void_p), idx.size,
                                             ctypes.byref(total))
        if st != OK:
            self._raise(st, "tersoff_get_neighbors")
        return offsets, idx

    def profile(self, enable: bool = True):
        st = self._lib.tersoff_profile(self._h, 1 if enable else 0)
        if st != OK:
            self._raise(st, "tersoff_profile")

    def profile_read(self):
        """Since the last read: dict of summed event times (ms) and launch counts
        of the main kernel, the neighbour builds and the force-gather kernel."""
        out = np.zeros(8)
        st = self._lib.tersoff_profile_read(self._h, out.ctypes.data_as(ctypes.c_void_p))
        if st != OK:
            self._raise(st, "tersoff_profile_read")
        return dict(kernel_ms=float(out[0]), kernels=int(out[1]), build_ms=float(out[2]),
                    builds=int(out[3]), gather_ms=float(out[4]), gathers=int(out[5]),
                    pack_ms=float(out[6]), packs=int(out[7]))

    def set_force_sum(self, mode: str):
        """'planes' (default: atomic-free, reproducible) or 'atomic' (FP64
        atomic scatter, the comparison point)."""
        st = self._lib.tersoff_set_force_sum(self._h, {"planes": 0, "atomic": 1}[mode])
        if st != OK:
            self._raise(st, "tersoff_set_force_sum")

    def set_mapping(self, mode: str):
        """'pair' (default: a lane per packed pair) or 'triplet' (a lane per
        triplet, the comparison point; FP64 and mixed)."""
        st = self._lib.tersoff_set_mapping(self._h, {"pair": 0, "triplet": 1}[mode])
        if st != OK:
            self._raise(st, "tersoff_set_mapping")

    def set_packing(self, mode: str):
        """'separate' (default: a packing kernel writes records to memory) or
        'fused' (packed inside the compute kernel where rows allow)."""
        st = self._lib.tersoff_set_packing(self._h, {"separate": 0, "fused": 1}[mode])
        if st != OK:
            self._raise(st, "tersoff_set_packing")

    def set_batch_atoms(self, atoms: int):
        st = self._lib.tersoff_set_batch_atoms(self._h, int(atoms))
        if st != OK:
            self._raise(st, "tersoff_set_batch_atoms")

    def counts(self):
        c = np.zeros(3, dtype=np.int64)
        st = self._lib.tersoff_get_counts(self._h, c.ctypes.data_as(ctypes.c_void_p))
        if st != OK:
            self._raise(st, "tersoff_get_counts")
        return tuple(int(v) for v in c)

    def md_run(self, pos, vel, types, box, masses, dt, nsteps, precision="fp64", cutoff=0.0, skin=1.0, forces=None):
        """Velocity-Verlet NVE on device arrays (advanced in place).  Returns a
        dict: epot, ekin (eV), builds, temperature (K), and the forces tensor."""
        import torch
        _check_dev(pos, torch.float64, (3,), "pos")
        _check_dev(vel, torch.float64, (3,), "vel")
        _check_dev(types, torch.int32, None, "types")
        if forces is None:
            forces = torch.empty_like(pos)
        _check_dev(forces, torch.float64, (3,), "forces")
        m = np.ascontiguousarray(np.asarray(masses, dtype=np.float64).reshape(-1))
        if m.size != self.ntypes:
            raise ValueError("one mass per type")
        b = np.ascontiguousarray(np.asarray(box, dtype=np.float64).reshape(3))
        cfg = MDConfig(float(dt), int(nsteps), PRECISIONS[precision], m.ctypes.data, float(cutoff), float(skin))
        out = np.zeros(4)
        st = self._lib.tersoff_md_run(self._h, pos.data_ptr(), vel.data_ptr(), forces.data_ptr(), types.data_ptr(),
                                      pos.shape[0], b.ctypes.data_as(ctypes.c_void_p), ctypes.byref(cfg),
                                      out.ctypes.data_as(ctypes.c_void_p), _stream_ptr(torch, pos.device))
        if st != OK:
            self._raise(st, "tersoff_md_run")
        return dict(epot=float(out[0]), ekin=float(out[1]), builds=int(out[2]), temperature=float(out[3]),
                    forces=forces)

    # ---- serving -------------------------------------------------------------
    def serve_start(self, max_batch_atoms, max_batch_systems, max_neighbors=0, cutoff=0.0, skin=1.0,
                    max_queued=0, host_threads=0):
        cfg = ServeConfig(int(max_batch_atoms), int(max_batch_systems), int(max_neighbors), float(cutoff),
                          float(skin), int(max_queued), int(host_threads), 0)
        st = self._lib.tersoff_serve_start(self._h, ctypes.byref(cfg))
        if st != OK:
            self._raise(st, "tersoff_serve_start")
        self._held = {}

    def serve_stop(self):
        st = self._lib.tersoff_serve_stop(self._h)
        self._held = {}
        if st != OK:
            self._raise(st, "tersoff_serve_stop")

    def submit(self, pos, types, box, precision="mixed", forces=None, tag=0, release_ns=0):
        """Queue one configuration: host numpy arrays, or torch tensors on the
        context's GPU (device-resident buffers), kept alive here until its
        result is collected.  Returns the ticket; raises TersoffError (status
        E_AGAIN when the queue is full)."""
        def dev(t):
            return hasattr(t, "is_cuda") and t.is_cuda

        def ptr(t):
            return t.data_ptr() if dev(t) else t.ctypes.data

        if dev(pos):
            import torch
            _check_dev(pos, torch.float64, (3,), "pos")
        if dev(types):
            import torch
            if types.dtype != torch.int32 or not types.is_contiguous():
                raise ValueError("device types must be a contiguous int32 tensor")
        if not dev(pos):
            pos = np.ascontiguousarray(pos, dtype=np.float64)
        if not dev(types):
            types = np.ascontiguousarray(types, dtype=np.int32)
        n = pos.shape[0]
        if len(pos.shape) != 2 or pos.shape[1] != 3 or tuple(types.shape) != (n,):
            raise ValueError("pos must be (n, 3) and types (n,)")
        if forces is not None:
            if dev(forces):
                import torch
                _check_dev(forces, torch.float64, (3,), "forces")
                if tuple(forces.shape) != (n, 3):
                    raise ValueError("forces must be shaped like pos")
            elif forces.dtype != np.float64 or forces.shape != (n, 3) or not forces.flags.c_contiguous:
                raise ValueError("forces must be a C-contiguous float64 array shaped like pos")
        req = Request()
        req.pos = ptr(pos)
        req.types = ptr(types)
        req.n = n
        for a, v in enumerate(np.asarray(box, dtype=np.float64).reshape(3)):
            req.box[a] = float(v)
        req.precision = PRECISIONS[precision]
        req.forces = ptr(forces) if forces is not None else None
        req.tag = int(tag)
        req.release_ns = int(release_ns)
        t = ctypes.c_uint64(0)
        st = self._lib.tersoff_submit(self._h, ctypes.byref(req), ctypes.byref(t))
        if st != OK:
            raise TersoffError(st, "tersoff_submit rejected the request")
        self._held[t.value] = (pos, types, forces)
        return t.value

    def poll(self, ticket, timeout_ms=0.0):
        """Result dict of a ticket, or None while it is pending."""
        r = Result()
        st = self._lib.tersoff_poll(self._h, int(ticket), float(timeout_ms), ctypes.byref(r))
        if st == -8:
            return None
        if st != OK:
            raise TersoffError(st, "tersoff_poll")
        held = self._held.pop(int(ticket), (None, None, None))
        return dict(status=int(r.status), energy=float(r.energy), virial=np.array(r.virial[:]),
                    latency_ms=float(r.latency_ms), tag=int(r.tag), n=int(r.n),
                    batch_systems=int(r.batch_systems), forces=held[2])

    def wait(self, ticket, timeout_ms=60000.0):
        res = self.poll(ticket, timeout_ms)
        if res is None:
            raise TimeoutError(f"ticket {ticket} not ready after {timeout_ms} ms")
        return res

    def serve_stats(self):
        out = np.zeros(6)
        st = self._lib.tersoff_serve_stats(self._h, out.ctypes.data_as(ctypes.c_void_p))
        if st != OK:
            self._raise(st, "tersoff_serve_stats")
        return dict(batches=int(out[0]), systems=int(out[1]), atoms=int(out[2]), device_bytes=int(out[3]),
                    max_batch_atoms=int(out[4]), max_batch_systems=int(out[5]))


def clock_ns() -> int:
    """The library's monotonic clock (the time base of release_ns)."""
    return int(load().tersoff_clock_ns())


def parse_params(text: str, elements) -> np.ndarray:
    """Parameter table (ntypes^3 x 14) from a LAMMPS-format Tersoff parameter
    file's text; type t is elements[t]."""
    lib = load()
    names = [e.encode() for e in elements]
    arr = (ctypes.c_char_p * len(names))(*names)
    nt = len(names)
    out = np.zeros(nt ** 3 * 14)
    st = lib.tersoff_parse_params(text.encode(), arr, nt, out.ctypes.data_as(ctypes.c_void_p))
    if st != OK:
        raise TersoffError(st, "tersoff_parse_params rejected the file")
    return out.reshape(nt ** 3, 14)
