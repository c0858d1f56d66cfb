"""Thin Python binding of libqsv (ctypes): argument marshalling only.

Every step of the simulation runs in the library's HIP kernels; PyTorch is
used only to own device memory (the state tensor) and to supply the HIP
stream.  If ``libqsv.so`` has not been built this module raises on import of
the library -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
import re
from typing import Iterable, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqsv.so")
HEADER_PATH = os.path.join(os.path.dirname(_HERE), "include", "qsv.h")

QSV_OK, QSV_ERR_ARG, QSV_ERR_OOM, QSV_ERR_HIP, QSV_ERR_UNSUPPORTED, QSV_ERR_STATE = 0, -1, -2, -3, -4, -5
QSV_C64, QSV_C128 = 1, 2
GATES = {
    "I": 0, "X": 1, "Y": 2, "Z": 3, "H": 4, "S": 5, "SDG": 6, "T": 7, "TDG": 8,
    "RX": 9, "RY": 10, "RZ": 11, "CNOT": 12, "CZ": 13, "CPHASE": 14, "SWAP": 15, "MAT": 16,
}
NPARAMS = {"RX": 1, "RY": 1, "RZ": 1, "CPHASE": 1}
MODES = {"auto": 0, "pergate": 1, "fused": 2, "tuned": 3}


class QsvError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("qsv error %d: %s" % (code, msg))
        self.code = code


class QsvOp(ctypes.Structure):
    _fields_ = [("gate", ctypes.c_int32), ("nq", ctypes.c_int32), ("q", ctypes.c_int32 * 6),
                ("p", ctypes.c_double * 3), ("mat", ctypes.POINTER(ctypes.c_double))]


class QsvPlanOpts(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("tile_qubits", ctypes.c_int32),
                ("state_is_output", ctypes.c_int32), ("graph", ctypes.c_int32),
                ("race_check", ctypes.c_int32), ("reserved", ctypes.c_int32 * 3)]


assert ctypes.sizeof(QsvOp) == 64

_lib = None


def lib():
    """Load libqsv.so (raises if it was not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libqsv.so is not built (expected at %s); run "
                          "paper_1807_07914_amd/csrc/build.py or __graft_entry__.build()" % LIB_PATH)
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, u64p = ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_uint64)
    dp, ip = ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int32)
    sig = {
        "qsv_alloc_state": [i32, i32, vp, ctypes.c_size_t, vp, ctypes.POINTER(vp)],
        "qsv_free_state": [vp],
        "qsv_state_info": [vp, ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(vp)],
        "qsv_set_basis": [vp, ctypes.c_uint64],
        "qsv_apply_gate": [vp, i32, ip, i32, dp, i32],
        "qsv_apply_fused": [vp, ip, i32, dp],
        "qsv_apply_circuit": [vp, ctypes.POINTER(QsvOp), i32, ctypes.POINTER(QsvPlanOpts)],
        "qsv_expval": [vp, u64p, u64p, dp, i32, dp, dp],
        "qsv_expval_noalloc": [vp, i32, i32, u64p, u64p, dp, i32, vp, dp, dp],
        "qsv_norm": [vp, dp],
        "qsv_sample": [vp, dp, i32, u64p],
        "qsv_copy_to_host": [vp, vp, ctypes.c_size_t],
        "qsv_copy_from_host": [vp, vp, ctypes.c_size_t],
        "qsv_synchronize": [vp],
        "qsv_plan_info": [i32, i32, ctypes.POINTER(QsvOp), i32, i32, ctypes.POINTER(i32),
                          ctypes.POINTER(i32)],
        "qsv_adjoint": [vp, ctypes.POINTER(QsvOp), i32, u64p, u64p, dp, i32,
                        ctypes.POINTER(QsvPlanOpts), dp, dp],
        "qsv_batch_create": [i32, i32, ip, ip, ctypes.POINTER(QsvOp), ip, u64p, dp, i32,
                             ctypes.POINTER(vp)],
        "qsv_batch_update": [vp, ctypes.POINTER(QsvOp)],
        "qsv_batch_run": [vp, dp],
        "qsv_batch_info": [vp, ctypes.POINTER(i32), ctypes.POINTER(i32),
                           ctypes.POINTER(ctypes.c_int64)],
        "qsv_batch_free": [vp],
        "qsv_mps_alloc": [i32, i32, ctypes.c_double, vp, ctypes.POINTER(vp)],
        "qsv_mps_free": [vp],
        "qsv_mps_apply_circuit": [vp, ctypes.POINTER(QsvOp), i32],
        "qsv_mps_amplitudes": [vp, u64p, ctypes.c_int64, dp],
        "qsv_mps_bonds": [vp, ip, dp],
        "qsv_mps_info": [vp, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    L.qsv_last_error.argtypes = []
    L.qsv_last_error.restype = ctypes.c_char_p
    _lib = L
    return L


def expval_noalloc(amps_dev_ptr: int, n_qubits: int, dtype: str, hamiltonian, stream_ptr: int = 0,
                   per_term: bool = False):
    """qsv_expval_noalloc: the expectation value of a Pauli sum on caller-owned
    device amplitudes (a device address, e.g. a tensor's data_ptr()), with
    no device allocation by the library."""
    x, z, c = pauli_masks(hamiltonian)
    tot = ctypes.c_double()
    terms = np.zeros(max(1, len(c)), dtype=np.float64)
    dp = ctypes.POINTER(ctypes.c_double)
    u64 = ctypes.POINTER(ctypes.c_uint64)
    check(lib().qsv_expval_noalloc(ctypes.c_void_p(int(amps_dev_ptr)), int(n_qubits),
                                   QSV_C64 if dtype == "c64" else QSV_C128, x.ctypes.data_as(u64),
                                   z.ctypes.data_as(u64), c.ctypes.data_as(dp), len(c),
                                   ctypes.c_void_p(int(stream_ptr)), ctypes.byref(tot),
                                   terms.ctypes.data_as(dp)))
    return terms[: len(c)].tolist() if per_term else tot.value


def header_functions(path: str = HEADER_PATH) -> list:
    """Names of the functions declared in include/qsv.h."""
    txt = open(path).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(qsv_[a-z0-9_]+)\s*\(", txt)))


def check(rc: int) -> None:
    if rc != QSV_OK:
        msg = lib().qsv_last_error()
        raise QsvError(rc, msg.decode() if msg else "")


def _i32(xs):
    return (ctypes.c_int32 * max(1, len(xs)))(*[int(x) for x in xs])


def _f64(xs):
    return (ctypes.c_double * max(1, len(xs)))(*[float(x) for x in xs])


def pauli_masks(hamiltonian) -> tuple:
    """((coeff, ((P, q), ...)), ...) -> (xmask, zmask, coeff) arrays."""
    xs, zs, cs = [], [], []
    for c, term in hamiltonian:
        x = z = 0
        for p, q in term:
            b = 1 << int(q)
            if (x | z) & b:
                raise ValueError("qubit repeated within a Pauli string")
            if p == "X":
                x |= b
            elif p == "Z":
                z |= b
            elif p == "Y":
                x |= b
                z |= b
            else:
                raise ValueError("unknown Pauli %r" % (p,))
        xs.append(x); zs.append(z); cs.append(float(c))
    return (np.asarray(xs, dtype=np.uint64), np.asarray(zs, dtype=np.uint64),
            np.asarray(cs, dtype=np.float64))


class OpList:
    """Gate records marshalled into a contiguous qsv_op array (keeps the
    explicit matrices alive for the duration of the call)."""

    def __init__(self, ops: Iterable):
        ops = list(ops)
        self.arr = (QsvOp * max(1, len(ops)))()
        self.n = len(ops)
        self._keep = []
        for i, o in enumerate(ops):
            r = self.arr[i]
            name = o.name if o.name != "U" else "MAT"
            r.gate = GATES[name]
            r.nq = len(o.qubits)
            if r.nq > 6:
                raise ValueError("at most 6 qubits per op")
            for j, q in enumerate(o.qubits):
                r.q[j] = int(q)
            for j, p in enumerate(o.params[:3]):
                r.p[j] = float(p)
            if name == "MAT":
                m = np.ascontiguousarray(np.asarray(o.mat, dtype=np.complex128))
                self._keep.append(m)
                r.mat = m.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def plan_info(n: int, dtype: str, ops, tile_qubits: int = 0) -> dict:
    """Tile passes and separately launched ops of the fused plan (host only)."""
    ol = ops if isinstance(ops, OpList) else OpList(ops)
    p, f = ctypes.c_int(), ctypes.c_int()
    check(lib().qsv_plan_info(int(n), QSV_C64 if dtype == "c64" else QSV_C128, ol.arr, ol.n,
                              int(tile_qubits), ctypes.byref(p), ctypes.byref(f)))
    return {"passes": p.value, "separate_ops": f.value}


class State:
    """A device-resident state vector of n qubits (complex64 or complex128)
    whose storage is a torch CUDA tensor owned by this object (or borrowed)."""

    def __init__(self, n: int, dtype: str = "c64", device: int = 0, tensor=None, stream=None):
        import torch
        if dtype not in ("c64", "c128"):
            raise ValueError("dtype must be 'c64' or 'c128'")
        self.n = int(n)
        self.dtype = dtype
        tdt = torch.complex64 if dtype == "c64" else torch.complex128
        if tensor is None:
            tensor = torch.empty(1 << self.n, dtype=tdt, device="cuda:%d" % device)
        if tensor.dtype != tdt or not tensor.is_cuda or not tensor.is_contiguous():
            raise ValueError("tensor must be a contiguous CUDA tensor of the state dtype")
        self.tensor = tensor
        if stream is None:
            stream = torch.cuda.current_stream(tensor.device)
        self.stream = stream
        h = ctypes.c_void_p()
        check(lib().qsv_alloc_state(self.n, QSV_C64 if dtype == "c64" else QSV_C128,
                                    ctypes.c_void_p(tensor.data_ptr()),
                                    tensor.numel() * tensor.element_size(),
                                    ctypes.c_void_p(stream.cuda_stream), ctypes.byref(h)))
        self._h = h

    # -- lifetime ---------------------------------------------------------
    @property
    def handle(self):
        if self._h is None:
            raise QsvError(QSV_ERR_STATE, "state already closed")
        return self._h

    def close(self):
        if getattr(self, "_h", None) is not None:
            check(lib().qsv_free_state(self._h))
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

    # -- gates ------------------------------------------------------------
    def set_basis(self, x: int) -> None:
        check(lib().qsv_set_basis(self.handle, int(x)))

    def apply_gate(self, name: str, qubits: Sequence[int], params: Sequence[float] = ()) -> None:
        check(lib().qsv_apply_gate(self.handle, GATES[name], _i32(qubits), len(qubits),
                                   _f64(params), len(params)))

    def apply_fused(self, qubits: Sequence[int], mat) -> None:
        m = np.ascontiguousarray(np.asarray(mat, dtype=np.complex128))
        check(lib().qsv_apply_fused(self.handle, _i32(qubits), len(qubits),
                                    m.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))

    def apply_circuit(self, ops, mode: str = "auto", tile_qubits: int = 0, graph: bool = False,
                      race_check: bool = False) -> None:
        """Apply a gate list.  graph=True launches the fused plan's passes as
        the state's hipGraph (captured once per plan structure, replayed with
        this call's angles); the state must be on a non-null stream.
        race_check=True runs every fused pass out of place into a poisoned
        buffer first and raises QsvError if an amplitude was left unwritten
        or differs from the in-place pass."""
        ol = ops if isinstance(ops, OpList) else OpList(ops)
        opts = QsvPlanOpts()
        opts.mode = MODES[mode]
        opts.tile_qubits = int(tile_qubits)
        opts.graph = 1 if graph else 0
        opts.race_check = 1 if race_check else 0
        check(lib().qsv_apply_circuit(self.handle, ol.arr, ol.n, ctypes.byref(opts)))

    def plan_info(self, ops, tile_qubits: int = 0) -> dict:
        return plan_info(self.n, self.dtype, ops, tile_qubits)

    # -- reductions -------------------------------------------------------
    def expval(self, hamiltonian, per_term: bool = False):
        x, z, c = pauli_masks(hamiltonian)
        tot = ctypes.c_double()
        terms = np.zeros(max(1, len(c)), dtype=np.float64)
        dp = ctypes.POINTER(ctypes.c_double)
        check(lib().qsv_expval(self.handle, x.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                               z.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                               c.ctypes.data_as(dp), len(c), ctypes.byref(tot),
                               terms.ctypes.data_as(dp)))
        return terms[: len(c)].tolist() if per_term else tot.value

    def adjoint(self, ops, hamiltonian, mode: str = "auto", tile_qubits: int = 0,
                state_is_output: bool = False):
        """Apply ops to the current state, return (E, dE/dtheta per op) from
        one adjoint sweep; the state holds its input again afterwards.  With
        state_is_output the state already holds the ops' output (an earlier
        apply_circuit of the same ops) and the ops are not applied again."""
        ol = ops if isinstance(ops, OpList) else OpList(ops)
        x, z, c = pauli_masks(hamiltonian)
        opts = QsvPlanOpts()
        opts.mode = MODES[mode]
        opts.tile_qubits = int(tile_qubits)
        opts.state_is_output = 1 if state_is_output else 0
        e = ctypes.c_double()
        g = np.zeros(max(1, ol.n), dtype=np.float64)
        dp = ctypes.POINTER(ctypes.c_double)
        u64 = ctypes.POINTER(ctypes.c_uint64)
        check(lib().qsv_adjoint(self.handle, ol.arr, ol.n, x.ctypes.data_as(u64),
                                z.ctypes.data_as(u64), c.ctypes.data_as(dp), len(c),
                                ctypes.byref(opts), ctypes.byref(e), g.ctypes.data_as(dp)))
        return e.value, g[: ol.n]

    def norm(self) -> float:
        out = ctypes.c_double()
        check(lib().qsv_norm(self.handle, ctypes.byref(out)))
        return out.value

    def sample(self, uniforms) -> np.ndarray:
        u = np.ascontiguousarray(uniforms, dtype=np.float64)
        out = np.zeros(u.size, dtype=np.uint64)
        check(lib().qsv_sample(self.handle, u.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                               int(u.size), out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))))
        return out

    # -- copies -----------------------------------------------------------
    def to_numpy(self) -> np.ndarray:
        out = np.empty(1 << self.n, dtype=np.complex64 if self.dtype == "c64" else np.complex128)
        check(lib().qsv_copy_to_host(self.handle, out.ctypes.data_as(ctypes.c_void_p), out.nbytes))
        return out

    def from_numpy(self, a: np.ndarray) -> None:
        a = np.ascontiguousarray(a, dtype=np.complex64 if self.dtype == "c64" else np.complex128)
        check(lib().qsv_copy_from_host(self.handle, a.ctypes.data_as(ctypes.c_void_p), a.nbytes))

    def synchronize(self) -> None:
        check(lib().qsv_synchronize(self.handle))


class Batch:
    """Many independent circuits (uneven widths, each from |0...0>) evaluated
    by one persistent kernel replayed from a HIP graph.  ``hamiltonians[i]``
    must contain Z-strings only; ``run()`` returns one FP64 energy per circuit."""

    def __init__(self, circuits, widths, hamiltonians, dtype: str = "c64", tile_qubits: int = 0):
        circuits = [list(c) for c in circuits]
        self.n = len(circuits)
        self.dtype = dtype
        self._offsets = np.zeros(self.n + 1, dtype=np.int32)
        flat = []
        for i, c in enumerate(circuits):
            flat += c
            self._offsets[i + 1] = len(flat)
        toff = np.zeros(self.n + 1, dtype=np.int32)
        zs, cs = [], []
        for i, ham in enumerate(hamiltonians):
            x, z, c = pauli_masks(ham)
            if np.any(x != 0):
                raise ValueError("batched Hamiltonians must be diagonal (Z-strings only)")
            zs += list(z)
            cs += list(c)
            toff[i + 1] = len(zs)
        self._z = np.ascontiguousarray(zs, dtype=np.uint64) if zs else np.zeros(1, np.uint64)
        self._c = np.ascontiguousarray(cs, dtype=np.float64) if cs else np.zeros(1, np.float64)
        self._toff = toff
        self._w = np.ascontiguousarray(widths, dtype=np.int32)
        ol = OpList(flat)
        h = ctypes.c_void_p()
        check(lib().qsv_batch_create(QSV_C64 if dtype == "c64" else QSV_C128, self.n,
                                     _ptr_i32(self._w), _ptr_i32(self._offsets), ol.arr,
                                     _ptr_i32(self._toff),
                                     self._z.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                                     self._c.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                     int(tile_qubits), ctypes.byref(h)))
        self._h = h

    def update(self, circuits) -> None:
        flat = [o for c in circuits for o in c]
        if len(flat) != int(self._offsets[-1]):
            raise ValueError("op count differs from the batch structure")
        check(lib().qsv_batch_update(self._h, OpList(flat).arr))

    def run(self) -> np.ndarray:
        out = np.zeros(self.n, dtype=np.float64)
        check(lib().qsv_batch_run(self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return out

    def info(self) -> dict:
        t, p, sb = ctypes.c_int(), ctypes.c_int(), ctypes.c_int64()
        check(lib().qsv_batch_info(self._h, ctypes.byref(t), ctypes.byref(p), ctypes.byref(sb)))
        return {"tile_qubits": t.value, "passes": p.value, "scratch_bytes": sb.value}

    def close(self) -> None:
        if getattr(self, "_h", None) is not None:
            check(lib().qsv_batch_free(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


MPS_MAX_CHI = 64        # bond cap the library accepts (its slot stride)
MPS_DEFAULT_CHI = 32    # bonds up to this size keep the whole SVD in LDS


class MPS:
    """Matrix-product state on the GPU (complex128 site tensors, Schmidt
    coefficients per bond); qubit q lives at site q.  Gates are applied by
    two-site SVD updates with the given cutoff and bond-dimension cap."""

    def __init__(self, n: int, chi_max: int = MPS_DEFAULT_CHI, cutoff: float = 1e-4, stream=None):
        self.n = n
        h = ctypes.c_void_p()
        st = ctypes.c_void_p(stream.cuda_stream if stream is not None else None)
        check(lib().qsv_mps_alloc(int(n), int(chi_max), float(cutoff), st, ctypes.byref(h)))
        self._h = h

    def apply_circuit(self, ops) -> None:
        ol = ops if isinstance(ops, OpList) else OpList(ops)
        check(lib().qsv_mps_apply_circuit(self._h, ol.arr, ol.n))

    def amplitudes(self, idx) -> np.ndarray:
        idx = np.ascontiguousarray(idx, dtype=np.uint64)
        out = np.zeros(2 * max(1, idx.size), dtype=np.float64)
        check(lib().qsv_mps_amplitudes(self._h, idx.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                                       idx.size, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return out[: 2 * idx.size].view(np.complex128)

    def to_numpy(self) -> np.ndarray:
        return self.amplitudes(np.arange(1 << self.n, dtype=np.uint64))

    def bonds(self):
        """(dims list of n+1, Schmidt coefficients per bond as a list of arrays)."""
        dims = np.zeros(self.n + 1, dtype=np.int32)
        lam = np.zeros((self.n + 1) * MPS_MAX_CHI, dtype=np.float64)
        check(lib().qsv_mps_bonds(self._h, _ptr_i32(dims),
                                  lam.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        lam = lam.reshape(self.n + 1, MPS_MAX_CHI)
        return [int(d) for d in dims], [lam[b, : dims[b]].copy() for b in range(self.n + 1)]

    def info(self) -> dict:
        b, l = ctypes.c_int64(), ctypes.c_int64()
        check(lib().qsv_mps_info(self._h, ctypes.byref(b), ctypes.byref(l)))
        return {"bond_updates": b.value, "launches": l.value}

    def memory_bytes(self) -> int:
        """Bytes of the site tensors and Schmidt vectors at their current
        dimensions (complex128 / float64), the paper's O(n chi^2) measure."""
        d, _ = self.bonds()
        return sum(d[l] * 2 * d[l + 1] * 16 for l in range(self.n)) + sum(8 * x for x in d)

    def close(self) -> None:
        if getattr(self, "_h", None) is not None:
            check(lib().qsv_mps_free(self._h))
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _ptr_i32(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
