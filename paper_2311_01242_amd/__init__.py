"""MI355X-native VQE statevector engine (thin Python binding over libvqe.so).

Every step of the hot path runs in the library's HIP kernels; this module
only marshals arguments.  PyTorch is used, when present, for the HIP stream
of the caller (``torch.cuda.current_stream()``) and for device tensors that a
statevector may borrow.

Method (arXiv:2311.01242): VQE objective E(theta) = <HF|U^dag H U|HF>
(Sec. 2.1.1, Eq. 1) for the Jordan-Wigner form of Eq. 2 and a UCCSD ansatz
(Sec. 2.1.2); gradients by an adjoint reverse sweep; BFGS (Sec. 3.1).
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _lib
from ._lib import Options, Result, lib

VQE_OK, VQE_EINVAL, VQE_ERANGE, VQE_ENOMEM, VQE_EDEVICE, VQE_ENUMERIC = 0, -1, -2, -3, -4, -5

__all__ = [
    "VQEError", "Hamiltonian", "Ansatz", "State", "Batch", "energy_grad", "energy_grad_noalloc", "EnergyGrad",
    "minimize_bfgs", "run_vqe", "Options", "Result", "lib", "current_stream", "set_tuning",
    "set_packed", "set_real", "real_enabled", "set_run_threads", "copy_ceiling", "lds_ceiling", "set_persistent", "set_tile_cap",
]


def set_tuning(n_qubits: int, batched: bool, fwd_lds_bytes: int = 0, adj_lds_bytes: int = 0,
               hx_tile_bits: int = 0):
    """Override the launch parameters for n_qubits (all zeros: built-in choice)."""
    _check(lib().vqe_set_tuning(int(n_qubits), int(bool(batched)), int(fwd_lds_bytes),
                                int(adj_lds_bytes), int(hx_tile_bits)))


def set_run_threads(n_qubits: int, batched: bool, fwd_threads: int = 0, adj_threads: int = 0):
    """Least threads per packed run tile (64/256/512/1024; zeros: built-in)."""
    _check(lib().vqe_set_run_threads(int(n_qubits), int(bool(batched)), int(fwd_threads),
                                     int(adj_threads)))


def set_packed(mode=True):
    """Evaluation layout of UCCSD programs (applies to plans made afterwards):
    True or 2 = packed sector layout with the string-product H-apply (the
    default), 1 = packed layout with the block-order H-apply, False or 0 =
    full 2^n vectors."""
    m = 2 if mode is True else (0 if mode is False else int(mode))
    _check(lib().vqe_set_packed(m))


_real = [True]


def set_real(on=True):
    """Real amplitudes on the string-product path (the default; applies to
    plans made afterwards): phi and lambda of excitation programs are real, so
    one double per amplitude is stored instead of two.  False keeps complex
    amplitudes there."""
    _check(lib().vqe_set_real(int(bool(on))))
    _real[0] = bool(on)


def real_enabled():
    """Whether plans made now use real amplitudes on the string-product path."""
    return _real[0]


def set_tile_cap(n_qubits: int, batched: bool, entries: int = 0):
    """Largest packed run tile (entries per vector) for n_qubits; 0 = the
    default (2400 entries, or two of the layout's largest blocks when they
    hold more).  Applies to plans made afterwards."""
    _check(lib().vqe_set_tile_cap(int(n_qubits), int(bool(batched)), int(entries)))


def set_persistent(mode: bool = True, block_bits: int = 0):
    """Persistent batch gate passes on or off (off by default); block_bits:
    the common block bits of their packed layout (0 = 12).  Applies to
    batches created afterwards."""
    _check(lib().vqe_set_persistent(int(bool(mode)), int(block_bits)))


def copy_ceiling(src, dst, passes: int = 1) -> float:
    """Milliseconds of one library launch that copies the bytes of device
    tensor src into dst `passes` times (a measured bandwidth ceiling for the
    rooflines, not a step of the method).  Same-size contiguous tensors."""
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nbytes or not (src.is_contiguous() and dst.is_contiguous()):
        raise ValueError("src and dst must be contiguous tensors of the same byte size")
    ms = C.c_double()
    _check(lib().vqe_copy_ceiling(C.c_void_p(src.data_ptr()), C.c_void_p(dst.data_ptr()),
                                  int(nbytes), int(passes), current_stream(), C.byref(ms)))
    return ms.value


def lds_ceiling(iters: int = 4000):
    """(milliseconds, bytes) of one library launch that reads and writes back
    LDS on every compute unit `iters` times (a measured on-chip ceiling for
    the gate kernels, not a step of the method)."""
    ms, nb = C.c_double(), C.c_double()
    _check(lib().vqe_lds_ceiling(int(iters), current_stream(), C.byref(ms), C.byref(nb)))
    return ms.value, nb.value


_MAPS = {"jw": 0, "bk": 1}


class VQEError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"[{code}] {msg}")
        self.code = code


def _check(rc: int):
    if rc != VQE_OK:
        raise VQEError(rc, lib().vqe_last_error().decode(errors="replace"))


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _u32(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_uint32))


def current_stream():
    """hipStream_t of torch's current stream on the current device, or None."""
    try:
        import torch
        if torch.cuda.is_available():
            return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    except ImportError:
        pass
    return None


class Hamiltonian:
    """Jordan-Wigner qubit Hamiltonian (folded real form c' X^x Z^z)."""

    def __init__(self, handle):
        self._h = handle

    @classmethod
    def from_integrals(cls, n_qubits: int, h0: float, h, g):
        h = np.ascontiguousarray(h, dtype=np.float64)
        g = np.ascontiguousarray(g, dtype=np.float64)
        out = C.c_void_p()
        _check(lib().vqe_hamiltonian_from_integrals(int(n_qubits), float(h0), _dptr(h), _dptr(g),
                                                    C.byref(out)))
        return cls(out)

    @classmethod
    def from_integrals_map(cls, n_qubits: int, mapping: str, h0: float, h, g):
        """Qubit Hamiltonian of Eq. 2 under mapping "jw" or "bk"."""
        h = np.ascontiguousarray(h, dtype=np.float64)
        g = np.ascontiguousarray(g, dtype=np.float64)
        out = C.c_void_p()
        _check(lib().vqe_hamiltonian_from_integrals_map(int(n_qubits), _MAPS[mapping], float(h0),
                                                        _dptr(h), _dptr(g), C.byref(out)))
        return cls(out)

    @classmethod
    def pairs_from_integrals(cls, n_orbitals: int, h0: float, h, g):
        """Hard-core-boson (pUCCD) Hamiltonian on n_orbitals qubits."""
        h = np.ascontiguousarray(h, dtype=np.float64)
        g = np.ascontiguousarray(g, dtype=np.float64)
        out = C.c_void_p()
        _check(lib().vqe_hamiltonian_pairs_from_integrals(int(n_orbitals), float(h0), _dptr(h),
                                                          _dptr(g), C.byref(out)))
        return cls(out)

    @classmethod
    def from_paulis(cls, n_qubits: int, x, z, coef):
        x = np.ascontiguousarray(x, dtype=np.uint32)
        z = np.ascontiguousarray(z, dtype=np.uint32)
        coef = np.ascontiguousarray(coef, dtype=np.float64)
        out = C.c_void_p()
        _check(lib().vqe_hamiltonian_from_paulis(int(n_qubits), x.size, _u32(x), _u32(z),
                                                 _dptr(coef), C.byref(out)))
        return cls(out)

    def info(self):
        n, t, g = C.c_int(), C.c_int64(), C.c_int64()
        _check(lib().vqe_hamiltonian_info(self._h, C.byref(n), C.byref(t), C.byref(g)))
        return n.value, t.value, g.value

    def terms(self):
        _, t, _ = self.info()
        x = np.empty(t, np.uint32)
        z = np.empty(t, np.uint32)
        c = np.empty(t, np.float64)
        cnt = C.c_int64(t)
        _check(lib().vqe_hamiltonian_terms(self._h, C.byref(cnt), _u32(x), _u32(z), _dptr(c)))
        return x, z, c

    def close(self):
        if self._h:
            lib().vqe_hamiltonian_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Ansatz:
    def __init__(self, handle):
        self._h = handle

    @classmethod
    def uccsd(cls, n_qubits: int, n_electrons: int):
        out = C.c_void_p()
        m = C.c_int32()
        _check(lib().vqe_ansatz_uccsd(int(n_qubits), int(n_electrons), C.byref(out), C.byref(m)))
        return cls(out)

    @classmethod
    def uccsd_map(cls, n_qubits: int, n_electrons: int, mapping: str):
        """UCCSD under mapping "jw" (excitation gates) or "bk" (Pauli rotations)."""
        out = C.c_void_p()
        m = C.c_int32()
        _check(lib().vqe_ansatz_uccsd_map(int(n_qubits), int(n_electrons), _MAPS[mapping],
                                          C.byref(out), C.byref(m)))
        return cls(out)

    def reference(self) -> int:
        v = C.c_uint64()
        _check(lib().vqe_ansatz_reference(self._h, C.byref(v)))
        return v.value

    @classmethod
    def uccsd_trotter(cls, n_qubits: int, n_electrons: int, steps: int):
        """UCCSD with `steps` Trotter steps (angles theta / steps, shared)."""
        out = C.c_void_p()
        m = C.c_int32()
        _check(lib().vqe_ansatz_uccsd_trotter(int(n_qubits), int(n_electrons), int(steps),
                                              C.byref(out), C.byref(m)))
        return cls(out)

    @classmethod
    def kupccgsd(cls, n_qubits: int, n_electrons: int, k: int):
        """k-UpCCGSD: k layers of generalised singles and pair doubles."""
        out = C.c_void_p()
        m = C.c_int32()
        _check(lib().vqe_ansatz_kupccgsd(int(n_qubits), int(n_electrons), int(k), C.byref(out),
                                         C.byref(m)))
        return cls(out)

    @classmethod
    def puccd(cls, n_orbitals: int, n_pairs: int):
        """pUCCD on the pair space (evaluate with n_electrons = n_pairs)."""
        out = C.c_void_p()
        m = C.c_int32()
        _check(lib().vqe_ansatz_puccd(int(n_orbitals), int(n_pairs), C.byref(out), C.byref(m)))
        return cls(out)

    @classmethod
    def from_rotations(cls, n_qubits: int, n_params: int, x, z, param_index, scale):
        x = np.ascontiguousarray(x, dtype=np.uint32)
        z = np.ascontiguousarray(z, dtype=np.uint32)
        pi = np.ascontiguousarray(param_index, dtype=np.int32)
        sc = np.ascontiguousarray(scale, dtype=np.float64)
        out = C.c_void_p()
        _check(lib().vqe_ansatz_from_rotations(int(n_qubits), int(n_params), x.size, _u32(x), _u32(z),
                                               pi.ctypes.data_as(C.POINTER(C.c_int32)), _dptr(sc),
                                               C.byref(out)))
        return cls(out)

    def select(self, param_index):
        """Sub-ansatz of this pool: the gates of pool parameter param_index[0],
        then param_index[1], ... (one new parameter each)."""
        idx = np.ascontiguousarray(param_index, dtype=np.int32)
        out = C.c_void_p()
        _check(lib().vqe_ansatz_select(self._h, idx.size, idx.ctypes.data_as(C.POINTER(C.c_int32)),
                                       C.byref(out)))
        return Ansatz(out)

    def info(self):
        n, p, g, e = C.c_int(), C.c_int32(), C.c_int64(), C.c_int()
        _check(lib().vqe_ansatz_info(self._h, C.byref(n), C.byref(p), C.byref(g), C.byref(e)))
        return n.value, p.value, g.value, e.value

    @property
    def n_params(self) -> int:
        return self.info()[1]

    def excitations(self):
        _, _, g, _ = self.info()
        buf = np.empty(4 * g, np.int32)
        cnt = C.c_int64(g)
        _check(lib().vqe_ansatz_excitations(self._h, C.byref(cnt),
                                            buf.ctypes.data_as(C.POINTER(C.c_int32))))
        return [tuple(int(v) for v in buf[4 * k:4 * k + 4] if v >= 0) for k in range(cnt.value)]

    def close(self):
        if self._h:
            lib().vqe_ansatz_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class State:
    """Device statevector (complex128[2^n]); library-owned or borrowed from a
    torch tensor (which must stay alive as long as the State)."""

    def __init__(self, handle, n, keep=None):
        self._h = handle
        self.n = n
        self._keep = keep

    @classmethod
    def create(cls, n_qubits: int, stream=None):
        out = C.c_void_p()
        _check(lib().vqe_state_create(int(n_qubits), stream if stream is not None else current_stream(),
                                      C.byref(out)))
        return cls(out, n_qubits)

    @classmethod
    def wrap(cls, tensor, stream=None):
        import torch
        if tensor.dtype != torch.complex128 or not tensor.is_cuda or not tensor.is_contiguous():
            raise ValueError("need a contiguous complex128 device tensor")
        n = int(tensor.numel()).bit_length() - 1
        if (1 << n) != tensor.numel():
            raise ValueError("length must be a power of two")
        out = C.c_void_p()
        _check(lib().vqe_state_wrap(n, C.c_void_p(tensor.data_ptr()),
                                    stream if stream is not None else current_stream(), C.byref(out)))
        return cls(out, n, keep=tensor)

    def data_ptr(self) -> int:
        p = C.c_void_p()
        _check(lib().vqe_state_data(self._h, C.byref(p)))
        return p.value

    def prepare_hf(self, n_electrons: int):
        _check(lib().vqe_prepare_hf(self._h, int(n_electrons)))

    def prepare_basis(self, index: int):
        _check(lib().vqe_prepare_basis(self._h, C.c_uint64(int(index))))

    def apply_pauli_rotation(self, x: int, z: int, theta: float):
        _check(lib().vqe_apply_pauli_rotation(self._h, int(x), int(z), float(theta)))

    def apply_ansatz(self, ansatz: Ansatz, theta):
        theta = np.ascontiguousarray(theta, dtype=np.float64)
        _check(lib().vqe_apply_ansatz(self._h, ansatz._h, _dptr(theta)))

    def expectation(self, ham: Hamiltonian) -> float:
        e = C.c_double()
        _check(lib().vqe_expectation(self._h, ham._h, C.byref(e)))
        return e.value

    def close(self):
        if self._h:
            lib().vqe_state_free(self._h)
            self._h = None
        self._keep = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def energy_grad(ham: Hamiltonian, ansatz: Ansatz, n_electrons: int, theta, grad: bool = True,
                stream=None):
    """(E, dE/dtheta or None) at theta (float64, n_params)."""
    theta = np.ascontiguousarray(theta, dtype=np.float64)
    e = C.c_double()
    g = np.empty(max(theta.size, 1), np.float64) if grad else None
    _check(lib().vqe_energy_grad(ham._h, ansatz._h, int(n_electrons), _dptr(theta), C.byref(e),
                                 _dptr(g) if grad else None,
                                 stream if stream is not None else current_stream()))
    return e.value, (g[:theta.size] if grad else None)


def energy_grad_noalloc(ham: Hamiltonian, ansatz: Ansatz, n_electrons: int, theta, grad: bool = True,
                        stream=None):
    """energy_grad through the library's allocation-free entry point (its
    workspace is a static device array; energy_grad must have run once with
    the same ham, ansatz and n_electrons on this device)."""
    theta = np.ascontiguousarray(theta, dtype=np.float64)
    e = C.c_double()
    g = np.empty(max(theta.size, 1), np.float64) if grad else None
    _check(lib().vqe_energy_grad_noalloc(ham._h, ansatz._h, int(n_electrons), _dptr(theta), C.byref(e),
                                         _dptr(g) if grad else None,
                                         stream if stream is not None else current_stream()))
    return e.value, (g[:theta.size] if grad else None)


def pool_gradient(ham: Hamiltonian, ansatz: Ansatz, pool: Ansatz, n_electrons: int, theta,
                  stream=None):
    """(E at theta, d E / d t of each pool operator appended at angle t = 0)."""
    theta = np.ascontiguousarray(theta, dtype=np.float64)
    e = C.c_double()
    g = np.empty(pool.n_params, np.float64)
    _check(lib().vqe_pool_gradient(ham._h, ansatz._h, pool._h, int(n_electrons), _dptr(theta),
                                   C.byref(e), _dptr(g),
                                   stream if stream is not None else current_stream()))
    return e.value, g


def pool_gradient_profile(ham: Hamiltonian, ansatz: Ansatz, pool: Ansatz, n_electrons: int, theta,
                          reps: int = 3, stream=None):
    """(ms, work) of the pool gradient: per-phase milliseconds (forward,
    H-apply, pool sweep, reductions) and (forward bytes, 0, pool-sweep bytes,
    pool-sweep launches)."""
    theta = np.ascontiguousarray(theta, dtype=np.float64)
    ms = np.empty(4, np.float64)
    w = np.empty(4, np.float64)
    _check(lib().vqe_pool_gradient_profile(ham._h, ansatz._h, pool._h, int(n_electrons),
                                           _dptr(theta), int(reps), _dptr(ms), _dptr(w),
                                           stream if stream is not None else current_stream()))
    return ms, w


def _energy_grad_fn():
    import torch

    class EnergyGrad(torch.autograd.Function):
        """E(theta) with the adjoint gradient; theta is a float64 tensor (any
        device; it is read on the host).  backward returns gE * dE/dtheta."""

        @staticmethod
        def forward(ctx, theta, ham, ansatz, n_electrons):
            th = theta.detach().to("cpu", torch.float64).contiguous().numpy()
            e, g = energy_grad(ham, ansatz, n_electrons, th, grad=True)
            ctx.save_for_backward(torch.from_numpy(g).to(theta.device))
            return torch.tensor(e, dtype=torch.float64, device=theta.device)

        @staticmethod
        def backward(ctx, ge):
            (g,) = ctx.saved_tensors
            return ge * g, None, None, None

    return EnergyGrad


class _Lazy:
    _cls = None

    def __getattr__(self, item):
        if _Lazy._cls is None:
            _Lazy._cls = _energy_grad_fn()
        return getattr(_Lazy._cls, item)


EnergyGrad = _Lazy()


class Batch:
    """Many independent (H, ansatz, n_e) problems evaluated by one HIP-graph
    launch.  The Hamiltonians and ansatzes must outlive the batch."""

    def __init__(self, hams, ansatzes, n_electrons, stream=None):
        S = len(hams)
        self._refs = (list(hams), list(ansatzes))
        Hs = (C.c_void_p * S)(*[h._h.value for h in hams])
        As = (C.c_void_p * S)(*[a._h.value for a in ansatzes])
        ne = (C.c_int * S)(*[int(v) for v in n_electrons])
        out = C.c_void_p()
        _check(lib().vqe_batch_create(S, Hs, As, ne, stream if stream is not None else current_stream(),
                                      C.byref(out)))
        self._h = out
        self.S = S
        offs = np.empty(S + 1, np.int64)
        _check(lib().vqe_batch_offsets(self._h, offs.ctypes.data_as(C.POINTER(C.c_int64))))
        self.offsets = offs

    def energy_grad(self, theta_all, grad: bool = True):
        theta_all = np.ascontiguousarray(theta_all, dtype=np.float64)
        if theta_all.size != self.offsets[-1]:
            raise ValueError("theta_all has the wrong length")
        e = np.empty(self.S, np.float64)
        g = np.empty(max(theta_all.size, 1), np.float64) if grad else None
        _check(lib().vqe_batch_energy_grad(self._h, _dptr(theta_all), _dptr(e),
                                           _dptr(g) if grad else None))
        return e, (g[:theta_all.size] if grad else None)

    def energy_grad_device(self, theta_all, e_all, g_all=None):
        """The evaluation on device buffers (float64 tensors on the batch's
        device: theta_all [total params], e_all [S], g_all [total params] or
        None), ordered on the stream the batch was created with; nothing is
        copied to the host and nothing is checked there."""
        import torch
        P = int(self.offsets[-1])
        for name, t, size in (("theta_all", theta_all, P), ("e_all", e_all, self.S),
                              ("g_all", g_all, P)):
            if t is None:
                if name != "g_all":
                    raise ValueError(f"{name} is required")
                continue
            if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous() and t.numel() == size):
                raise ValueError(f"{name} must be a contiguous float64 device tensor of {size} entries")
        _check(lib().vqe_batch_energy_grad_device(self._h, C.c_void_p(theta_all.data_ptr()),
                                                  C.c_void_p(e_all.data_ptr()),
                                                  C.c_void_p(g_all.data_ptr()) if g_all is not None else None))

    def profile(self, theta_all, reps: int = 3):
        """Per-phase milliseconds of one evaluation (forward, H-apply, adjoint,
        reductions), timed with HIP events on the batch stream."""
        theta_all = np.ascontiguousarray(theta_all, dtype=np.float64)
        ms = np.empty(4, np.float64)
        _check(lib().vqe_batch_profile(self._h, _dptr(theta_all), int(reps), _dptr(ms)))
        return ms

    def work(self):
        """Work of one evaluation: (forward bytes, packed pair updates per pass,
        adjoint bytes, all phi + lambda bytes, forward launches, H-apply
        launches, adjoint launches, states with real amplitudes)."""
        w = np.empty(8, np.float64)
        _check(lib().vqe_batch_work(self._h, _dptr(w)))
        return w

    def persistent(self):
        """Persistent-pass layout: dict(on, queues, grid_fwd, grid_adj,
        items_fwd, pmax, lds_fwd, lds_adj); on = 0 when the batch uses one
        launch per run and size class."""
        info = (C.c_int * 8)()
        _check(lib().vqe_batch_persistent(self._h, info))
        keys = ("on", "queues", "grid_fwd", "grid_adj", "items_fwd", "pmax", "lds_fwd", "lds_adj")
        return dict(zip(keys, list(info)))

    def test_wait(self, spin_limit: int = 0, poison: bool = False):
        """Test hook of the persistent passes' bounded waits (see vqe.h)."""
        _check(lib().vqe_batch_test_wait(self._h, int(spin_limit), int(bool(poison))))

    def close(self):
        if self._h:
            lib().vqe_batch_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _options(max_iter=200, gtol=1e-8, ftol=0.0, max_seconds=0.0, record_trace=True):
    return Options(int(max_iter), float(gtol), float(ftol), float(max_seconds), int(bool(record_trace)))


def minimize_bfgs(fun, x0, **opts):
    """BFGS of the library on a Python objective fun(x) -> (f, g).
    Returns (x, Result, trace)."""
    x0 = np.ascontiguousarray(x0, dtype=np.float64)
    n = x0.size
    o = _options(**opts)
    err = []

    def cb(ctx, nn, xp, fp, gp):
        try:
            x = np.ctypeslib.as_array(xp, shape=(nn,)).copy()
            f, g = fun(x)
            fp[0] = float(f)
            np.ctypeslib.as_array(gp, shape=(nn,))[:] = g
            return 0
        except Exception as exc:  # reported as an aborted minimisation
            err.append(exc)
            return 1

    cfun = _lib.OBJECTIVE(cb)
    x = np.empty(n, np.float64)
    trace = np.empty(o.max_iter + 1, np.float64)
    res = Result()
    rc = lib().vqe_minimize_bfgs(n, cfun, None, _dptr(x0), C.byref(o), _dptr(x), _dptr(trace),
                                 C.byref(res))
    if err:
        raise err[0]
    _check(rc)
    return x, res, trace


def run_vqe(ham: Hamiltonian, ansatz: Ansatz, n_electrons: int, theta0=None, stream=None, **opts):
    """VQE by BFGS over the library's energy + adjoint gradient.
    Returns (theta, Result, trace)."""
    m = ansatz.n_params
    o = _options(**opts)
    th0 = None if theta0 is None else np.ascontiguousarray(theta0, dtype=np.float64)
    x = np.empty(m, np.float64)
    trace = np.empty(o.max_iter + 1, np.float64)
    res = Result()
    _check(lib().vqe_run(ham._h, ansatz._h, int(n_electrons), _dptr(th0) if th0 is not None else None,
                         C.byref(o), _dptr(x), _dptr(trace), C.byref(res),
                         stream if stream is not None else current_stream()))
    return x, res, trace


def run_adapt(ham: Hamiltonian, pool: Ansatz, n_electrons: int, grad_tol=1e-3, tie_tol=1e-10,
              max_operators=None, stream=None, **opts):
    """ADAPT-VQE from the identity ansatz over `pool`.  Returns (selected pool
    indices, angles, energies, gradient norms, AdaptResult); the last two have
    one entry per ansatz size 0 .. len(selected)."""
    cap = pool.n_params if max_operators is None else int(max_operators)
    o = _lib.AdaptOptions(float(grad_tol), float(tie_tol), cap, _options(**opts))
    sel = np.empty(max(cap, 1), np.int32)
    th = np.empty(max(cap, 1), np.float64)
    es = np.empty(cap + 1, np.float64)
    ns = np.empty(cap + 1, np.float64)
    res = _lib.AdaptResult()
    _check(lib().vqe_adapt(ham._h, pool._h, int(n_electrons), C.byref(o),
                           sel.ctypes.data_as(C.POINTER(C.c_int32)), _dptr(th), _dptr(es),
                           _dptr(ns), C.byref(res),
                           stream if stream is not None else current_stream()))
    k = res.n_operators
    return sel[:k].tolist(), th[:k].copy(), es[:k + 1].copy(), ns[:k + 1].copy(), res
