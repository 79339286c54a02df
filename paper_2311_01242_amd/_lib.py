"""ctypes declarations of the C ABI in include/vqe.h (argument marshalling only)."""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libvqe.so")

c_int, c_int32, c_int64, c_uint32, c_double = C.c_int, C.c_int32, C.c_int64, C.c_uint32, C.c_double
vp = C.c_void_p
P = C.POINTER


class Options(C.Structure):
    _fields_ = [("max_iter", c_int), ("gtol", c_double), ("ftol", c_double),
                ("max_seconds", c_double), ("record_trace", c_int)]


class Result(C.Structure):
    _fields_ = [("energy", c_double), ("iters", c_int), ("n_evals", c_int), ("converged", c_int)]


class AdaptOptions(C.Structure):
    _fields_ = [("grad_tol", c_double), ("tie_tol", c_double), ("max_operators", c_int),
                ("vqe", Options)]


class AdaptResult(C.Structure):
    _fields_ = [("energy", c_double), ("grad_norm", c_double), ("n_operators", c_int),
                ("converged", c_int), ("n_evals", c_int), ("vqe_iters", c_int)]


OBJECTIVE = C.CFUNCTYPE(c_int, vp, c_int, P(c_double), P(c_double), P(c_double))

# name -> (restype, argtypes); the order follows include/vqe.h
SIGNATURES = {
    "vqe_abi_version": (c_int, []),
    "vqe_last_error": (C.c_char_p, []),
    "vqe_hamiltonian_from_integrals": (c_int, [c_int, c_double, P(c_double), P(c_double), P(vp)]),
    "vqe_hamiltonian_from_paulis": (c_int, [c_int, c_int64, P(c_uint32), P(c_uint32), P(c_double), P(vp)]),
    "vqe_hamiltonian_from_integrals_map": (c_int, [c_int, c_int, c_double, P(c_double),
                                                   P(c_double), P(vp)]),
    "vqe_hamiltonian_pairs_from_integrals": (c_int, [c_int, c_double, P(c_double), P(c_double),
                                                     P(vp)]),
    "vqe_hamiltonian_info": (c_int, [vp, P(c_int), P(c_int64), P(c_int64)]),
    "vqe_hamiltonian_terms": (c_int, [vp, P(c_int64), P(c_uint32), P(c_uint32), P(c_double)]),
    "vqe_hamiltonian_free": (None, [vp]),
    "vqe_ansatz_uccsd": (c_int, [c_int, c_int, P(vp), P(c_int32)]),
    "vqe_ansatz_uccsd_map": (c_int, [c_int, c_int, c_int, P(vp), P(c_int32)]),
    "vqe_ansatz_reference": (c_int, [vp, P(C.c_uint64)]),
    "vqe_ansatz_uccsd_trotter": (c_int, [c_int, c_int, c_int, P(vp), P(c_int32)]),
    "vqe_ansatz_kupccgsd": (c_int, [c_int, c_int, c_int, P(vp), P(c_int32)]),
    "vqe_ansatz_puccd": (c_int, [c_int, c_int, P(vp), P(c_int32)]),
    "vqe_ansatz_from_rotations": (c_int, [c_int, c_int32, c_int64, P(c_uint32), P(c_uint32),
                                          P(c_int32), P(c_double), P(vp)]),
    "vqe_ansatz_select": (c_int, [vp, c_int64, P(c_int32), P(vp)]),
    "vqe_ansatz_info": (c_int, [vp, P(c_int), P(c_int32), P(c_int64), P(c_int)]),
    "vqe_ansatz_excitations": (c_int, [vp, P(c_int64), P(c_int32)]),
    "vqe_ansatz_free": (None, [vp]),
    "vqe_state_create": (c_int, [c_int, vp, P(vp)]),
    "vqe_state_wrap": (c_int, [c_int, vp, vp, P(vp)]),
    "vqe_state_data": (c_int, [vp, P(vp)]),
    "vqe_state_free": (None, [vp]),
    "vqe_prepare_hf": (c_int, [vp, c_int]),
    "vqe_prepare_basis": (c_int, [vp, C.c_uint64]),
    "vqe_apply_pauli_rotation": (c_int, [vp, c_uint32, c_uint32, c_double]),
    "vqe_apply_ansatz": (c_int, [vp, vp, P(c_double)]),
    "vqe_expectation": (c_int, [vp, vp, P(c_double)]),
    "vqe_energy_grad": (c_int, [vp, vp, c_int, P(c_double), P(c_double), P(c_double), vp]),
    "vqe_energy_grad_noalloc": (c_int, [vp, vp, c_int, P(c_double), P(c_double), P(c_double), vp]),
    "vqe_pool_gradient": (c_int, [vp, vp, vp, c_int, P(c_double), P(c_double), P(c_double), vp]),
    "vqe_pool_gradient_profile": (c_int, [vp, vp, vp, c_int, P(c_double), c_int, P(c_double),
                                          P(c_double), vp]),
    "vqe_batch_create": (c_int, [c_int, P(vp), P(vp), P(c_int), vp, P(vp)]),
    "vqe_batch_offsets": (c_int, [vp, P(c_int64)]),
    "vqe_batch_energy_grad": (c_int, [vp, P(c_double), P(c_double), P(c_double)]),
    "vqe_batch_energy_grad_device": (c_int, [vp, vp, vp, vp]),
    "vqe_batch_free": (None, [vp]),
    "vqe_batch_profile": (c_int, [vp, P(c_double), c_int, P(c_double)]),
    "vqe_batch_work": (c_int, [vp, P(c_double)]),
    "vqe_set_tuning": (c_int, [c_int, c_int, c_int64, c_int64, c_int]),
    "vqe_set_packed": (c_int, [c_int]),
    "vqe_set_real": (c_int, [c_int]),
    "vqe_set_tile_cap": (c_int, [c_int, c_int, c_int]),
    "vqe_set_persistent": (c_int, [c_int, c_int]),
    "vqe_batch_persistent": (c_int, [vp, P(c_int)]),
    "vqe_batch_test_wait": (c_int, [vp, c_int, c_int]),
    "vqe_copy_ceiling": (c_int, [vp, vp, c_int64, c_int, vp, P(c_double)]),
    "vqe_lds_ceiling": (c_int, [c_int, vp, P(c_double), P(c_double)]),
    "vqe_set_run_threads": (c_int, [c_int, c_int, c_int, c_int]),
    "vqe_mlp_create": (c_int, [c_int, P(c_int32), vp, P(vp)]),
    "vqe_mlp_n_params": (c_int, [vp, P(c_int64)]),
    "vqe_mlp_set_params": (c_int, [vp, P(C.c_float)]),
    "vqe_mlp_get_params": (c_int, [vp, P(C.c_float)]),
    "vqe_mlp_forward": (c_int, [vp, c_int, P(C.c_float), P(C.c_float)]),
    "vqe_mlp_loss_grad": (c_int, [vp, c_int, P(C.c_float), P(C.c_float), P(C.c_float), P(C.c_float)]),
    "vqe_mlp_train": (c_int, [vp, c_int, P(C.c_float), P(C.c_float), c_int, C.c_float, C.c_float,
                              C.c_float, C.c_float, P(C.c_float)]),
    "vqe_mlp_free": (None, [vp]),
    "vqe_minimize_bfgs": (c_int, [c_int, OBJECTIVE, vp, P(c_double), P(Options), P(c_double),
                                  P(c_double), P(Result)]),
    "vqe_run": (c_int, [vp, vp, c_int, P(c_double), P(Options), P(c_double), P(c_double),
                        P(Result), vp]),
    "vqe_adapt": (c_int, [vp, vp, c_int, P(AdaptOptions), P(c_int32), P(c_double), P(c_double),
                          P(c_double), P(AdaptResult), vp]),
}

_lib = None


def lib():
    """Load libvqe.so (built in-tree).  Fails loudly if it is missing: there
    is no fallback path."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                               "or python -m paper_2311_01242_amd.build")
        lib_ = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(lib_, name)
            f.restype = res
            f.argtypes = args
        _lib = lib_
    return _lib
