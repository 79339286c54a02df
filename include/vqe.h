/*
 * vqe.h — C ABI of the MI355X (gfx950) VQE statevector library.
 *
 * The library computes the VQE objective of Sec. 2.1.1, Eq. 1,
 *     E(theta) = <HF| U(theta)^dag H U(theta) |HF>,
 * for a Jordan-Wigner qubit Hamiltonian H = sum_k c_k P_k (the qubit form of
 * Eq. 2, Sec. 2.1.1) and a UCCSD ansatz U = exp(T - T^dag) (Sec. 2.1.2),
 * together with its exact gradient (adjoint reverse sweep) and a BFGS-driven
 * VQE loop (Sec. 3.1 "Results for parameter optimisation" names BFGS).
 *
 * Conventions
 * -----------
 * - Qubit q is spin orbital q: spatial orbital q/2, spin q%2 (0 = alpha,
 *   1 = beta).  Odd qubit counts leave the last spatial orbital alpha-only.
 *   Bit q of a statevector index is the occupation of spin orbital q.
 * - A statevector is complex128[2^n], interleaved (re, im), in device memory,
 *   256-byte aligned.
 * - Pauli masks are uint32: bit q of x is an X or Y on qubit q, bit q of z a
 *   Z or Y.  Two different forms are used, and each call says which:
 *     * Hermitian string P(x, z): Y where x and z are both set,
 *       P = i^{popcount(x&z)} X^x Z^z;
 *     * folded form X^x Z^z (Z applied first) with a REAL coefficient
 *       c' = c * i^{popcount(x&z)}; X^x Z^z |b> = (-1)^{popcount(b&z)} |b^x>.
 *   Hamiltonians are exchanged in folded form (real coefficients); rotations
 *   exp(-i phi/2 P) take Hermitian strings.
 * - Every call returns an int status: VQE_OK (0) or a negative error code;
 *   vqe_last_error() returns a thread-local message for the last failure.
 *   The library never aborts or exits.  Arguments are validated on the host
 *   before any HIP call, so argument errors are reported without a GPU.
 * - The caller owns every host array passed in; the library copies what it
 *   keeps.  Handles are not safe for concurrent use from several threads.
 * - hip_stream arguments are hipStream_t values (NULL = the null stream);
 *   work is ordered on that stream.  Calls that return host results
 *   synchronise that stream before returning.
 */
#ifndef VQE_H
#define VQE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define VQE_ABI_VERSION 1

enum {
    VQE_OK = 0,
    VQE_EINVAL = -1,   /* bad argument: null pointer, NaN, asymmetric integrals, ... */
    VQE_ERANGE = -2,   /* size out of range: n_qubits, n_electrons, indices */
    VQE_ENOMEM = -3,   /* host or device allocation failed / would not fit */
    VQE_EDEVICE = -4,  /* HIP runtime error (message carries hipGetErrorString) */
    VQE_ENUMERIC = -5  /* non-finite energy or gradient produced */
};

typedef struct vqe_hamiltonian vqe_hamiltonian;
typedef struct vqe_ansatz vqe_ansatz;
typedef struct vqe_state vqe_state;
typedef struct vqe_batch vqe_batch;

int vqe_abi_version(void);
const char* vqe_last_error(void);

/* ---------------------------------------------------------------------------
 * Hamiltonians (host-only construction; uploaded to a device on first use)
 * ------------------------------------------------------------------------ */

/* Jordan-Wigner qubit Hamiltonian of Eq. 2 (Sec. 2.1.1) from real spatial
 * integrals, read as
 *   H = h0 + sum_{pq,s} h[p][q] a+_{ps} a_{qs}
 *          + 1/2 sum_{pqrs,s,t} (pq|rs) a+_{ps} a+_{rt} a_{st} a_{qs},
 * with ns = ceil(n_qubits/2) spatial orbitals; h is row-major [ns][ns] and
 * g row-major [ns][ns][ns][ns] holding chemist integrals (pq|rs).
 * Requires 1 <= n_qubits <= 32 (ERANGE), h symmetric and g 8-fold symmetric
 * within 1e-12 and every value finite (EINVAL).  Terms with |c'| <= 1e-12
 * after accumulation are dropped.  *out is freed with vqe_hamiltonian_free. */
int vqe_hamiltonian_from_integrals(int n_qubits, double h0, const double* h,
                                   const double* g, vqe_hamiltonian** out);

/* Fermion-to-qubit mappings (Sec. 2.1.1 names Jordan-Wigner and
 * Bravyi-Kitaev).  Both are linear encodings b = beta n (mod 2) of the
 * occupation vector n: JW beta = 1; BK qubit j holds the parity of orbitals
 * j + 1 - lowbit(j + 1) .. j (Fenwick-tree rows). */
#define VQE_MAP_JW 0
#define VQE_MAP_BK 1

/* vqe_hamiltonian_from_integrals under `mapping` (VQE_MAP_JW gives the same
 * terms as vqe_hamiltonian_from_integrals).  With beta as above,
 * a_P = X^{c_P} Z^{s_P} (1 - Z^{r_P})/2 and a+_P = X^{c_P} Z^{s_P} (1 + Z^{r_P})/2
 * (c_P column P of beta, r_P row P of beta^{-1}, s_P the XOR of rows P' < P
 * of beta^{-1}).  ERANGE for an unknown mapping. */
int vqe_hamiltonian_from_integrals_map(int n_qubits, int mapping, double h0, const double* h,
                                       const double* g, vqe_hamiltonian** out);

/* Eq. 2 projected onto the seniority-zero space, in the hard-core-boson
 * form used by pUCCD (Sec. 2.1, ansatz list): qubit p is spatial orbital p
 * (n_orbitals qubits, half the Jordan-Wigner count), bit p = 1 when both
 * of its spin orbitals are occupied.  With N_p the pair number and b_p the
 * pair annihilator,
 *   H = h0 + sum_p (2 h_pp + (pp|pp)) N_p
 *          + sum_{p<q} 2 [2 (pp|qq) - (pq|qp)] N_p N_q
 *          + sum_{p<q} (pq|pq) (b_p^dag b_q + b_q^dag b_p),
 * N_p = (1 - Z_p)/2, b_p^dag b_q + h.c. = (X_p X_q + Y_p Y_q)/2.  h is
 * [n][n] and g [n][n][n][n] chemist integrals, with the same checks as
 * vqe_hamiltonian_from_integrals.  |c'| <= 1e-12 terms are dropped. */
int vqe_hamiltonian_pairs_from_integrals(int n_orbitals, double h0, const double* h,
                                         const double* g, vqe_hamiltonian** out);

/* Hamiltonian sum_k coef[k] X^{x[k]} Z^{z[k]} in folded form (see above).
 * Masks must fit n_qubits bits (ERANGE); duplicate (x, z) pairs are summed;
 * a nonzero term with odd popcount(x&z) makes H non-symmetric and is
 * rejected (EINVAL); coefficients must be finite (EINVAL). */
int vqe_hamiltonian_from_paulis(int n_qubits, int64_t n_terms, const uint32_t* x,
                                const uint32_t* z, const double* coef,
                                vqe_hamiltonian** out);

/* Sizes: qubits, terms, x-mask groups (any pointer may be NULL). */
int vqe_hamiltonian_info(const vqe_hamiltonian* H, int* n_qubits, int64_t* n_terms,
                         int64_t* n_groups);

/* Export the terms in folded form, sorted by (x, z).  *n_terms is the
 * capacity of x/z/coef on input and the term count on output; with a
 * capacity smaller than the count nothing is written and ERANGE returned. */
int vqe_hamiltonian_terms(const vqe_hamiltonian* H, int64_t* n_terms, uint32_t* x,
                          uint32_t* z, double* coef);

void vqe_hamiltonian_free(vqe_hamiltonian* H);

/* ---------------------------------------------------------------------------
 * Ansatz programs (host-only construction)
 * ------------------------------------------------------------------------ */

/* UCCSD (Sec. 2.1.2), one Trotter step, on the HF reference of n_electrons:
 * singles T = a+_a a_i, doubles T = a+_a a+_b a_j a_i (i < j occupied, a < b
 * virtual, spin-conserving), U_j = exp(theta_j (T_j - T_j^dag)), applied as
 * U_M ... U_1 with all singles first (a outer, i inner) and then doubles
 * ((a, b) outer, (i, j) inner), ascending.  *n_params receives M. */
int vqe_ansatz_uccsd(int n_qubits, int n_electrons, vqe_ansatz** out, int32_t* n_params);

/* UCCSD under `mapping`: VQE_MAP_JW is vqe_ansatz_uccsd; otherwise each
 * generator T - T^dag is written with the encoded ladder operators as
 * sum_k i d_k P_k (commuting Hermitian strings) and applied as the Pauli
 * rotations exp(-i (-2 d_k theta) / 2 P_k), on full 2^n vectors, from the
 * encoded reference beta (2^n_electrons - 1) (vqe_ansatz_reference).
 * Excitations are reported as for vqe_ansatz_uccsd.  Energy and gradient
 * evaluations (vqe_energy_grad, its allocation-free form, vqe_batch_*,
 * vqe_run) with the packed layout on (vqe_set_packed, default) evaluate
 * the program in the occupation basis instead: the encoded program and
 * Hamiltonian are the occupation-basis ones conjugated by the basis
 * relabelling b = beta n, so the same energy and gradient come from the
 * decoded reference, the occupation-basis excitations and the Hamiltonian's
 * terms taken to that basis (X^x Z^z -> X^{beta^-1 x} Z^{beta^T z}, made once
 * per Hamiltonian and encoding), on the packed sector path.  With the
 * packed layout off the rotations run on full vectors as given. */
int vqe_ansatz_uccsd_map(int n_qubits, int n_electrons, int mapping, vqe_ansatz** out,
                         int32_t* n_params);

/* Basis index of the reference the evaluation calls prepare for this ansatz:
 * 2^n_electrons - 1 unless a mapping moved it.  EINVAL without a reference. */
int vqe_ansatz_reference(const vqe_ansatz* A, uint64_t* index);

/* UCCSD with `steps` Trotter steps (the UCCSD depth of Sec. 2.1's ansatz
 * list): the vqe_ansatz_uccsd product with every angle theta_j / steps,
 * repeated steps times (1 <= steps <= 64; parameters shared).  Excitations
 * are reported once per repetition. */
int vqe_ansatz_uccsd_trotter(int n_qubits, int n_electrons, int steps, vqe_ansatz** out,
                             int32_t* n_params);

/* k-UpCCGSD (Sec. 2.1, ansatz list) on the HF reference: a layer holds every
 * generalised single T = a+_q a_p (p < q, equal spin; q outer, p inner,
 * ascending), reported as (p, q, -1, -1), then every pair double
 * T = a+_{2q} a+_{2q+1} a_{2p+1} a_{2p} (spatial p < q with both spin
 * orbitals; q outer, p inner), reported as (2p, 2p+1, 2q, 2q+1);
 * U_j = exp(theta_j (T_j - T_j^dag)); k layers (1..64) with their own
 * angles.  n_qubits in [2, 32]. */
int vqe_ansatz_kupccgsd(int n_qubits, int n_electrons, int k, vqe_ansatz** out,
                        int32_t* n_params);

/* pUCCD (Sec. 2.1, ansatz list) in the hard-core-boson form on n_orbitals
 * qubits: for occupied pairs i < n_pairs and empty orbitals a >= n_pairs
 * (a outer, i inner, ascending), U = exp(theta (b_a^dag b_i - b_i^dag b_a)),
 * the Givens rotation of D (bit i set, bit a clear) and D ^ (2^i + 2^a)
 * with T|D> = +|D ^ ...>.  The reference is the n_pairs lowest qubits
 * (pass n_electrons = n_pairs to the evaluation calls).  Evaluated on full
 * 2^n vectors.  *n_params receives n_pairs (n_orbitals - n_pairs). */
int vqe_ansatz_puccd(int n_orbitals, int n_pairs, vqe_ansatz** out, int32_t* n_params);

/* Ansatz of explicit Pauli rotations applied in the given order:
 * gate k is exp(-i (scale[k] * theta[param_index[k]]) / 2 * P(x[k], z[k]))
 * with P a Hermitian Pauli string.  0 <= param_index[k] < n_params. */
int vqe_ansatz_from_rotations(int n_qubits, int32_t n_params, int64_t n_rot,
                              const uint32_t* x, const uint32_t* z,
                              const int32_t* param_index, const double* scale,
                              vqe_ansatz** out);

/* Sub-ansatz of a pool (ADAPT-VQE, Sec. 2.1): the gates of pool parameter
 * param_index[0], then those of param_index[1], ..., each keeping the pool's
 * gate order; parameter k of the result drives the gates of param_index[k],
 * so an operator may appear more than once.  count = 0 gives the identity
 * program (the HF state).  Errors: ERANGE for an index outside the pool's
 * parameters or a negative count. */
int vqe_ansatz_select(const vqe_ansatz* pool, int64_t count, const int32_t* param_index,
                      vqe_ansatz** out);

/* Sizes: qubits, parameters, gates, electrons of the reference (-1 if none). */
int vqe_ansatz_info(const vqe_ansatz* A, int* n_qubits, int32_t* n_params,
                    int64_t* n_gates, int* n_electrons);

/* Excitation list of a UCCSD ansatz in application order: orbitals[4*k..]
 * = (i, a, -1, -1) for a single, (i, j, a, b) for a double.  *n is capacity
 * in / count out (ERANGE if too small; EINVAL for a rotation ansatz). */
int vqe_ansatz_excitations(const vqe_ansatz* A, int64_t* n, int32_t* orbitals);

void vqe_ansatz_free(vqe_ansatz* A);

/* ---------------------------------------------------------------------------
 * Device statevectors
 * ------------------------------------------------------------------------ */

/* Library-owned statevector of n_qubits (1..32) on the current HIP device,
 * ordered on hip_stream.  Contents are undefined until prepared. */
int vqe_state_create(int n_qubits, void* hip_stream, vqe_state** out);

/* Borrow caller memory (complex128[2^n], device, 256-byte aligned); the
 * library never frees it.  The memory must outlive the handle. */
int vqe_state_wrap(int n_qubits, void* dev_complex128, void* hip_stream, vqe_state** out);

/* Device pointer of the amplitudes. */
int vqe_state_data(const vqe_state* s, void** dev_ptr);

void vqe_state_free(vqe_state* s);

/* |HF> = the basis state with the lowest n_electrons spin orbitals occupied
 * (index 2^n_e - 1), the reference |0> of Eq. 1. */
int vqe_prepare_hf(vqe_state* s, int n_electrons);

/* |index>, a computational basis state (ERANGE beyond 2^n_qubits). */
int vqe_prepare_basis(vqe_state* s, uint64_t index);

/* psi <- exp(-i theta/2 P(x, z)) psi for a Hermitian Pauli string. */
int vqe_apply_pauli_rotation(vqe_state* s, uint32_t x, uint32_t z, double theta);

/* psi <- U(theta) psi; theta is a host array of the ansatz's n_params. */
int vqe_apply_ansatz(vqe_state* s, const vqe_ansatz* A, const double* theta);

/* *energy = Re <psi|H|psi> (Eq. 1's expectation; psi is not renormalised).
 * Synchronises the state's stream. */
int vqe_expectation(const vqe_state* s, const vqe_hamiltonian* H, double* energy);

/* Energy and exact gradient at theta (host array, n_params):
 * prepares |HF> of n_electrons, applies U(theta), evaluates E, and when grad
 * is non-NULL runs the adjoint reverse sweep for dE/dtheta (n_params
 * doubles).  Scratch memory is cached per (device, stream) and reused.
 * NaN/Inf results return ENUMERIC (outputs still written). */
int vqe_energy_grad(const vqe_hamiltonian* H, const vqe_ansatz* A, int n_electrons,
                    const double* theta, double* energy, double* grad, void* hip_stream);

/* vqe_energy_grad without allocation, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, results and kernels as
 * vqe_energy_grad; calls no hipMalloc, hipFree or allocating library routine.
 * Preconditions: vqe_energy_grad has run once with the same H, A and
 * n_electrons on the current device (it builds the plans this call reuses;
 * else EINVAL).  Workspace: a static device array of 64 MiB per device
 * (held from module load until the process ends) holding phi, lambda, the
 * H-apply's lambda planes, the angles, partials and outputs; evaluations
 * that need more (on the packed layout with real amplitudes, beyond 24
 * qubits; on full 2^n vectors, from 21 qubits on) return ERANGE before any
 * device work.  Every call on a device shares that
 * device's array: calls that overlap on one device (from several host
 * threads or streams) race.  Synchronises hip_stream.  Errors: EINVAL,
 * ERANGE, EDEVICE, ENUMERIC. */
int vqe_energy_grad_noalloc(const vqe_hamiltonian* H, const vqe_ansatz* A, int n_electrons,
                            const double* theta, double* energy, double* grad, void* hip_stream);

/* ADAPT-VQE pool gradient (Sec. 2.1, "ADAPT-VQE algorithm"): with
 * psi = U_A(theta)|HF>, *energy = <psi|H|psi> and, for every parameter k of
 * `pool`, pool_grad[k] = d/dt <psi_t|H|psi_t> at t = 0, where psi_t applies
 * the pool's gates of parameter k at angle t after U_A(theta).  One forward
 * pass, one H-apply and one sweep of the pool at angle zero, where every
 * gate is the identity: psi and H psi are only read, and in the packed
 * layout the whole pool is one launch.  theta: host, A's n_params; pool_grad:
 * host, the pool's n_params.  The pool must act on the same qubits and
 * reference as A; in the packed sector layout it must fit the layout chosen
 * for A (EINVAL otherwise).  NaN/Inf results return ENUMERIC. */
int vqe_pool_gradient(const vqe_hamiltonian* H, const vqe_ansatz* A, const vqe_ansatz* pool,
                      int n_electrons, const double* theta, double* energy, double* pool_grad,
                      void* hip_stream);

/* vqe_pool_gradient timed with HIP events on hip_stream, repeated reps
 * times: ms[0..3] = mean milliseconds of the forward pass, the H-apply, the
 * pool sweep and the reductions; work[0] = forward algorithmic bytes,
 * work[1] = 0, work[2] = pool-sweep algorithmic bytes (packed layout: phi
 * and lambda of every live tile of every run, read once; full layout: read
 * and written by each reverse-sweep launch), work[3] = pool-sweep launches.
 * All host arrays of 4 doubles. */
int vqe_pool_gradient_profile(const vqe_hamiltonian* H, const vqe_ansatz* A,
                              const vqe_ansatz* pool, int n_electrons, const double* theta,
                              int reps, double* ms, double* work, void* hip_stream);

/* ---------------------------------------------------------------------------
 * Batched evaluation of many independent problems
 * ------------------------------------------------------------------------ */

/* A batch of n_states problems (H[i], A[i], n_electrons[i]); qubit counts
 * may differ.  Device buffers for every state are allocated here; the
 * per-evaluation launch sequence is captured once into a HIP graph. */
int vqe_batch_create(int n_states, const vqe_hamiltonian* const* H,
                     const vqe_ansatz* const* A, const int* n_electrons,
                     void* hip_stream, vqe_batch** out);

/* Parameter layout of the batch: offsets[i] is the first entry of state i
 * in theta_all / g_all, offsets[n_states] the total (n_states + 1 ints). */
int vqe_batch_offsets(const vqe_batch* b, int64_t* offsets);

/* Energies e_all[n_states] and gradients g_all[total params] (nullable) for
 * the concatenated host parameters theta_all; one graph launch. */
int vqe_batch_energy_grad(vqe_batch* b, const double* theta_all, double* e_all,
                          double* g_all);

/* The same evaluation with every buffer in device memory of the batch's
 * device: theta_all (total params doubles) is read, e_all[n_states] and
 * g_all[total params] (nullable) are written, with the gradient in the same
 * bits as vqe_batch_energy_grad's.  Asynchronous: ordered after the work
 * already enqueued on the hip_stream given to vqe_batch_create, and that
 * stream waits for the results, so the caller synchronises it (or orders
 * later work on it) before reading them.  No host copy and no host-side
 * check: non-finite values are not reported (the caller tests them), and the
 * call returns EINVAL on a batch with persistent passes, whose wait checks
 * need the host.  The first call with g_all builds the batch's parameter map
 * (device allocation, synchronous); later calls allocate nothing.  The
 * buffers must stay valid until the stream has passed the call. */
int vqe_batch_energy_grad_device(vqe_batch* b, const double* theta_all, double* e_all,
                                 double* g_all);

void vqe_batch_free(vqe_batch* b);

/* Phase timing of one evaluation, measured with HIP events on the batch
 * stream over `reps` eager (not graph) launches of the same kernel sequence:
 * ms[0] forward sweep (angles, |HF>, gate runs), ms[1] H-apply + energy
 * partials, ms[2] adjoint reverse sweep, ms[3] reductions; averages in ms. */
int vqe_batch_profile(vqe_batch* b, const double* theta_all, int reps, double* ms);

/* Algorithmic work of one evaluation of the whole batch, from the launch
 * plan (8 doubles): w[0] forward-sweep bytes (each run tile read and written
 * once, plus the |HF> write), w[1] pair updates of one pass over the gates
 * on the packed layout (live tiles; the reverse sweep makes as many), w[2]
 * reverse-sweep bytes (phi and
 * lambda tiles read and written once), w[3] bytes of all phi + lambda,
 * w[4] gate-step launches of the forward sweep, w[5] H-apply launches,
 * w[6] gate-step launches of the reverse sweep, w[7] states evaluated with
 * real amplitudes (vqe_set_real). */
int vqe_batch_work(const vqe_batch* b, double* w);

/* Launch-parameter override for states of n_qubits (batched = 1 for batch
 * members, 0 for single-state calls): LDS bytes of a forward and a reverse
 * run tile (4 KiB .. 160 KiB) and the low-bit tile of the sector H-apply
 * (2 .. 14).  All three <= 0 restores the built-in choice.  Applies to plans
 * made after the call (batches created later, later single-state calls). */
int vqe_set_tuning(int n_qubits, int batched, int64_t fwd_lds_bytes, int64_t adj_lds_bytes,
                   int hx_tile_bits);

/* Launch-shape override of the packed-layout gate runs for states of
 * n_qubits (batched as in vqe_set_tuning): the least number of threads per
 * run tile (64, 256, 512 or 1024) of the forward and of the reverse pass;
 * a tile too large for that count with the available shapes uses fewer
 * threads with more entries each.  Both <= 0 restores the built-in choice
 * (64 for batch members, 256 for single states).  Applies to plans made after
 * the call.  Errors: ERANGE. */
int vqe_set_run_threads(int n_qubits, int batched, int fwd_threads, int adj_threads);

/* Evaluation layout switch (process-wide, default 2).  With 1 or 2, energy
 * and gradient evaluations of programs made only of number- and
 * spin-conserving excitations (UCCSD, Sec. 2.1.2) run on the packed sector
 * layout: only the amplitudes of the reference's (N, S_z) sector are stored,
 * C(ceil(n/2), N_alpha) C(floor(n/2), N_beta) per vector instead of 2^n, and
 * the hx tile bits are raised to the number of electrons if smaller.  Mode 2
 * also applies H in string-product order (alpha string x beta string) when
 * both spins have at most 13 orbitals and at most 1024 beta strings; mode 1
 * applies it in the packed block order.  With 0 evaluations use full 2^n
 * vectors.  Results agree to rounding; applies to plans made after the call.
 * Errors: ERANGE for other modes. */
int vqe_set_packed(int mode);

/* Real-amplitude switch for the string-product path of mode 2 (process-wide,
 * default on).  Excitation gates are real rotations (Sec. 2.1.2) and the
 * Hamiltonian is a real matrix here (every Pauli term's i^#Y phase is folded
 * into its real coefficient, Eq. 2), so from the real reference phi = U|HF>
 * and lambda = H phi are real: with the switch on, that path stores and
 * moves one double per amplitude instead of two.  Off keeps complex
 * amplitudes.  Results agree to rounding; applies to plans made after the
 * call (a batch's persistent passes always use complex amplitudes).
 * Never fails. */
int vqe_set_real(int on);

/* Tile size of the packed runs for n_qubits (batched or single-state
 * launches; applies to plans made after the call).  A run is a stretch of
 * consecutive gates whose high orbitals (above the block bits) fit a window
 * of at most 4 bits, applied tile by tile, a tile being the blocks that agree
 * outside the window; entries (16..8192) bounds the largest tile, so that
 * fewer block bits with more window bits mean fewer runs (fewer passes over
 * the state) at the same tile size.  0 restores the default: 2400 entries,
 * or two of the layout's largest blocks when they hold more.  Errors: ERANGE. */
int vqe_set_tile_cap(int n_qubits, int batched, int entries);

/* Persistent batch passes (process-wide, applies to batches created after
 * the call).  mode 1: when every state of a batch runs on the
 * packed sector layout and the device's XCDs can be identified (a probe
 * launch reads the XCD id of its workgroups and must find one per 32 CUs),
 * the forward and the reverse gate passes of all states are each ONE launch
 * of one-wave workgroups that take (state, run, tile) items from per-XCD
 * queues, every state's items on one XCD, an item starting once the state's
 * earlier runs are done (bounded waits; a wait that gives up makes
 * vqe_batch_energy_grad return EDEVICE).  All states then use block_bits
 * (0 = 12; range 8..14) block bits.  mode 0 (default): one launch per run
 * and size class.  Results agree to rounding.  Errors: ERANGE. */
int vqe_set_persistent(int mode, int block_bits);

/* Persistent-pass layout of a batch: info[8] receives {on, queues, forward
 * grid, reverse grid, forward items, pair slots per lane, forward LDS bytes,
 * reverse LDS bytes} (zeros when the batch does not use them).  Errors:
 * EINVAL. */
int vqe_batch_persistent(const vqe_batch* b, int* info);

/* Test hook of the persistent passes' bounded waits: spin_limit > 0 sets the
 * polls after which a dependency wait gives up (0: the default, about a
 * second); poison = 1 makes the first forward item that has a dependency wait
 * for a count that is never reached, so that the next evaluation reports
 * EDEVICE after spin_limit polls while every kernel still exits; poison = 0
 * restores it.  Synchronises the batch's stream.  Errors: EINVAL (no
 * persistent passes), ERANGE. */
int vqe_batch_test_wait(vqe_batch* b, int spin_limit, int poison);

/* Measurement helper, not a step of the method: one launch that copies
 * `bytes` (a positive multiple of 16) from device buffer src to device
 * buffer dst (both 16-byte aligned, not overlapping, caller-owned) `passes`
 * times (1..100000), timed with HIP events on hip_stream; *ms receives the
 * launch time.  2 * bytes * passes / time is the measured copy bandwidth
 * the gate kernels' rooflines are reported against (a buffer pair of about
 * 64 MB stays in the last-level cache between passes; a pair of several GB
 * streams from HBM).  Synchronises the stream.  Errors: EINVAL (null or
 * misaligned), ERANGE (sizes), EDEVICE. */
int vqe_copy_ceiling(const void* src, void* dst, int64_t bytes, int passes, void* hip_stream,
                     double* ms);

/* Measurement helper, not a step of the method: one launch of two 512-thread
 * workgroups per compute unit, each reading, changing and writing back its
 * own 64 KiB LDS array (16-byte accesses, consecutive lanes on consecutive
 * addresses) `iters` times (1..1000000), timed with HIP events on
 * hip_stream.  *ms receives the launch time and *bytes the LDS bytes moved
 * (reads + writes); their ratio is the measured LDS ceiling the gate
 * kernels' on-chip traffic (each pair's amplitudes read and written back
 * through LDS) is reported against.  No device memory is allocated.
 * Synchronises the stream.  Errors: EINVAL (null output), ERANGE (iters),
 * EDEVICE. */
int vqe_lds_ceiling(int iters, void* hip_stream, double* ms, double* bytes);

/* ---------------------------------------------------------------------------
 * BFGS and the VQE loop
 * ------------------------------------------------------------------------ */

typedef struct {
    int max_iter;        /* iteration cap (accepted steps) */
    double gtol;         /* stop when max |g_i| <= gtol */
    double ftol;         /* stop when |f_k - f_{k+1}| <= ftol * max(1, |f_k|); 0 disables */
    double max_seconds;  /* wall-clock budget; <= 0 disables */
    int record_trace;    /* write f after each iteration into trace_out */
} vqe_options;

typedef struct {
    double energy;       /* final objective value */
    int iters;           /* accepted BFGS iterations */
    int n_evals;         /* objective + gradient evaluations */
    int converged;       /* 1 if gtol or ftol was met, else 0 */
} vqe_result;

/* Objective callback: writes f and g (n doubles) at x; returns 0 on success,
 * nonzero to abort the minimisation (reported as EINVAL). */
typedef int (*vqe_objective_fn)(void* ctx, int n, const double* x, double* f, double* g);

/* BFGS (inverse-Hessian form, H0 = I rescaled by y's/y'y before the first
 * update) with a strong-Wolfe line search (c1 = 1e-4, c2 = 0.9; bracketing
 * and zoom with cubic interpolation).  trace_out (nullable) receives
 * max_iter + 1 doubles: f after 0, 1, ... iterations (unused entries NaN).
 * Non-convergence returns VQE_OK with converged = 0; a non-finite f or g
 * returns ENUMERIC. */
int vqe_minimize_bfgs(int n, vqe_objective_fn fn, void* ctx, const double* x0,
                      const vqe_options* opts, double* x_out, double* trace_out,
                      vqe_result* res);

/* VQE (Sec. 2.1.1, Eq. 1): vqe_minimize_bfgs over vqe_energy_grad from
 * theta0 (NULL = all zeros, the HF state).  theta_out receives n_params. */
int vqe_run(const vqe_hamiltonian* H, const vqe_ansatz* A, int n_electrons,
            const double* theta0, const vqe_options* opts, double* theta_out,
            double* trace_out, vqe_result* res, void* hip_stream);

typedef struct {
    double grad_tol;      /* stop once the pool gradient's L2 norm < grad_tol */
    double tie_tol;       /* |g| within tie_tol of the largest count as tied;
                           * ties go to the lowest pool index */
    int max_operators;    /* cap on operators added (>= 0) */
    vqe_options vqe;      /* options of each re-optimisation */
} vqe_adapt_options;

typedef struct {
    double energy;        /* energy of the final ansatz at its optimum */
    double grad_norm;     /* pool-gradient L2 norm there */
    int n_operators;      /* operators in the final ansatz */
    int converged;        /* 1 if grad_norm < grad_tol */
    int n_evals;          /* energy (+gradient) evaluations, pool gradients included */
    int vqe_iters;        /* BFGS iterations summed over the re-optimisations */
} vqe_adapt_result;

/* ADAPT-VQE (Sec. 2.1, "ADAPT-VQE algorithm"; Fig. 2(b)) from the identity
 * ansatz: evaluate the pool gradient at the current optimum; stop when its
 * L2 norm is below grad_tol or max_operators are in; else append the
 * selected pool operator (applied last, new angle 0, earlier angles kept)
 * and run vqe_run over all angles.  Outputs (host): selected[k] and
 * theta_out[k] for k < res->n_operators (capacity max_operators);
 * energy_trace / grad_norm_trace (NULL allowed; capacity max_operators + 1)
 * hold the energy and pool-gradient norm of the 0, 1, ... operator ansatz
 * at its optimum.  vqe_ansatz_select(pool, n, selected) rebuilds the final
 * ansatz.  Errors of the evaluations and of vqe_run are returned as is. */
int vqe_adapt(const vqe_hamiltonian* H, const vqe_ansatz* pool, int n_electrons,
              const vqe_adapt_options* opts, int32_t* selected, double* theta_out,
              double* energy_trace, double* grad_norm_trace, vqe_adapt_result* res,
              void* hip_stream);

/* ---------------------------------------------------------------------------
 * Warm-start MLP (a project addition beside the method: it predicts UCCSD
 * amplitudes for a new bond-stretch geometry from the converged amplitudes
 * of neighbouring geometries, Sec. 3.1 "Results for bond stretching")
 *
 * Layers z_l = a_{l-1} W_l^T + b_l, GELU (exact erf form) after every layer
 * but the last; loss = mean squared error; Adam.  Products take bfloat16
 * operands (round to nearest even) on the matrix cores with FP32
 * accumulation; biases, activations' pre-images, loss, master weights and
 * Adam moments are FP32.  Parameters are packed per layer as W_l
 * [out][in] row-major followed by b_l [out].  All arrays are host arrays.
 * ------------------------------------------------------------------------ */
typedef struct vqe_mlp vqe_mlp;

/* widths[0..n_layers]: input, hidden..., output (1 <= n_layers <= 8, each
 * width in [1, 8192]).  Parameters start at zero; hip_stream is unused (the
 * network orders its work on a private stream). */
int vqe_mlp_create(int n_layers, const int32_t* widths, void* hip_stream, vqe_mlp** out);
int vqe_mlp_n_params(const vqe_mlp* n, int64_t* count);
/* Load the FP32 master parameters (finite) and reset the Adam state. */
int vqe_mlp_set_params(vqe_mlp* n, const float* params);
int vqe_mlp_get_params(const vqe_mlp* n, float* params);
/* y[batch][out] = network(x[batch][in]); 1 <= batch <= 65536. */
int vqe_mlp_forward(vqe_mlp* n, int batch, const float* x, float* y);
/* Loss and its gradient with respect to the packed parameters (grad
 * nullable), without an update. */
int vqe_mlp_loss_grad(vqe_mlp* n, int batch, const float* x, const float* y, float* loss,
                      float* grad);
/* `steps` full-batch Adam steps (one HIP-graph launch per step); the Adam
 * step count continues across calls.  loss_trace (nullable, `steps` floats)
 * receives the loss before each step. */
int vqe_mlp_train(vqe_mlp* n, int batch, const float* x, const float* y, int steps, float lr,
                  float beta1, float beta2, float eps, float* loss_trace);
void vqe_mlp_free(vqe_mlp* n);

#ifdef __cplusplus
}
#endif

#endif /* VQE_H */
