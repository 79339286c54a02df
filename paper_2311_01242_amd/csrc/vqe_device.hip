// Device side of the VQE library for MI355X (gfx950, wave64): statevector
// kernels and the C-ABI entry points that launch them.
//
// Every kernel works on a table of StateDesc records and takes its state
// from blockIdx.y, so one launch serves a single state or a whole batch of
// structurally identical states.
//
// Kernels (all FP64, complex128 amplitudes as double2):
//   k_angles      (cos, sin) of every gate angle from the device theta vector
//   k_hf          |HF> = basis state 2^n_e - 1 (Sec. 2.1.1, Eq. 1 reference)
//   k_exc         UCCSD excitation gate exp(theta (T - T^dag)) (Sec. 2.1.2):
//                 Givens rotation on index pairs (D, D ^ x) with Jordan-Wigner
//                 parity sign (-1)^{popcount(D & chain)}
//   k_pauli       exp(-i phi/2 P) on pairs (b, b ^ x) with popcount phases
//   k_hx          lambda = H psi by x-mask groups (one gather of psi[b ^ x]
//                 serves every z-mask of the group) and per-block partials of
//                 Re <psi|lambda> (Eq. 1's expectation)
//   k_adj_*       one reverse-sweep step of the adjoint gradient: partial
//                 sums of <lambda| dU_j |phi> and U_j^dag on phi and lambda
//   k_reduce      fixed-order sums of the per-block partials (bitwise
//                 reproducible: no floating-point atomics anywhere)
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <tuple>

#include "internal.h"

namespace vqe {

constexpr int kBlock = 256;          // threads per block (4 wave64)
constexpr int kMaxBlocks = 2048;     // grid-stride cap (8 blocks per CU)

struct DevHam {
    GroupDesc* groups = nullptr;
    SubDesc* subs = nullptr;
    double* tabs = nullptr;
};

struct DevAnsatz {
    GateDesc* gates = nullptr;
};

struct StateDesc {
    double2* phi;            // forward state (overwritten by the reverse sweep)
    double2* lam;            // lambda = H phi (nullable for energy only)
    const GateDesc* gates;   // [M]
    double2* cs;             // [M] (cos, sin) of each gate's angle
    const double* theta;     // [P]
    const GroupDesc* groups; // [G]
    const SubDesc* subs;
    const double* tabs;
    double* part_e;          // [nblk_e] energy partials
    double* part_g;          // [M * nblk_g] gradient partials
    double* out_e;           // [1]
    double* out_g;           // [M] raw per-gate gradient sums
    int32_t n, G, M, ne;
};

// ------------------------------------------------------------------ helpers

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Fixed-order block sum; the result is valid in thread 0.
__device__ __forceinline__ double block_sum(double v) {
    __shared__ double sh[kBlock / 64];
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) sh[w] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0) {
#pragma unroll
        for (int i = 0; i < kBlock / 64; ++i) r += sh[i];
    }
    return r;
}

// Deposit the bits of t into the positions NOT set in x (zeros at x's bits).
__device__ __forceinline__ uint64_t insert_zeros(uint64_t t, uint32_t x) {
    while (x) {
        const int q = __ffs(x) - 1;
        x &= x - 1;
        const uint64_t lo = t & ((uint64_t(1) << q) - 1);
        t = ((t >> q) << (q + 1)) | lo;
    }
    return t;
}

__device__ __forceinline__ double parity_sign(uint32_t v) {
    return (__popc(v) & 1) ? -1.0 : 1.0;
}

// Table index: the bits of b at the group's (up to 4) x positions.
__device__ __forceinline__ uint32_t pext_pos(uint32_t b, uint32_t pos) {
    const int k = pos & 7;
    uint32_t u = 0;
    for (int i = 0; i < k; ++i) u |= ((b >> ((pos >> (3 + 5 * i)) & 31)) & 1u) << i;
    return u;
}

// ------------------------------------------------------------------ kernels

__global__ void k_angles(const StateDesc* __restrict__ sd) {
    const StateDesc& s = sd[blockIdx.y];
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= s.M) return;
    const GateDesc g = s.gates[j];
    double a = g.scale * s.theta[g.param];
    if (g.type == kPauli) a *= 0.5;
    double sn, c;
    sincos(a, &sn, &c);
    s.cs[j] = make_double2(c, sn);
}

__global__ void k_hf(const StateDesc* __restrict__ sd, uint64_t N) {
    const StateDesc& s = sd[blockIdx.y];
    const uint64_t hf = (uint64_t(1) << s.ne) - 1;
    for (uint64_t b = blockIdx.x * uint64_t(blockDim.x) + threadIdx.x; b < N;
         b += uint64_t(gridDim.x) * blockDim.x)
        s.phi[b] = make_double2(b == hf ? 1.0 : 0.0, 0.0);
}

// Forward excitation gate j on phi.
__global__ void k_exc(const StateDesc* __restrict__ sd, int j, uint64_t npairs) {
    const StateDesc& s = sd[blockIdx.y];
    const GateDesc g = s.gates[j];
    const double2 cs = s.cs[j];
    double2* __restrict__ psi = s.phi;
    for (uint64_t t = blockIdx.x * uint64_t(blockDim.x) + threadIdx.x; t < npairs;
         t += uint64_t(gridDim.x) * blockDim.x) {
        const uint64_t D = insert_zeros(t, g.x) | g.pd;
        const uint64_t E = D ^ g.x;
        const double ss = g.csign * parity_sign(uint32_t(D) & g.chain) * cs.y;
        const double2 pd = psi[D], pe = psi[E];
        psi[D] = make_double2(cs.x * pd.x - ss * pe.x, cs.x * pd.y - ss * pe.y);
        psi[E] = make_double2(cs.x * pe.x + ss * pd.x, cs.x * pe.y + ss * pd.y);
    }
}

// i^y for y = popcount(x & z) mod 4, times -i (the rotation's -i sin factor).
__device__ __forceinline__ double2 minus_i_times_i_pow(int y) {
    switch (y & 3) {
        case 0: return make_double2(0.0, -1.0);
        case 1: return make_double2(1.0, 0.0);
        case 2: return make_double2(0.0, 1.0);
        default: return make_double2(-1.0, 0.0);
    }
}

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// psi'[b] = c psi[b] + s f (-1)^{|b' & z|} psi[b'],  f = -i * i^{|x & z|},
// which is exp(-i phi/2 P) with P|b'> = i^y (-1)^{|b' & z|} |b>.
// s < 0 gives the inverse rotation.
__device__ __forceinline__ void pauli_pair(double2* psi, uint64_t b, uint32_t x, uint32_t z,
                                           double c, double s, double2 f) {
    const uint64_t bp = b ^ x;
    const double2 a0 = psi[b], a1 = psi[bp];
    const double s0 = s * parity_sign(uint32_t(bp) & z);   // factor on psi[b'] -> b
    const double s1 = s * parity_sign(uint32_t(b) & z);    // factor on psi[b] -> b'
    const double2 t0 = cmul(f, a1), t1 = cmul(f, a0);
    psi[b] = make_double2(c * a0.x + s0 * t0.x, c * a0.y + s0 * t0.y);
    psi[bp] = make_double2(c * a1.x + s1 * t1.x, c * a1.y + s1 * t1.y);
}

__device__ __forceinline__ void pauli_diag(double2* psi, uint64_t b, uint32_t z, double c,
                                           double s) {
    // (c - i s sigma) * psi[b], sigma = (-1)^{|b & z|}
    const double2 a = psi[b];
    const double ss = s * parity_sign(uint32_t(b) & z);
    psi[b] = make_double2(c * a.x + ss * a.y, c * a.y - ss * a.x);
}

__global__ void k_pauli(const StateDesc* __restrict__ sd, int j, uint64_t N, double dir) {
    const StateDesc& s = sd[blockIdx.y];
    const GateDesc g = s.gates[j];
    const double2 cs = s.cs[j];
    const double sn = dir * cs.y;
    const uint32_t x = g.x, z = g.chain;
    if (x == 0) {
        for (uint64_t b = blockIdx.x * uint64_t(blockDim.x) + threadIdx.x; b < N;
             b += uint64_t(gridDim.x) * blockDim.x)
            pauli_diag(s.phi, b, z, cs.x, sn);
        return;
    }
    const uint32_t low = x & (~x + 1u);
    const double2 f = minus_i_times_i_pow(__popc(x & z));
    for (uint64_t t = blockIdx.x * uint64_t(blockDim.x) + threadIdx.x; t < (N >> 1);
         t += uint64_t(gridDim.x) * blockDim.x)
        pauli_pair(s.phi, insert_zeros(t, low), x, z, cs.x, sn, f);
}

// lambda = H phi over the x-groups; partials of Re <phi|lambda>.
__global__ void __launch_bounds__(kBlock) k_hx(const StateDesc* __restrict__ sd, uint64_t N,
                                               int write_lam) {
    const StateDesc& s = sd[blockIdx.y];
    const double2* __restrict__ phi = s.phi;
    const GroupDesc* __restrict__ groups = s.groups;
    const SubDesc* __restrict__ subs = s.subs;
    const double* __restrict__ tabs = s.tabs;
    const int G = s.G;
    double acc = 0.0;
    for (uint64_t b = blockIdx.x * uint64_t(blockDim.x) + threadIdx.x; b < N;
         b += uint64_t(gridDim.x) * blockDim.x) {
        const uint32_t b32 = uint32_t(b);
        double lr = 0.0, li = 0.0;
        for (int gi = 0; gi < G; ++gi) {
            const GroupDesc gd = groups[gi];
            const double2 p = phi[b ^ gd.x];
            const uint32_t u = pext_pos(b32, gd.pos);
            double d = 0.0;
            for (int si = gd.sub_begin; si < gd.sub_end; ++si) {
                const SubDesc sub = subs[si];
                const double t = tabs[sub.tab + u];
                d += (__popc(b32 & sub.w) & 1) ? -t : t;
            }
            lr += d * p.x;
            li += d * p.y;
        }
        if (write_lam) s.lam[b] = make_double2(lr, li);
        const double2 q = phi[b];
        acc += q.x * lr + q.y * li;
    }
    const double r = block_sum(acc);
    if (threadIdx.x == 0) s.part_e[blockIdx.x] = r;
}

// Reverse-sweep step for excitation gate j: partial of Re <lambda| A_j phi>,
// then phi <- U_j^dag phi and lambda <- U_j^dag lambda.
__global__ void __launch_bounds__(kBlock) k_adj_exc(const StateDesc* __restrict__ sd, int j,
                                                    uint64_t npairs) {
    const StateDesc& s = sd[blockIdx.y];
    const GateDesc g = s.gates[j];
    const double2 cs = s.cs[j];
    double2* __restrict__ phi = s.phi;
    double2* __restrict__ lam = s.lam;
    double acc = 0.0;
    for (uint64_t t = blockIdx.x * uint64_t(blockDim.x) + threadIdx.x; t < npairs;
         t += uint64_t(gridDim.x) * blockDim.x) {
        const uint64_t D = insert_zeros(t, g.x) | g.pd;
        const uint64_t E = D ^ g.x;
        const double sg = g.csign * parity_sign(uint32_t(D) & g.chain);
        const double2 fD = phi[D], fE = phi[E], lD = lam[D], lE = lam[E];
        // A|D> = s|E>, A|E> = -s|D>:  <lam|A phi> = s (lam_E^* phi_D - lam_D^* phi_E)
        acc += sg * ((lE.x * fD.x + lE.y * fD.y) - (lD.x * fE.x + lD.y * fE.y));
        const double ss = sg * cs.y;   // U^dag = rotation by -theta
        phi[D] = make_double2(cs.x * fD.x + ss * fE.x, cs.x * fD.y + ss * fE.y);
        phi[E] = make_double2(cs.x * fE.x - ss * fD.x, cs.x * fE.y - ss * fD.y);
        lam[D] = make_double2(cs.x * lD.x + ss * lE.x, cs.x * lD.y + ss * lE.y);
        lam[E] = make_double2(cs.x * lE.x - ss * lD.x, cs.x * lE.y - ss * lD.y);
    }
    const double r = block_sum(acc);
    if (threadIdx.x == 0) s.part_g[size_t(j) * gridDim.x + blockIdx.x] = r;
}

// Reverse-sweep step for Pauli rotation j: partial of Im <lambda|P phi>,
// then the inverse rotation on phi and lambda.
__global__ void __launch_bounds__(kBlock) k_adj_pauli(const StateDesc* __restrict__ sd, int j,
                                                      uint64_t N) {
    const StateDesc& s = sd[blockIdx.y];
    const GateDesc g = s.gates[j];
    const double2 cs = s.cs[j];
    double2* __restrict__ phi = s.phi;
    double2* __restrict__ lam = s.lam;
    const uint32_t x = g.x, z = g.chain;
    double acc = 0.0;
    if (x == 0) {
        for (uint64_t b = blockIdx.x * uint64_t(blockDim.x) + threadIdx.x; b < N;
             b += uint64_t(gridDim.x) * blockDim.x) {
            const double sg = parity_sign(uint32_t(b) & z);
            const double2 f = phi[b], l = lam[b];
            acc += sg * (l.x * f.y - l.y * f.x);   // Im(conj(l) f) * sigma
            pauli_diag(phi, b, z, cs.x, -cs.y);
            pauli_diag(lam, b, z, cs.x, -cs.y);
        }
    } else {
        const uint32_t low = x & (~x + 1u);
        const int y = __popc(x & z) & 3;
        const double2 iy = (y == 0) ? make_double2(1, 0)
                         : (y == 1) ? make_double2(0, 1)
                         : (y == 2) ? make_double2(-1, 0) : make_double2(0, -1);
        const double2 f = minus_i_times_i_pow(y);
        for (uint64_t t = blockIdx.x * uint64_t(blockDim.x) + threadIdx.x; t < (N >> 1);
             t += uint64_t(gridDim.x) * blockDim.x) {
            const uint64_t b = insert_zeros(t, low), bp = b ^ x;
            const double2 f0 = phi[b], f1 = phi[bp], l0 = lam[b], l1 = lam[bp];
            // (P phi)[b] = i^y sigma(b') phi[b'],  (P phi)[b'] = i^y sigma(b) phi[b]
            const double2 p0 = cmul(iy, f1), p1 = cmul(iy, f0);
            const double s0 = parity_sign(uint32_t(bp) & z), s1 = parity_sign(uint32_t(b) & z);
            acc += s0 * (l0.x * p0.y - l0.y * p0.x) + s1 * (l1.x * p1.y - l1.y * p1.x);
            pauli_pair(phi, b, x, z, cs.x, -cs.y, f);
            pauli_pair(lam, b, x, z, cs.x, -cs.y, f);
        }
    }
    const double r = block_sum(acc);
    if (threadIdx.x == 0) s.part_g[size_t(j) * gridDim.x + blockIdx.x] = r;
}

// out[i] = sum_b part[i * nblk + b] in a fixed order; grid (count, states).
__global__ void __launch_bounds__(kBlock) k_reduce(const StateDesc* __restrict__ sd, int which,
                                                   int nblk) {
    const StateDesc& s = sd[blockIdx.y];
    const int i = blockIdx.x;
    const double* part = which == 0 ? s.part_e : s.part_g + size_t(i) * nblk;
    double acc = 0.0;
    for (int b = threadIdx.x; b < nblk; b += blockDim.x) acc += part[b];
    const double r = block_sum(acc);
    if (threadIdx.x == 0) {
        if (which == 0)
            s.out_e[0] = r;
        else
            s.out_g[i] = r;
    }
}

// ---------------------------------------------------------------- host glue

#define HIPCHK(expr)                                                                        \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess)                                                               \
            return fail(VQE_EDEVICE, std::string("HIP error in ") + #expr + ": " +         \
                                         hipGetErrorString(e_));                            \
    } while (0)

static int blocks_for(uint64_t work) {
    const uint64_t b = (work + kBlock - 1) / kBlock;
    return int(std::max<uint64_t>(1, std::min<uint64_t>(b, kMaxBlocks)));
}

template <class T>
static int upload(T** dst, const std::vector<T>& src) {
    *dst = nullptr;
    if (src.empty()) return VQE_OK;
    HIPCHK(hipMalloc(dst, src.size() * sizeof(T)));
    HIPCHK(hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice));
    return VQE_OK;
}

static int current_device(int* dev) {
    HIPCHK(hipGetDevice(dev));
    return VQE_OK;
}

static int dev_ham(const vqe_hamiltonian* H, DevHam** out) {
    int dev;
    if (int rc = current_device(&dev)) return rc;
    std::lock_guard<std::mutex> lk(H->mu);
    auto it = H->dev.find(dev);
    if (it != H->dev.end()) {
        *out = it->second;
        return VQE_OK;
    }
    auto* d = new DevHam();
    int rc = upload(&d->groups, H->groups);
    if (!rc) rc = upload(&d->subs, H->subs);
    if (!rc) rc = upload(&d->tabs, H->tabs);
    if (rc) {
        (void)hipFree(d->groups);
        (void)hipFree(d->subs);
        (void)hipFree(d->tabs);
        delete d;
        return rc;
    }
    H->dev[dev] = d;
    *out = d;
    return VQE_OK;
}

static int dev_ansatz(const vqe_ansatz* A, DevAnsatz** out) {
    int dev;
    if (int rc = current_device(&dev)) return rc;
    std::lock_guard<std::mutex> lk(A->mu);
    auto it = A->dev.find(dev);
    if (it != A->dev.end()) {
        *out = it->second;
        return VQE_OK;
    }
    auto* d = new DevAnsatz();
    if (int rc = upload(&d->gates, A->gates)) {
        delete d;
        return rc;
    }
    A->dev[dev] = d;
    *out = d;
    return VQE_OK;
}

// Reusable device scratch for single-state evaluations, one per
// (device, stream); grows, never shrinks.
struct Workspace {
    size_t state_bytes = 0;
    double2* phi = nullptr;
    double2* lam = nullptr;
    size_t scratch_bytes = 0;
    char* scratch = nullptr;     // theta, cs, partials, outputs, descriptor
};

static std::mutex g_ws_mu;
static std::map<std::pair<int, void*>, Workspace*> g_ws;

static int fits_device(size_t bytes) {
    size_t fr = 0, tot = 0;
    HIPCHK(hipMemGetInfo(&fr, &tot));
    if (bytes > fr)
        return fail(VQE_ENOMEM, "device memory: need " + std::to_string(bytes) + " bytes, " +
                                    std::to_string(fr) + " free");
    return VQE_OK;
}

static int workspace(void* stream, size_t state_bytes, bool two, size_t scratch_bytes,
                     Workspace** out) {
    int dev;
    if (int rc = current_device(&dev)) return rc;
    std::lock_guard<std::mutex> lk(g_ws_mu);
    Workspace*& ws = g_ws[{dev, stream}];
    if (!ws) ws = new Workspace();
    if (ws->state_bytes < state_bytes || (two && !ws->lam)) {
        HIPCHK(hipStreamSynchronize((hipStream_t)stream));
        (void)hipFree(ws->phi);
        (void)hipFree(ws->lam);
        ws->phi = ws->lam = nullptr;
        ws->state_bytes = 0;
        const size_t need = state_bytes * 2;   // always keep room for lambda
        if (int rc = fits_device(need)) return rc;
        HIPCHK(hipMalloc(&ws->phi, state_bytes));
        HIPCHK(hipMalloc(&ws->lam, state_bytes));
        ws->state_bytes = state_bytes;
    }
    if (ws->scratch_bytes < scratch_bytes) {
        HIPCHK(hipStreamSynchronize((hipStream_t)stream));
        (void)hipFree(ws->scratch);
        ws->scratch = nullptr;
        ws->scratch_bytes = 0;
        HIPCHK(hipMalloc(&ws->scratch, scratch_bytes));
        ws->scratch_bytes = scratch_bytes;
    }
    *out = ws;
    return VQE_OK;
}

// Bump allocator over a scratch block (256-byte aligned slices).
struct Carver {
    char* base;
    size_t off = 0;
    template <class T>
    T* take(size_t count) {
        off = (off + 255) & ~size_t(255);
        T* p = reinterpret_cast<T*>(base + off);
        off += count * sizeof(T);
        return p;
    }
};

static size_t carve_size(int64_t M, int64_t P, int nblk_e, int nblk_g) {
    size_t s = 0;
    auto add = [&](size_t bytes) { s = ((s + 255) & ~size_t(255)) + bytes; };
    add(sizeof(double) * std::max<int64_t>(P, 1));          // theta
    add(sizeof(double2) * std::max<int64_t>(M, 1));         // cs
    add(sizeof(double) * nblk_e);                           // part_e
    add(sizeof(double) * size_t(std::max<int64_t>(M, 1)) * nblk_g);  // part_g
    add(sizeof(double));                                    // out_e
    add(sizeof(double) * std::max<int64_t>(M, 1));          // out_g
    add(sizeof(StateDesc));
    return s + 256;
}

// Launch geometry shared by the single-state and batched paths.
struct Geometry {
    uint64_t N;
    int nblk_e, nblk_g;
};

static Geometry geometry(int n) {
    Geometry g;
    g.N = uint64_t(1) << n;
    g.nblk_e = blocks_for(g.N);
    g.nblk_g = blocks_for(g.N >> 2);
    return g;
}


// Enqueue one energy (+ gradient) evaluation for `count` consecutive
// StateDesc records at sd_dev, all with n qubits and the gate program of A.
static int enqueue_eval(const StateDesc* sd_dev, int count, int n, const vqe_ansatz* A,
                        bool grad, hipStream_t st) {
    const Geometry geo = geometry(n);
    const int64_t M = int64_t(A->gates.size());
    if (M > 0)
        hipLaunchKernelGGL(k_angles, dim3(unsigned((M + kBlock - 1) / kBlock), count),
                           dim3(kBlock), 0, st, sd_dev);
    hipLaunchKernelGGL(k_hf, dim3(blocks_for(geo.N), count), dim3(kBlock), 0, st, sd_dev, geo.N);
    for (int64_t j = 0; j < M; ++j) {
        const GateDesc& g = A->gates[j];
        if (g.type == kExcitation) {
            const uint64_t np = geo.N >> __builtin_popcount(g.x);
            hipLaunchKernelGGL(k_exc, dim3(blocks_for(np), count), dim3(kBlock), 0, st, sd_dev,
                               int(j), np);
        } else {
            hipLaunchKernelGGL(k_pauli, dim3(blocks_for(geo.N >> 1), count), dim3(kBlock), 0, st,
                               sd_dev, int(j), geo.N, 1.0);
        }
    }
    hipLaunchKernelGGL(k_hx, dim3(geo.nblk_e, count), dim3(kBlock), 0, st, sd_dev, geo.N,
                       grad ? 1 : 0);
    hipLaunchKernelGGL(k_reduce, dim3(1, count), dim3(kBlock), 0, st, sd_dev, 0, geo.nblk_e);
    if (grad && M > 0) {
        for (int64_t j = M - 1; j >= 0; --j) {
            const GateDesc& g = A->gates[j];
            if (g.type == kExcitation) {
                const uint64_t np = geo.N >> __builtin_popcount(g.x);
                hipLaunchKernelGGL(k_adj_exc, dim3(geo.nblk_g, count), dim3(kBlock), 0, st,
                                   sd_dev, int(j), np);
            } else {
                hipLaunchKernelGGL(k_adj_pauli, dim3(geo.nblk_g, count), dim3(kBlock), 0, st,
                                   sd_dev, int(j), geo.N);
            }
        }
        hipLaunchKernelGGL(k_reduce, dim3(unsigned(M), count), dim3(kBlock), 0, st, sd_dev, 1,
                           geo.nblk_g);
    }
    HIPCHK(hipGetLastError());
    return VQE_OK;
}

// Per-parameter gradient from the raw per-gate sums, in gate order.
static void accumulate_grad(const vqe_ansatz* A, const double* raw, double* grad) {
    std::fill(grad, grad + A->n_params, 0.0);
    for (size_t j = 0; j < A->gates.size(); ++j) {
        const GateDesc& g = A->gates[j];
        // excitation: dE/dtheta = 2 scale Re<lam|A phi>; rotation: scale Im<lam|P phi>
        grad[g.param] += (g.type == kExcitation ? 2.0 : 1.0) * g.scale * raw[j];
    }
}

static int check_pair(const vqe_hamiltonian* H, const vqe_ansatz* A, int ne) {
    if (!H || !A) return fail(VQE_EINVAL, "null Hamiltonian or ansatz");
    if (H->n != A->n) return fail(VQE_EINVAL, "Hamiltonian and ansatz qubit counts differ");
    if (ne < 0 || ne > H->n) return fail(VQE_ERANGE, "n_electrons must be in [0, n_qubits]");
    if (A->n_electrons >= 0 && A->n_electrons != ne)
        return fail(VQE_EINVAL, "n_electrons differs from the ansatz reference");
    return VQE_OK;
}

}  // namespace vqe

using namespace vqe;

// ===================================================================== C ABI

struct vqe_state {
    int n = 0;
    int dev = 0;
    double2* ptr = nullptr;
    bool owned = false;
    hipStream_t st = nullptr;
};

vqe_hamiltonian::~vqe_hamiltonian() {
    int cur = 0;
    (void)hipGetDevice(&cur);
    for (auto& kv : dev) {
        (void)hipSetDevice(kv.first);
        (void)hipFree(kv.second->groups);
        (void)hipFree(kv.second->subs);
        (void)hipFree(kv.second->tabs);
        delete kv.second;
    }
    (void)hipSetDevice(cur);
}

vqe_ansatz::~vqe_ansatz() {
    int cur = 0;
    (void)hipGetDevice(&cur);
    for (auto& kv : dev) {
        (void)hipSetDevice(kv.first);
        (void)hipFree(kv.second->gates);
        delete kv.second;
    }
    (void)hipSetDevice(cur);
}

extern "C" int vqe_state_create(int n, void* stream, vqe_state** out) {
    if (!out) return fail(VQE_EINVAL, "null output pointer");
    *out = nullptr;
    if (n < 1 || n > 32) return fail(VQE_ERANGE, "n_qubits must be in [1, 32]");
    const size_t bytes = sizeof(double2) << n;
    if (int rc = fits_device(bytes)) return rc;
    auto* s = new vqe_state();
    s->n = n;
    s->st = (hipStream_t)stream;
    s->owned = true;
    hipError_t e = hipGetDevice(&s->dev);
    if (e == hipSuccess) e = hipMalloc(&s->ptr, bytes);
    if (e != hipSuccess) {
        delete s;
        return fail(e == hipErrorOutOfMemory ? VQE_ENOMEM : VQE_EDEVICE,
                    std::string("state allocation: ") + hipGetErrorString(e));
    }
    *out = s;
    return VQE_OK;
}

extern "C" int vqe_state_wrap(int n, void* ptr, void* stream, vqe_state** out) {
    if (!out || !ptr) return fail(VQE_EINVAL, "null pointer argument");
    *out = nullptr;
    if (n < 1 || n > 32) return fail(VQE_ERANGE, "n_qubits must be in [1, 32]");
    if (reinterpret_cast<uintptr_t>(ptr) % 256 != 0)
        return fail(VQE_EINVAL, "state memory must be 256-byte aligned");
    auto* s = new vqe_state();
    s->n = n;
    s->st = (hipStream_t)stream;
    s->ptr = static_cast<double2*>(ptr);
    s->owned = false;
    if (hipGetDevice(&s->dev) != hipSuccess) {
        delete s;
        return fail(VQE_EDEVICE, "hipGetDevice failed");
    }
    *out = s;
    return VQE_OK;
}

extern "C" int vqe_state_data(const vqe_state* s, void** p) {
    if (!s || !p) return fail(VQE_EINVAL, "null pointer argument");
    *p = s->ptr;
    return VQE_OK;
}

extern "C" void vqe_state_free(vqe_state* s) {
    if (!s) return;
    if (s->owned) (void)hipFree(s->ptr);
    delete s;
}

// Small scratch carve for state-level calls: descriptor + a few buffers.
namespace {
struct StateCall {
    Workspace* ws;
    Carver cv;
    StateDesc sd{};
    StateDesc* sd_dev;
};

int begin_state_call(const vqe_state* s, int64_t M, int64_t P, int nblk_e, StateCall* c) {
    if (int rc = workspace(s->st, 0, false, carve_size(M, P, nblk_e, 1), &c->ws)) return rc;
    c->cv = Carver{c->ws->scratch};
    std::memset(&c->sd, 0, sizeof(StateDesc));
    c->sd.phi = s->ptr;
    c->sd.n = s->n;
    c->sd.theta = c->cv.take<double>(std::max<int64_t>(P, 1));
    c->sd.cs = c->cv.take<double2>(std::max<int64_t>(M, 1));
    c->sd.part_e = c->cv.take<double>(nblk_e);
    c->sd.out_e = c->cv.take<double>(1);
    c->sd_dev = c->cv.take<StateDesc>(1);
    return VQE_OK;
}
}  // namespace

extern "C" int vqe_prepare_hf(vqe_state* s, int ne) {
    if (!s) return fail(VQE_EINVAL, "null state");
    if (ne < 0 || ne > s->n) return fail(VQE_ERANGE, "n_electrons must be in [0, n_qubits]");
    StateCall c;
    if (int rc = begin_state_call(s, 0, 0, 1, &c)) return rc;
    c.sd.ne = ne;
    HIPCHK(hipMemcpyAsync(c.sd_dev, &c.sd, sizeof(StateDesc), hipMemcpyHostToDevice, s->st));
    const uint64_t N = uint64_t(1) << s->n;
    hipLaunchKernelGGL(k_hf, dim3(blocks_for(N), 1), dim3(kBlock), 0, s->st, c.sd_dev, N);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(s->st));
    return VQE_OK;
}

extern "C" int vqe_apply_pauli_rotation(vqe_state* s, uint32_t x, uint32_t z, double theta) {
    if (!s) return fail(VQE_EINVAL, "null state");
    const uint32_t lim = (s->n == 32) ? 0xffffffffu : ((1u << s->n) - 1u);
    if ((x & ~lim) || (z & ~lim)) return fail(VQE_ERANGE, "Pauli mask has a bit beyond n_qubits");
    if (!std::isfinite(theta)) return fail(VQE_EINVAL, "theta is not finite");
    StateCall c;
    if (int rc = begin_state_call(s, 1, 1, 1, &c)) return rc;
    GateDesc g{};
    g.type = kPauli;
    g.x = x;
    g.chain = z;
    g.scale = 1.0;
    g.csign = 1.0;
    GateDesc* g_dev = c.cv.take<GateDesc>(1);
    c.sd.gates = g_dev;
    c.sd.M = 1;
    HIPCHK(hipMemcpyAsync(g_dev, &g, sizeof(g), hipMemcpyHostToDevice, s->st));
    HIPCHK(hipMemcpyAsync(const_cast<double*>(c.sd.theta), &theta, sizeof(double),
                          hipMemcpyHostToDevice, s->st));
    HIPCHK(hipMemcpyAsync(c.sd_dev, &c.sd, sizeof(StateDesc), hipMemcpyHostToDevice, s->st));
    const uint64_t N = uint64_t(1) << s->n;
    hipLaunchKernelGGL(k_angles, dim3(1, 1), dim3(kBlock), 0, s->st, c.sd_dev);
    hipLaunchKernelGGL(k_pauli, dim3(blocks_for(N >> 1), 1), dim3(kBlock), 0, s->st, c.sd_dev, 0,
                       N, 1.0);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(s->st));
    return VQE_OK;
}

extern "C" int vqe_apply_ansatz(vqe_state* s, const vqe_ansatz* A, const double* theta) {
    if (!s || !A) return fail(VQE_EINVAL, "null state or ansatz");
    if (A->n != s->n) return fail(VQE_EINVAL, "ansatz and state qubit counts differ");
    if (A->n_params > 0 && !theta) return fail(VQE_EINVAL, "null theta");
    if (!finite_all(theta, A->n_params)) return fail(VQE_EINVAL, "theta has a non-finite entry");
    DevAnsatz* da;
    if (int rc = dev_ansatz(A, &da)) return rc;
    const int64_t M = int64_t(A->gates.size());
    StateCall c;
    if (int rc = begin_state_call(s, M, A->n_params, 1, &c)) return rc;
    c.sd.gates = da->gates;
    c.sd.M = int32_t(M);
    if (A->n_params > 0)
        HIPCHK(hipMemcpyAsync(const_cast<double*>(c.sd.theta), theta, sizeof(double) * A->n_params,
                              hipMemcpyHostToDevice, s->st));
    HIPCHK(hipMemcpyAsync(c.sd_dev, &c.sd, sizeof(StateDesc), hipMemcpyHostToDevice, s->st));
    const uint64_t N = uint64_t(1) << s->n;
    if (M > 0)
        hipLaunchKernelGGL(k_angles, dim3(unsigned((M + kBlock - 1) / kBlock), 1), dim3(kBlock), 0,
                           s->st, c.sd_dev);
    for (int64_t j = 0; j < M; ++j) {
        const GateDesc& g = A->gates[j];
        if (g.type == kExcitation) {
            const uint64_t np = N >> __builtin_popcount(g.x);
            hipLaunchKernelGGL(k_exc, dim3(blocks_for(np), 1), dim3(kBlock), 0, s->st, c.sd_dev,
                               int(j), np);
        } else {
            hipLaunchKernelGGL(k_pauli, dim3(blocks_for(N >> 1), 1), dim3(kBlock), 0, s->st,
                               c.sd_dev, int(j), N, 1.0);
        }
    }
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(s->st));
    return VQE_OK;
}

extern "C" int vqe_expectation(const vqe_state* s, const vqe_hamiltonian* H, double* energy) {
    if (!s || !H || !energy) return fail(VQE_EINVAL, "null pointer argument");
    if (H->n != s->n) return fail(VQE_EINVAL, "Hamiltonian and state qubit counts differ");
    DevHam* dh;
    if (int rc = dev_ham(H, &dh)) return rc;
    const Geometry geo = geometry(s->n);
    StateCall c;
    if (int rc = begin_state_call(s, 0, 0, geo.nblk_e, &c)) return rc;
    c.sd.groups = dh->groups;
    c.sd.subs = dh->subs;
    c.sd.tabs = dh->tabs;
    c.sd.G = int32_t(H->groups.size());
    HIPCHK(hipMemcpyAsync(c.sd_dev, &c.sd, sizeof(StateDesc), hipMemcpyHostToDevice, s->st));
    hipLaunchKernelGGL(k_hx, dim3(geo.nblk_e, 1), dim3(kBlock), 0, s->st, c.sd_dev, geo.N, 0);
    hipLaunchKernelGGL(k_reduce, dim3(1, 1), dim3(kBlock), 0, s->st, c.sd_dev, 0, geo.nblk_e);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(energy, c.sd.out_e, sizeof(double), hipMemcpyDeviceToHost, s->st));
    HIPCHK(hipStreamSynchronize(s->st));
    if (!std::isfinite(*energy)) return fail(VQE_ENUMERIC, "non-finite expectation value");
    return VQE_OK;
}

extern "C" int vqe_energy_grad(const vqe_hamiltonian* H, const vqe_ansatz* A, int ne,
                               const double* theta, double* energy, double* grad, void* stream) {
    if (int rc = check_pair(H, A, ne)) return rc;
    if (!energy) return fail(VQE_EINVAL, "null energy pointer");
    if (A->n_params > 0 && !theta) return fail(VQE_EINVAL, "null theta");
    if (!finite_all(theta, A->n_params)) return fail(VQE_EINVAL, "theta has a non-finite entry");
    hipStream_t st = (hipStream_t)stream;
    const int n = H->n;
    const Geometry geo = geometry(n);
    const int64_t M = int64_t(A->gates.size()), P = A->n_params;
    DevHam* dh;
    DevAnsatz* da;
    if (int rc = dev_ham(H, &dh)) return rc;
    if (int rc = dev_ansatz(A, &da)) return rc;
    Workspace* ws;
    if (int rc = workspace(stream, sizeof(double2) << n, grad != nullptr,
                           carve_size(M, P, geo.nblk_e, geo.nblk_g), &ws))
        return rc;
    Carver cv{ws->scratch};
    StateDesc sd{};
    sd.phi = ws->phi;
    sd.lam = ws->lam;
    sd.gates = da->gates;
    sd.theta = cv.take<double>(std::max<int64_t>(P, 1));
    sd.cs = cv.take<double2>(std::max<int64_t>(M, 1));
    sd.groups = dh->groups;
    sd.subs = dh->subs;
    sd.tabs = dh->tabs;
    sd.part_e = cv.take<double>(geo.nblk_e);
    sd.part_g = cv.take<double>(size_t(std::max<int64_t>(M, 1)) * geo.nblk_g);
    sd.out_e = cv.take<double>(1);
    sd.out_g = cv.take<double>(std::max<int64_t>(M, 1));
    sd.n = n;
    sd.G = int32_t(H->groups.size());
    sd.M = int32_t(M);
    sd.ne = ne;
    StateDesc* sd_dev = cv.take<StateDesc>(1);
    if (P > 0)
        HIPCHK(hipMemcpyAsync(const_cast<double*>(sd.theta), theta, sizeof(double) * P,
                              hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(sd_dev, &sd, sizeof(StateDesc), hipMemcpyHostToDevice, st));
    if (int rc = enqueue_eval(sd_dev, 1, n, A, grad != nullptr, st)) return rc;
    std::vector<double> raw(std::max<int64_t>(M, 1));
    HIPCHK(hipMemcpyAsync(energy, sd.out_e, sizeof(double), hipMemcpyDeviceToHost, st));
    if (grad && M > 0)
        HIPCHK(hipMemcpyAsync(raw.data(), sd.out_g, sizeof(double) * M, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    bool ok = std::isfinite(*energy);
    if (grad) {
        accumulate_grad(A, raw.data(), grad);
        ok = ok && finite_all(grad, P);
    }
    if (!ok) return fail(VQE_ENUMERIC, "non-finite energy or gradient");
    return VQE_OK;
}

// ===================================================================== batch

struct vqe_batch {
    int S = 0;
    int dev = 0;
    hipStream_t st = nullptr;
    std::vector<const vqe_ansatz*> A;
    std::vector<int64_t> poff;      // parameter offsets [S+1]
    std::vector<int64_t> goff;      // gate offsets [S+1]
    std::vector<char*> allocs;      // every device allocation
    double* theta_dev = nullptr;
    double* e_dev = nullptr;
    double* g_dev = nullptr;        // raw per-gate sums, concatenated
    double* theta_h = nullptr;      // pinned staging
    double* e_h = nullptr;
    double* g_h = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    ~vqe_batch() {
        int cur = 0;
        (void)hipGetDevice(&cur);
        (void)hipSetDevice(dev);
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        for (char* p : allocs) (void)hipFree(p);
        (void)hipHostFree(theta_h);
        (void)hipHostFree(e_h);
        (void)hipHostFree(g_h);
        (void)hipSetDevice(cur);
    }
};

namespace {
bool same_program(const vqe_ansatz* a, const vqe_ansatz* b) {
    return a->n == b->n && a->n_params == b->n_params && a->gates.size() == b->gates.size() &&
           std::memcmp(a->gates.data(), b->gates.data(), a->gates.size() * sizeof(GateDesc)) == 0;
}

template <class T>
int dalloc(vqe_batch* b, T** p, size_t count) {
    void* q = nullptr;
    hipError_t e = hipMalloc(&q, std::max<size_t>(count, 1) * sizeof(T));
    if (e != hipSuccess)
        return fail(e == hipErrorOutOfMemory ? VQE_ENOMEM : VQE_EDEVICE,
                    std::string("batch allocation: ") + hipGetErrorString(e));
    b->allocs.push_back(static_cast<char*>(q));
    *p = static_cast<T*>(q);
    return VQE_OK;
}
}  // namespace

extern "C" int vqe_batch_create(int S, const vqe_hamiltonian* const* H, const vqe_ansatz* const* A,
                                const int* ne, void* stream, vqe_batch** out) {
    if (!out || !H || !A || !ne) return fail(VQE_EINVAL, "null pointer argument");
    *out = nullptr;
    if (S < 1) return fail(VQE_ERANGE, "n_states must be >= 1");
    size_t need = 0;
    for (int i = 0; i < S; ++i) {
        if (int rc = check_pair(H[i], A[i], ne[i]))
            return fail(rc, "state " + std::to_string(i) + ": " + vqe_last_error());
        need += 2 * (sizeof(double2) << H[i]->n);
    }
    if (int rc = fits_device(need)) return rc;
    auto* b = new vqe_batch();
    std::unique_ptr<vqe_batch> guard(b);
    b->S = S;
    b->st = (hipStream_t)stream;
    HIPCHK(hipGetDevice(&b->dev));
    b->A.assign(A, A + S);
    b->poff.assign(S + 1, 0);
    b->goff.assign(S + 1, 0);
    for (int i = 0; i < S; ++i) {
        b->poff[i + 1] = b->poff[i] + A[i]->n_params;
        b->goff[i + 1] = b->goff[i] + int64_t(A[i]->gates.size());
    }
    // classes: states with equal qubit count and identical gate programs
    std::vector<int> cls(S, -1), rep;
    for (int i = 0; i < S; ++i) {
        for (size_t c = 0; c < rep.size(); ++c)
            if (same_program(A[rep[c]], A[i]) && A[rep[c]]->n_electrons == A[i]->n_electrons &&
                ne[rep[c]] == ne[i]) {
                cls[i] = int(c);
                break;
            }
        if (cls[i] < 0) {
            cls[i] = int(rep.size());
            rep.push_back(i);
        }
    }
    if (int rc = dalloc(b, &b->theta_dev, b->poff[S])) return rc;
    if (int rc = dalloc(b, &b->e_dev, S)) return rc;
    if (int rc = dalloc(b, &b->g_dev, b->goff[S])) return rc;
    HIPCHK(hipHostMalloc(&b->theta_h, sizeof(double) * std::max<int64_t>(b->poff[S], 1)));
    HIPCHK(hipHostMalloc(&b->e_h, sizeof(double) * S));
    HIPCHK(hipHostMalloc(&b->g_h, sizeof(double) * std::max<int64_t>(b->goff[S], 1)));
    // descriptors, ordered by class so each class is one contiguous slice
    std::vector<int> order(S);
    for (int i = 0; i < S; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int c) { return cls[a] < cls[c]; });
    std::vector<StateDesc> sds(S);
    for (int k = 0; k < S; ++k) {
        const int i = order[k];
        const int n = H[i]->n;
        const Geometry geo = geometry(n);
        const int64_t M = int64_t(A[i]->gates.size());
        DevHam* dh;
        DevAnsatz* da;
        if (int rc = dev_ham(H[i], &dh)) return rc;
        if (int rc = dev_ansatz(A[i], &da)) return rc;
        StateDesc& sd = sds[k];
        std::memset(&sd, 0, sizeof(sd));
        if (int rc = dalloc(b, &sd.phi, size_t(1) << n)) return rc;
        if (int rc = dalloc(b, &sd.lam, size_t(1) << n)) return rc;
        if (int rc = dalloc(b, &sd.cs, std::max<int64_t>(M, 1))) return rc;
        if (int rc = dalloc(b, &sd.part_e, geo.nblk_e)) return rc;
        if (int rc = dalloc(b, &sd.part_g, size_t(std::max<int64_t>(M, 1)) * geo.nblk_g)) return rc;
        sd.gates = da->gates;
        sd.theta = b->theta_dev + b->poff[i];
        sd.groups = dh->groups;
        sd.subs = dh->subs;
        sd.tabs = dh->tabs;
        sd.out_e = b->e_dev + i;
        sd.out_g = b->g_dev + b->goff[i];
        sd.n = n;
        sd.G = int32_t(H[i]->groups.size());
        sd.M = int32_t(M);
        sd.ne = ne[i];
    }
    StateDesc* sd_dev;
    if (int rc = dalloc(b, &sd_dev, S)) return rc;
    HIPCHK(hipMemcpy(sd_dev, sds.data(), sizeof(StateDesc) * S, hipMemcpyHostToDevice));
    // capture one evaluation of every class into a graph
    HIPCHK(hipStreamBeginCapture(b->st, hipStreamCaptureModeThreadLocal));
    int k0 = 0;
    int cap_rc = VQE_OK;
    while (k0 < S && cap_rc == VQE_OK) {
        int k1 = k0;
        while (k1 < S && cls[order[k1]] == cls[order[k0]]) ++k1;
        const vqe_ansatz* a = A[order[k0]];
        cap_rc = enqueue_eval(sd_dev + k0, k1 - k0, a->n, a, true, b->st);
        k0 = k1;
    }
    hipError_t ce = hipStreamEndCapture(b->st, &b->graph);
    if (cap_rc) return cap_rc;
    HIPCHK(ce);
    HIPCHK(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
    *out = guard.release();
    return VQE_OK;
}

extern "C" int vqe_batch_offsets(const vqe_batch* b, int64_t* offsets) {
    if (!b || !offsets) return fail(VQE_EINVAL, "null pointer argument");
    std::copy(b->poff.begin(), b->poff.end(), offsets);
    return VQE_OK;
}

extern "C" int vqe_batch_energy_grad(vqe_batch* b, const double* theta_all, double* e_all,
                                     double* g_all) {
    if (!b || !e_all) return fail(VQE_EINVAL, "null pointer argument");
    const int64_t P = b->poff[b->S];
    if (P > 0 && !theta_all) return fail(VQE_EINVAL, "null theta_all");
    if (!finite_all(theta_all, P)) return fail(VQE_EINVAL, "theta_all has a non-finite entry");
    int cur = 0;
    HIPCHK(hipGetDevice(&cur));
    if (cur != b->dev) return fail(VQE_EINVAL, "batch belongs to another device");
    std::memcpy(b->theta_h, theta_all, sizeof(double) * P);
    HIPCHK(hipMemcpyAsync(b->theta_dev, b->theta_h, sizeof(double) * P, hipMemcpyHostToDevice,
                          b->st));
    HIPCHK(hipGraphLaunch(b->exec, b->st));
    HIPCHK(hipMemcpyAsync(b->e_h, b->e_dev, sizeof(double) * b->S, hipMemcpyDeviceToHost, b->st));
    if (g_all)
        HIPCHK(hipMemcpyAsync(b->g_h, b->g_dev, sizeof(double) * b->goff[b->S],
                              hipMemcpyDeviceToHost, b->st));
    HIPCHK(hipStreamSynchronize(b->st));
    std::memcpy(e_all, b->e_h, sizeof(double) * b->S);
    bool ok = finite_all(e_all, b->S);
    if (g_all) {
        for (int i = 0; i < b->S; ++i) accumulate_grad(b->A[i], b->g_h + b->goff[i], g_all + b->poff[i]);
        ok = ok && finite_all(g_all, P);
    }
    if (!ok) return fail(VQE_ENUMERIC, "non-finite energy or gradient");
    return VQE_OK;
}

extern "C" void vqe_batch_free(vqe_batch* b) { delete b; }
