// Gate kernels of the statevector path (gfx950, wave64, FP64).
//
//  k_angles       (cos, sin) of every gate angle from the device theta vector
//  k_hf           |HF> = basis state 2^n_e - 1 (reference |0> of Sec. 2.1.1, Eq. 1)
//  k_exc          one UCCSD excitation exp(theta (T - T^dag)) (Sec. 2.1.2): a
//                 Givens rotation on the index pairs (D, D ^ x) whose Jordan-
//                 Wigner sign is (-1)^{popcount(D & chain)}
//  k_pauli        one exp(-i phi/2 P) on the pairs (b, b ^ x), popcount phases
//  k_adj_exc/_pauli  one reverse-sweep step of the adjoint gradient
//  k_run_fwd      a run of excitations sharing their created orbitals, applied
//                 to an LDS tile in one read and one write of the tile
//  k_run_adj      the same run reverse-swept on phi and lambda in LDS, with the
//                 per-gate gradient partials
//  k_reduce_*     fixed-order sums of per-block partials (no float atomics,
//                 so results are bitwise reproducible)
#include "device_common.h"

#include <algorithm>

namespace vqe {

int blocks_for(uint64_t work) {
    const uint64_t b = (work + kBlock - 1) / kBlock;
    return int(b < 1 ? 1 : (b > uint64_t(kMaxBlocks) ? uint64_t(kMaxBlocks) : b));
}

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
    const uint64_t hf = s.ref;
    for (uint64_t b = blockIdx.x * uint64_t(blockDim.x) + threadIdx.x; b < N;
         b += uint64_t(gridDim.x) * blockDim.x)
        nt_store(&s.phi[b], make_double2(b == hf ? 1.0 : 0.0, 0.0));
}

__global__ void k_fill_zero(double2* __restrict__ p, uint64_t n) {
    for (uint64_t i = blockIdx.x * uint64_t(blockDim.x) + threadIdx.x; i < n;
         i += uint64_t(gridDim.x) * blockDim.x)
        p[i] = make_double2(0.0, 0.0);
}

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
        double2 a = psi[D], b = psi[E];
        givens(a, b, cs.x, ss);
        psi[D] = a;
        psi[E] = b;
    }
}

// -i * i^y for y = popcount(x & z) mod 4 (the rotation's -i sin(phi/2) factor times P's phase).
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

// exp(-i phi/2 P) on the pair (b, b' = b ^ x), with P|b'> = i^y (-1)^{|b' & z|} |b>:
// psi'[b] = c psi[b] + s f (-1)^{|b' & z|} psi[b'],  f = -i * i^y.  s < 0 inverts.
__device__ __forceinline__ void pauli_pair(double2* psi, uint64_t b, uint32_t x, uint32_t z,
                                           double c, double s, double2 f) {
    const uint64_t bp = b ^ x;
    const double2 a0 = psi[b], a1 = psi[bp];
    const double s0 = s * parity_sign(uint32_t(bp) & z);
    const double s1 = s * parity_sign(uint32_t(b) & z);
    const double2 t0 = cmul(f, a1), t1 = cmul(f, a0);
    psi[b] = make_double2(c * a0.x + s0 * t0.x, c * a0.y + s0 * t0.y);
    psi[bp] = make_double2(c * a1.x + s1 * t1.x, c * a1.y + s1 * t1.y);
}

// Diagonal rotation: psi[b] <- (c - i s sigma(b)) psi[b], sigma = (-1)^{|b & z|}.
__device__ __forceinline__ void pauli_diag(double2* psi, uint64_t b, uint32_t z, double c,
                                           double s) {
    const double2 a = psi[b];
    const double ss = s * parity_sign(uint32_t(b) & z);
    psi[b] = make_double2(c * a.x + ss * a.y, c * a.y - ss * a.x);
}

__global__ void k_pauli(const StateDesc* __restrict__ sd, int j, uint64_t N) {
    const StateDesc& s = sd[blockIdx.y];
    const GateDesc g = s.gates[j];
    const double2 cs = s.cs[j];
    const uint32_t x = g.x, z = g.chain;
    if (x == 0) {
        for (uint64_t b = blockIdx.x * uint64_t(blockDim.x) + threadIdx.x; b < N;
             b += uint64_t(gridDim.x) * blockDim.x)
            pauli_diag(s.phi, b, z, cs.x, cs.y);
        return;
    }
    const uint32_t low = x & (~x + 1u);
    const double2 f = minus_i_times_i_pow(__popc(x & z));
    for (uint64_t t = blockIdx.x * uint64_t(blockDim.x) + threadIdx.x; t < (N >> 1);
         t += uint64_t(gridDim.x) * blockDim.x)
        pauli_pair(s.phi, insert_zeros(t, low), x, z, cs.x, cs.y, f);
}

__global__ void __launch_bounds__(kBlock) k_adj_exc(const StateDesc* __restrict__ sd, int j,
                                                    uint64_t npairs) {
    __shared__ double red[kBlock / 64];
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
        double2 fD = phi[D], fE = phi[E], lD = lam[D], lE = lam[E];
        // A|D> = s|E>, A|E> = -s|D>:  <lam|A phi> = s (lam_E^* phi_D - lam_D^* phi_E)
        acc += sg * ((lE.x * fD.x + lE.y * fD.y) - (lD.x * fE.x + lD.y * fE.y));
        const double ss = -sg * cs.y;   // U^dag: rotation by -theta
        givens(fD, fE, cs.x, ss);
        givens(lD, lE, cs.x, ss);
        phi[D] = fD;
        phi[E] = fE;
        lam[D] = lD;
        lam[E] = lE;
    }
    const double r = block_sum(acc, red);
    if (threadIdx.x == 0) s.part_g[size_t(j) * s.gstride + blockIdx.x] = r;
}

__global__ void __launch_bounds__(kBlock) k_adj_pauli(const StateDesc* __restrict__ sd, int j,
                                                      uint64_t N) {
    __shared__ double red[kBlock / 64];
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
            acc += sg * (l.x * f.y - l.y * f.x);   // Im(conj(l) (P phi)[b])
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
    const double r = block_sum(acc, red);
    if (threadIdx.x == 0) s.part_g[size_t(j) * s.gstride + blockIdx.x] = r;
}

__global__ void __launch_bounds__(kBlock) k_reduce_e(const StateDesc* __restrict__ sd, int nblk) {
    __shared__ double red[kBlock / 64];
    const StateDesc& s = sd[blockIdx.y];
    double acc = 0.0;
    for (int b = threadIdx.x; b < nblk; b += kBlock) acc += s.part_e[b];
    const double r = block_sum(acc, red);
    if (threadIdx.x == 0) s.out_e[0] = r;
}

// out_g[j] = the sum of gate j's partials: one wave per gate (lane l adds
// partials l, l + 64, ... in order, then the fixed-order wave total), four
// gates per workgroup.
__global__ void __launch_bounds__(256) k_reduce_g(const StateDesc* __restrict__ sd,
                                                  const int32_t* __restrict__ cnt, int cnt_uniform, int M) {
    const StateDesc& s = sd[blockIdx.y];
    const int j = blockIdx.x * 4 + int(threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (j >= M) return;   // whole waves
    const int nb = cnt ? cnt[j] : cnt_uniform;
    const double* part = s.part_g + size_t(j) * s.gstride;
    double acc = 0.0;
    for (int b = lane; b < nb; b += 64) acc += part[b];
    acc = wave_total(acc);
    if (lane == 0) s.out_g[j] = acc;
}

// Per-parameter gradient from the raw per-gate sums: parameter q takes, in
// gate order, coef[k] * raw[gate[k]] for k in [start[q], start[q + 1]), each
// product rounded before its addition (the host accumulation's arithmetic, so
// both give the same bits).
__global__ void k_param_grad(const int64_t* __restrict__ start, const int64_t* __restrict__ gate,
                             const double* __restrict__ coef, const double* __restrict__ raw,
                             double* __restrict__ g, int64_t P) {
    const int64_t q = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (q >= P) return;
    double acc = 0.0;
    for (int64_t k = start[q]; k < start[q + 1]; ++k) acc = __dadd_rn(acc, __dmul_rn(coef[k], raw[gate[k]]));
    g[q] = acc;
}

// ------------------------------------------------------------ fused runs

__device__ __forceinline__ uint32_t tile_index(const RunDesc& run, uint32_t o_dep, uint32_t e,
                                               uint32_t half) {
    const uint32_t r = e & (half - 1);
    const uint32_t in = run.contiguous ? r : pdep32(r, run.inner);
    return o_dep | in | ((e >= half) ? run.key : 0u);
}

// Global <-> LDS tile copies use non-temporal accesses: a run reads every
// tile element once and writes it back once, so the lines have no reuse in
// L2; streaming them past the cache roughly doubles the sustained bandwidth
// of this in-place pattern on gfx950 (measured on the 20-qubit batch tiles:
// 2.5 -> 5.2 TB/s for load + store alone).
constexpr int kRunThreads = 512;   // threads per block of the run kernels (8 wave64)

// A run block walks the (state, tile) pairs id = blockIdx.x, blockIdx.x +
// gridDim.x, ...: the tile is loaded into registers (EPT elements per thread
// and vector, all loads in flight at once), copied to LDS, swept through the
// run's gates and written back; with a grid smaller than the tile count the
// next tile's loads are issued before the current gate chain starts.
template <int EPT>
__device__ __forceinline__ void regs_load(double2 (&v)[EPT], const double2* __restrict__ src,
                                          const RunDesc& run, uint32_t o_dep, uint32_t half,
                                          uint32_t T) {
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
        const uint32_t e = threadIdx.x + k * kRunThreads;
        if (e < T) v[k] = nt_load(&src[tile_index(run, o_dep, e, half)]);
    }
}

template <int EPT>
__device__ __forceinline__ void regs_to_lds(double2* __restrict__ dst, const double2 (&v)[EPT],
                                            uint32_t T) {
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
        const uint32_t e = threadIdx.x + k * kRunThreads;
        if (e < T) dst[e] = v[k];
    }
}

template <int EPT>
__device__ __forceinline__ void lds_to_global(double2* __restrict__ dst,
                                              const double2* __restrict__ src, const RunDesc& run,
                                              uint32_t o_dep, uint32_t half, uint32_t T) {
    double2 v[EPT];
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
        const uint32_t e = threadIdx.x + k * kRunThreads;
        if (e < T) v[k] = src[e];
    }
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
        const uint32_t e = threadIdx.x + k * kRunThreads;
        if (e < T) nt_store(&dst[tile_index(run, o_dep, e, half)], v[k]);
    }
}

template <int EPT>
__global__ void __launch_bounds__(kRunThreads) k_run_fwd(const StateDesc* __restrict__ sd, RunDesc run,
                                                         const TileGate* __restrict__ tg, int total) {
    extern __shared__ double2 sh[];
    const uint32_t half = 1u << run.m, T = half << 1;
    int id = blockIdx.x;
    if (id >= total) return;
    double2 pf[EPT];
    regs_load<EPT>(pf, sd[id / run.ntiles].phi, run, pdep32(id % run.ntiles, run.outer), half, T);
    while (true) {
        const StateDesc& s = sd[id / run.ntiles];
        const uint32_t o_dep = pdep32(id % run.ntiles, run.outer);
        __syncthreads();   // the previous tile's write-back has read the LDS tile
        regs_to_lds<EPT>(sh, pf, T);
        __syncthreads();
        const int next = id + gridDim.x;
        if (next < total)
            regs_load<EPT>(pf, sd[next / run.ntiles].phi, run, pdep32(next % run.ntiles, run.outer),
                           half, T);
        for (int j = run.g0; j < run.g1; ++j) {
            const TileGate t = tg[j - run.g0];
            const double2 cs = s.cs[j];
            const double base = t.csign * parity_sign(o_dep & t.chain_out) * cs.y;
            const uint32_t np = half >> __popc(t.xr);
            for (uint32_t p = threadIdx.x; p < np; p += kRunThreads) {
                const uint32_t rD = uint32_t(insert_zeros(p, t.xr)) | t.pdr;
                const uint32_t iE = half + (rD ^ t.xr);
                givens(sh[rD], sh[iE], cs.x, base * parity_sign(rD & t.chr));
            }
            __syncthreads();
        }
        lds_to_global<EPT>(s.phi, sh, run, o_dep, half, T);
        if (next >= total) break;
        id = next;
    }
}

template <int EPT>
__global__ void __launch_bounds__(kRunThreads) k_run_adj(const StateDesc* __restrict__ sd, RunDesc run,
                                                         const TileGate* __restrict__ tg, int total) {
    extern __shared__ double2 sh[];
    __shared__ double red[kMaxRunGates][kRunThreads / 64];   // per-gate, per-wave partial sums
    const uint32_t half = 1u << run.m, T = half << 1;
    double2* shp = sh;
    double2* shl = sh + T;
    int id = blockIdx.x;
    if (id >= total) return;
    double2 pfp[EPT], pfl[EPT];
    {
        const StateDesc& s0 = sd[id / run.ntiles];
        const uint32_t o0 = pdep32(id % run.ntiles, run.outer);
        regs_load<EPT>(pfp, s0.phi, run, o0, half, T);
        regs_load<EPT>(pfl, s0.lam, run, o0, half, T);
    }
    while (true) {
        const StateDesc& s = sd[id / run.ntiles];
        const int o = id % run.ntiles;
        const uint32_t o_dep = pdep32(o, run.outer);
        __syncthreads();   // the previous tile's write-back has read the LDS tiles
        regs_to_lds<EPT>(shp, pfp, T);
        regs_to_lds<EPT>(shl, pfl, T);
        __syncthreads();
        const int next = id + gridDim.x;
        if (next < total) {
            const StateDesc& sn = sd[next / run.ntiles];
            const uint32_t on = pdep32(next % run.ntiles, run.outer);
            regs_load<EPT>(pfp, sn.phi, run, on, half, T);
            regs_load<EPT>(pfl, sn.lam, run, on, half, T);
        }
        for (int j = run.g1 - 1; j >= run.g0; --j) {
            const TileGate t = tg[j - run.g0];
            const double2 cs = s.cs[j];
            const double base = t.csign * parity_sign(o_dep & t.chain_out);
            const uint32_t np = half >> __popc(t.xr);
            double acc = 0.0;
            for (uint32_t p = threadIdx.x; p < np; p += kRunThreads) {
                const uint32_t rD = uint32_t(insert_zeros(p, t.xr)) | t.pdr;
                const uint32_t iE = half + (rD ^ t.xr);
                const double sg = base * parity_sign(rD & t.chr);
                double2 fD = shp[rD], fE = shp[iE], lD = shl[rD], lE = shl[iE];
                // <lam| A phi> with A|D> = s|E>, A|E> = -s|D>
                acc += sg * ((lE.x * fD.x + lE.y * fD.y) - (lD.x * fE.x + lD.y * fE.y));
                const double ss = -sg * cs.y;   // U^dag: rotation by -theta
                givens(fD, fE, cs.x, ss);
                givens(lD, lE, cs.x, ss);
                shp[rD] = fD;
                shp[iE] = fE;
                shl[rD] = lD;
                shl[iE] = lE;
            }
            acc = wave_sum(acc);
            if ((threadIdx.x & 63) == 0) red[j - run.g0][threadIdx.x >> 6] = acc;
            __syncthreads();   // orders this gate's updates before the next gate
        }
        // fixed-order sum of the per-wave partials of every gate of the run
        for (int jl = threadIdx.x; jl < run.g1 - run.g0; jl += kRunThreads) {
            double r = 0.0;
#pragma unroll
            for (int w = 0; w < kRunThreads / 64; ++w) r += red[jl][w];
            s.part_g[size_t(run.g0 + jl) * s.gstride + o] = r;
        }
        lds_to_global<EPT>(s.phi, shp, run, o_dep, half, T);
        lds_to_global<EPT>(s.lam, shl, run, o_dep, half, T);
        if (next >= total) break;
        id = next;
    }
}

// ------------------------------------------------ fused Pauli-rotation runs

// A run of consecutive rotations exp(-i phi/2 P(x, z)) whose flip masks all
// lie in the tile's inner bits: one block per (state, tile), the tile of 2^m
// amplitudes (outer bits fixed) staged in LDS, every rotation applied there
// (pairs (r, r ^ x_r), or a phase when x = 0), written back once.  The sign
// (-1)^{|b & z|} splits into the tile's outer part and the r-space part.
__device__ __forceinline__ uint32_t rot_index(const RunDesc& run, uint32_t o_dep, uint32_t e) {
    return o_dep | (run.contiguous ? e : pdep32(e, run.inner));
}

template <int EPT>
__device__ __forceinline__ void rot_load(double2* __restrict__ dst, const double2* __restrict__ src,
                                         const RunDesc& run, uint32_t o_dep, uint32_t T) {
    double2 v[EPT];
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
        const uint32_t e = threadIdx.x + k * kRunThreads;
        if (e < T) v[k] = nt_load(&src[rot_index(run, o_dep, e)]);
    }
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
        const uint32_t e = threadIdx.x + k * kRunThreads;
        if (e < T) dst[e] = v[k];
    }
}

template <int EPT>
__device__ __forceinline__ void rot_store(double2* __restrict__ dst, const double2* __restrict__ src,
                                          const RunDesc& run, uint32_t o_dep, uint32_t T) {
    double2 v[EPT];
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
        const uint32_t e = threadIdx.x + k * kRunThreads;
        if (e < T) v[k] = src[e];
    }
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
        const uint32_t e = threadIdx.x + k * kRunThreads;
        if (e < T) nt_store(&dst[rot_index(run, o_dep, e)], v[k]);
    }
}

// exp(-i phi/2 P) (s = sin(phi/2)) or its inverse (s < 0) on the LDS tile.
__device__ __forceinline__ void rot_tile(double2* __restrict__ sh, const TileGate& t, uint32_t T,
                                         double c, double s) {
    if (t.xr == 0) {
        for (uint32_t e = threadIdx.x; e < T; e += kRunThreads) {
            const double ss = s * parity_sign(e & t.pdr);
            const double2 a = sh[e];
            sh[e] = make_double2(c * a.x + ss * a.y, c * a.y - ss * a.x);
        }
        return;
    }
    const uint32_t low = t.xr & (~t.xr + 1u);
    const double2 f = minus_i_times_i_pow(int(t.chr));
    for (uint32_t p = threadIdx.x; p < (T >> 1); p += kRunThreads) {
        const uint32_t r0 = uint32_t(insert_zeros(p, low)), r1 = r0 ^ t.xr;
        const double2 a0 = sh[r0], a1 = sh[r1];
        const double s0 = s * parity_sign(r1 & t.pdr), s1 = s * parity_sign(r0 & t.pdr);
        const double2 t0 = cmul(f, a1), t1 = cmul(f, a0);
        sh[r0] = make_double2(c * a0.x + s0 * t0.x, c * a0.y + s0 * t0.y);
        sh[r1] = make_double2(c * a1.x + s1 * t1.x, c * a1.y + s1 * t1.y);
    }
}

template <int EPT>
__global__ void __launch_bounds__(kRunThreads) k_rot_fwd(const StateDesc* __restrict__ sd, RunDesc run,
                                                         const TileGate* __restrict__ tg, int total) {
    extern __shared__ double2 sh[];
    const uint32_t T = 1u << run.m;
    const int id = blockIdx.x;
    if (id >= total) return;
    const StateDesc& s = sd[id / run.ntiles];
    const uint32_t o_dep = pdep32(id % run.ntiles, run.outer);
    rot_load<EPT>(sh, s.phi, run, o_dep, T);
    __syncthreads();
    for (int j = run.g0; j < run.g1; ++j) {
        const TileGate t = tg[j - run.g0];
        const double2 cs = s.cs[j];
        rot_tile(sh, t, T, cs.x, cs.y * parity_sign(o_dep & t.chain_out));
        __syncthreads();
    }
    rot_store<EPT>(s.phi, sh, run, o_dep, T);
}

// The reverse sweep of a rotation run on phi and lambda: per gate the
// partial of Im <lambda|P phi> over the tile, then the inverse rotation.
template <int EPT>
__global__ void __launch_bounds__(kRunThreads) k_rot_adj(const StateDesc* __restrict__ sd, RunDesc run,
                                                         const TileGate* __restrict__ tg, int total) {
    extern __shared__ double2 sh[];
    __shared__ double red[kMaxRunGates][kRunThreads / 64];
    const uint32_t T = 1u << run.m;
    double2* shp = sh;
    double2* shl = sh + T;
    const int id = blockIdx.x;
    if (id >= total) return;
    const StateDesc& s = sd[id / run.ntiles];
    const int o = id % run.ntiles;
    const uint32_t o_dep = pdep32(o, run.outer);
    rot_load<EPT>(shp, s.phi, run, o_dep, T);
    rot_load<EPT>(shl, s.lam, run, o_dep, T);
    __syncthreads();
    for (int j = run.g1 - 1; j >= run.g0; --j) {
        const TileGate t = tg[j - run.g0];
        const double2 cs = s.cs[j];
        const double so = parity_sign(o_dep & t.chain_out);
        double acc = 0.0;
        if (t.xr == 0) {
            for (uint32_t e = threadIdx.x; e < T; e += kRunThreads) {
                const double sg = so * parity_sign(e & t.pdr);
                const double2 f = shp[e], l = shl[e];
                acc += sg * (l.x * f.y - l.y * f.x);   // Im(conj(l) (P phi)[b])
            }
        } else {
            const uint32_t low = t.xr & (~t.xr + 1u);
            const int y = int(t.chr);
            const double2 iy = (y == 0) ? make_double2(1, 0)
                             : (y == 1) ? make_double2(0, 1)
                             : (y == 2) ? make_double2(-1, 0) : make_double2(0, -1);
            for (uint32_t p = threadIdx.x; p < (T >> 1); p += kRunThreads) {
                const uint32_t r0 = uint32_t(insert_zeros(p, low)), r1 = r0 ^ t.xr;
                const double2 f0 = shp[r0], f1 = shp[r1], l0 = shl[r0], l1 = shl[r1];
                // (P phi)[b] = i^y sigma(b') phi[b'],  (P phi)[b'] = i^y sigma(b) phi[b]
                const double2 p0 = cmul(iy, f1), p1 = cmul(iy, f0);
                const double s0 = so * parity_sign(r1 & t.pdr), s1 = so * parity_sign(r0 & t.pdr);
                acc += s0 * (l0.x * p0.y - l0.y * p0.x) + s1 * (l1.x * p1.y - l1.y * p1.x);
            }
        }
        __syncthreads();   // every partial read this gate's inputs before they change
        rot_tile(shp, t, T, cs.x, -cs.y * so);
        rot_tile(shl, t, T, cs.x, -cs.y * so);
        acc = wave_sum(acc);
        if ((threadIdx.x & 63) == 0) red[j - run.g0][threadIdx.x >> 6] = acc;
        __syncthreads();
    }
    for (int jl = threadIdx.x; jl < run.g1 - run.g0; jl += kRunThreads) {
        double r = 0.0;
#pragma unroll
        for (int w = 0; w < kRunThreads / 64; ++w) r += red[jl][w];
        s.part_g[size_t(run.g0 + jl) * s.gstride + o] = r;
    }
    rot_store<EPT>(s.phi, shp, run, o_dep, T);
    rot_store<EPT>(s.lam, shl, run, o_dep, T);
}

// ------------------------------------------------------------ launchers

void launch_angles(const StateDesc* sd, int count, int M, hipStream_t st) {
    if (M <= 0) return;
    hipLaunchKernelGGL(k_angles, dim3(unsigned((M + kBlock - 1) / kBlock), count), dim3(kBlock), 0,
                       st, sd);
}

void launch_hf(const StateDesc* sd, int count, uint64_t N, hipStream_t st) {
    hipLaunchKernelGGL(k_hf, dim3(blocks_for(N), count), dim3(kBlock), 0, st, sd, N);
}

void launch_fill_zero(double2* p, uint64_t n, hipStream_t st) {
    hipLaunchKernelGGL(k_fill_zero, dim3(blocks_for(n)), dim3(kBlock), 0, st, p, n);
}

void launch_exc(const StateDesc* sd, int count, int j, uint64_t npairs, hipStream_t st) {
    hipLaunchKernelGGL(k_exc, dim3(blocks_for(npairs), count), dim3(kBlock), 0, st, sd, j, npairs);
}

void launch_pauli(const StateDesc* sd, int count, int j, uint64_t N, hipStream_t st) {
    hipLaunchKernelGGL(k_pauli, dim3(blocks_for(N >> 1), count), dim3(kBlock), 0, st, sd, j, N);
}

void launch_adj_exc(const StateDesc* sd, int count, int j, uint64_t npairs, int nblk,
                    hipStream_t st) {
    hipLaunchKernelGGL(k_adj_exc, dim3(nblk, count), dim3(kBlock), 0, st, sd, j, npairs);
}

void launch_adj_pauli(const StateDesc* sd, int count, int j, uint64_t N, int nblk,
                      hipStream_t st) {
    hipLaunchKernelGGL(k_adj_pauli, dim3(nblk, count), dim3(kBlock), 0, st, sd, j, N);
}

void launch_param_grad(const int64_t* start, const int64_t* gate, const double* coef, const double* raw,
                       double* g, int64_t P, hipStream_t st) {
    if (P <= 0) return;
    hipLaunchKernelGGL(k_param_grad, dim3(unsigned((P + kBlock - 1) / kBlock)), dim3(kBlock), 0, st, start, gate,
                       coef, raw, g, P);
}

void launch_reduce_e(const StateDesc* sd, int count, int nblk, hipStream_t st) {
    hipLaunchKernelGGL(k_reduce_e, dim3(1, count), dim3(kBlock), 0, st, sd, nblk);
}

void launch_reduce_g(const StateDesc* sd, int count, int M, const int32_t* cnt, int cnt_uniform,
                     hipStream_t st) {
    if (M <= 0) return;
    hipLaunchKernelGGL(k_reduce_g, dim3((M + 3) / 4, count), dim3(256), 0, st, sd, cnt, cnt_uniform, M);
}

static size_t run_lds(const RunDesc& run, int vectors) {
    return (size_t(2) << run.m) * sizeof(double2) * vectors;
}

static int g_cus = 0;

static int device_cus() {
    if (g_cus == 0) {
        int dev = 0, cus = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess)
            g_cus = cus;
        if (g_cus <= 0) g_cus = 256;
    }
    return g_cus;
}

// Grid of a run launch.  The kernels can walk several tiles per block with
// the next tile prefetched into registers; measured on the 20-qubit batch
// this was 10-20% slower than one tile per block (the hardware already
// overlaps the load, gate-chain and store phases of co-resident blocks), so
// every (state, tile) pair gets its own block unless `persistent` is set.
static bool g_persistent = false;

static int run_grid(size_t lds, int total) {
    if (!g_persistent) return total;
    const size_t per_cu = std::max<size_t>(1, std::min<size_t>(4, (160u << 10) / (lds + 8192)));
    return int(std::max<int64_t>(1, std::min<int64_t>(total, int64_t(per_cu) * device_cus())));
}

#define VQE_RUN_DISPATCH(KERNEL, VEC)                                                           \
    do {                                                                                        \
        const uint32_t T = 2u << run.m;                                                         \
        const int ept = int((T + kRunThreads - 1) / kRunThreads);                              \
        const int total = run.ntiles * count;                                                   \
        const size_t lds = run_lds(run, VEC);                                                   \
        const dim3 grid(run_grid(lds, total)), block(kRunThreads);                             \
        if (ept <= 1) hipLaunchKernelGGL(KERNEL<1>, grid, block, lds, st, sd, run, tg, total);   \
        else if (ept <= 2) hipLaunchKernelGGL(KERNEL<2>, grid, block, lds, st, sd, run, tg, total); \
        else if (ept <= 4) hipLaunchKernelGGL(KERNEL<4>, grid, block, lds, st, sd, run, tg, total); \
        else if (ept <= 8) hipLaunchKernelGGL(KERNEL<8>, grid, block, lds, st, sd, run, tg, total); \
        else if (ept <= 16) hipLaunchKernelGGL(KERNEL<16>, grid, block, lds, st, sd, run, tg, total); \
        else hipLaunchKernelGGL(KERNEL<32>, grid, block, lds, st, sd, run, tg, total);           \
    } while (0)

#define VQE_ROT_DISPATCH(KERNEL, VEC)                                                           \
    do {                                                                                        \
        const uint32_t T = 1u << run.m;                                                         \
        const int ept = int((T + kRunThreads - 1) / kRunThreads);                              \
        const int total = run.ntiles * count;                                                   \
        const size_t lds = size_t(T) * sizeof(double2) * VEC;                                  \
        const dim3 grid(total), block(kRunThreads);                                             \
        if (ept <= 1) hipLaunchKernelGGL(KERNEL<1>, grid, block, lds, st, sd, run, tg, total);   \
        else if (ept <= 2) hipLaunchKernelGGL(KERNEL<2>, grid, block, lds, st, sd, run, tg, total); \
        else if (ept <= 4) hipLaunchKernelGGL(KERNEL<4>, grid, block, lds, st, sd, run, tg, total); \
        else if (ept <= 8) hipLaunchKernelGGL(KERNEL<8>, grid, block, lds, st, sd, run, tg, total); \
        else if (ept <= 16) hipLaunchKernelGGL(KERNEL<16>, grid, block, lds, st, sd, run, tg, total); \
        else hipLaunchKernelGGL(KERNEL<32>, grid, block, lds, st, sd, run, tg, total);           \
    } while (0)

void launch_run_fwd(const StateDesc* sd, int count, const RunDesc& run, const TileGate* tg,
                    hipStream_t st) {
    if (run.kind == 1)
        VQE_ROT_DISPATCH(k_rot_fwd, 1);
    else
        VQE_RUN_DISPATCH(k_run_fwd, 1);
}

void launch_run_adj(const StateDesc* sd, int count, const RunDesc& run, const TileGate* tg,
                    hipStream_t st) {
    if (run.kind == 1)
        VQE_ROT_DISPATCH(k_rot_adj, 2);
    else
        VQE_RUN_DISPATCH(k_run_adj, 2);
}

// Largest tile (elements = 2^(m+1)) a run kernel may be asked for: the
// register prefetch holds at most 32 elements per thread and vector.
int max_run_m() { return 13; }

// Large dynamic LDS (above 64 KiB) has to be enabled per kernel once.
int enable_large_lds(size_t bytes) {
    hipError_t e = hipSuccess;
    auto set = [&](const void* f) {
        hipError_t r = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, int(bytes));
        if (r != hipSuccess) e = r;
    };
    set(reinterpret_cast<const void*>(&k_run_fwd<1>));
    set(reinterpret_cast<const void*>(&k_run_fwd<2>));
    set(reinterpret_cast<const void*>(&k_run_fwd<4>));
    set(reinterpret_cast<const void*>(&k_run_fwd<8>));
    set(reinterpret_cast<const void*>(&k_run_fwd<16>));
    set(reinterpret_cast<const void*>(&k_run_fwd<32>));
    set(reinterpret_cast<const void*>(&k_run_adj<1>));
    set(reinterpret_cast<const void*>(&k_run_adj<2>));
    set(reinterpret_cast<const void*>(&k_run_adj<4>));
    set(reinterpret_cast<const void*>(&k_run_adj<8>));
    set(reinterpret_cast<const void*>(&k_run_adj<16>));
    set(reinterpret_cast<const void*>(&k_run_adj<32>));
    set(reinterpret_cast<const void*>(&k_rot_fwd<1>));
    set(reinterpret_cast<const void*>(&k_rot_fwd<2>));
    set(reinterpret_cast<const void*>(&k_rot_fwd<4>));
    set(reinterpret_cast<const void*>(&k_rot_fwd<8>));
    set(reinterpret_cast<const void*>(&k_rot_fwd<16>));
    set(reinterpret_cast<const void*>(&k_rot_fwd<32>));
    set(reinterpret_cast<const void*>(&k_rot_adj<1>));
    set(reinterpret_cast<const void*>(&k_rot_adj<2>));
    set(reinterpret_cast<const void*>(&k_rot_adj<4>));
    set(reinterpret_cast<const void*>(&k_rot_adj<8>));
    set(reinterpret_cast<const void*>(&k_rot_adj<16>));
    set(reinterpret_cast<const void*>(&k_rot_adj<32>));
    return e == hipSuccess ? 0 : -1;
}

}  // namespace vqe
