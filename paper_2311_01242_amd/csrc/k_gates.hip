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
    const uint64_t hf = (uint64_t(1) << s.ne) - 1;
    for (uint64_t b = blockIdx.x * uint64_t(blockDim.x) + threadIdx.x; b < N;
         b += uint64_t(gridDim.x) * blockDim.x)
        s.phi[b] = make_double2(b == hf ? 1.0 : 0.0, 0.0);
}

__global__ void k_fill_zero(double2* __restrict__ p, uint64_t n) {
    for (uint64_t i = blockIdx.x * uint64_t(blockDim.x) + threadIdx.x; i < n;
         i += uint64_t(gridDim.x) * blockDim.x)
        p[i] = make_double2(0.0, 0.0);
}

// Pair update of an excitation: D' = c D - ss E, E' = c E + ss D (ss = s * sin).
__device__ __forceinline__ void givens(double2& d, double2& e, double c, double ss) {
    const double2 pd = d, pe = e;
    d = make_double2(c * pd.x - ss * pe.x, c * pd.y - ss * pe.y);
    e = make_double2(c * pe.x + ss * pd.x, c * pe.y + ss * pd.y);
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

__global__ void __launch_bounds__(kBlock) k_reduce_g(const StateDesc* __restrict__ sd,
                                                     const int32_t* __restrict__ cnt,
                                                     int cnt_uniform) {
    __shared__ double red[kBlock / 64];
    const StateDesc& s = sd[blockIdx.y];
    const int j = blockIdx.x;
    const int nb = cnt ? cnt[j] : cnt_uniform;
    const double* part = s.part_g + size_t(j) * s.gstride;
    double acc = 0.0;
    for (int b = threadIdx.x; b < nb; b += kBlock) acc += part[b];
    const double r = block_sum(acc, red);
    if (threadIdx.x == 0) s.out_g[j] = r;
}

// ------------------------------------------------------------ fused runs

__device__ __forceinline__ uint32_t tile_index(const RunDesc& run, uint32_t o_dep, uint32_t e,
                                               uint32_t half) {
    const uint32_t r = e & (half - 1);
    const uint32_t in = run.contiguous ? r : pdep32(r, run.inner);
    return o_dep | in | ((e >= half) ? run.key : 0u);
}

__global__ void __launch_bounds__(kBlock) k_run_fwd(const StateDesc* __restrict__ sd, RunDesc run,
                                                    const TileGate* __restrict__ tg) {
    extern __shared__ double2 sh[];
    const StateDesc& s = sd[blockIdx.y];
    const uint32_t o_dep = pdep32(blockIdx.x, run.outer);
    const uint32_t half = 1u << run.m, T = half << 1;
    double2* __restrict__ phi = s.phi;
    for (uint32_t e = threadIdx.x; e < T; e += kBlock) sh[e] = phi[tile_index(run, o_dep, e, half)];
    __syncthreads();
    for (int j = run.g0; j < run.g1; ++j) {
        const TileGate t = tg[j - run.g0];
        const double2 cs = s.cs[j];
        const double base = t.csign * parity_sign(o_dep & t.chain_out) * cs.y;
        const uint32_t np = half >> __popc(t.xr);
        for (uint32_t p = threadIdx.x; p < np; p += kBlock) {
            const uint32_t rD = uint32_t(insert_zeros(p, t.xr)) | t.pdr;
            const uint32_t iE = half + (rD ^ t.xr);
            givens(sh[rD], sh[iE], cs.x, base * parity_sign(rD & t.chr));
        }
        __syncthreads();
    }
    for (uint32_t e = threadIdx.x; e < T; e += kBlock) phi[tile_index(run, o_dep, e, half)] = sh[e];
}

__global__ void __launch_bounds__(kBlock) k_run_adj(const StateDesc* __restrict__ sd, RunDesc run,
                                                    const TileGate* __restrict__ tg) {
    extern __shared__ double2 sh[];
    __shared__ double red[kBlock / 64];
    const StateDesc& s = sd[blockIdx.y];
    const uint32_t o_dep = pdep32(blockIdx.x, run.outer);
    const uint32_t half = 1u << run.m, T = half << 1;
    double2* __restrict__ phi = s.phi;
    double2* __restrict__ lam = s.lam;
    double2* shp = sh;
    double2* shl = sh + T;
    for (uint32_t e = threadIdx.x; e < T; e += kBlock) {
        const uint32_t gi = tile_index(run, o_dep, e, half);
        shp[e] = phi[gi];
        shl[e] = lam[gi];
    }
    __syncthreads();
    for (int j = run.g1 - 1; j >= run.g0; --j) {
        const TileGate t = tg[j - run.g0];
        const double2 cs = s.cs[j];
        const double base = t.csign * parity_sign(o_dep & t.chain_out);
        const uint32_t np = half >> __popc(t.xr);
        double acc = 0.0;
        for (uint32_t p = threadIdx.x; p < np; p += kBlock) {
            const uint32_t rD = uint32_t(insert_zeros(p, t.xr)) | t.pdr;
            const uint32_t iE = half + (rD ^ t.xr);
            const double sg = base * parity_sign(rD & t.chr);
            double2 fD = shp[rD], fE = shp[iE], lD = shl[rD], lE = shl[iE];
            acc += sg * ((lE.x * fD.x + lE.y * fD.y) - (lD.x * fE.x + lD.y * fE.y));
            const double ss = -sg * cs.y;
            givens(fD, fE, cs.x, ss);
            givens(lD, lE, cs.x, ss);
            shp[rD] = fD;
            shp[iE] = fE;
            shl[rD] = lD;
            shl[iE] = lE;
        }
        // block_sum's barriers also order this gate's updates before the next gate
        const double r = block_sum(acc, red);
        if (threadIdx.x == 0) s.part_g[size_t(j) * s.gstride + blockIdx.x] = r;
    }
    __syncthreads();
    for (uint32_t e = threadIdx.x; e < T; e += kBlock) {
        const uint32_t gi = tile_index(run, o_dep, e, half);
        phi[gi] = shp[e];
        lam[gi] = shl[e];
    }
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

void launch_reduce_e(const StateDesc* sd, int count, int nblk, hipStream_t st) {
    hipLaunchKernelGGL(k_reduce_e, dim3(1, count), dim3(kBlock), 0, st, sd, nblk);
}

void launch_reduce_g(const StateDesc* sd, int count, int M, const int32_t* cnt, int cnt_uniform,
                     hipStream_t st) {
    if (M <= 0) return;
    hipLaunchKernelGGL(k_reduce_g, dim3(M, count), dim3(kBlock), 0, st, sd, cnt, cnt_uniform);
}

static size_t run_lds(const RunDesc& run, int vectors) {
    return (size_t(2) << run.m) * sizeof(double2) * vectors;
}

void launch_run_fwd(const StateDesc* sd, int count, const RunDesc& run, const TileGate* tg,
                    hipStream_t st) {
    hipLaunchKernelGGL(k_run_fwd, dim3(run.ntiles, count), dim3(kBlock), run_lds(run, 1), st, sd,
                       run, tg);
}

void launch_run_adj(const StateDesc* sd, int count, const RunDesc& run, const TileGate* tg,
                    hipStream_t st) {
    hipLaunchKernelGGL(k_run_adj, dim3(run.ntiles, count), dim3(kBlock), run_lds(run, 2), st, sd,
                       run, tg);
}

// Large dynamic LDS (above 64 KiB) has to be enabled per kernel once.
int enable_large_lds(size_t bytes) {
    hipError_t e1 = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_run_fwd),
                                        hipFuncAttributeMaxDynamicSharedMemorySize, int(bytes));
    hipError_t e2 = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_run_adj),
                                        hipFuncAttributeMaxDynamicSharedMemorySize, int(bytes));
    return (e1 == hipSuccess && e2 == hipSuccess) ? 0 : -1;
}

}  // namespace vqe
