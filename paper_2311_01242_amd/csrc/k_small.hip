// Whole-state evaluation in one workgroup for programs that conserve the
// number of set qubits (Sec. 2.1.1, Eq. 1 and its gradient): the pUCCD
// ansatz in the hard-core-boson form (qubit p = spatial orbital p occupied by
// a pair; its pair moves change the pair count of no state) conserves the
// number of pairs k, so a state prepared from the reference lives on the
// C(n, k) strings of k set qubits.  When that sector is small, a state's
// amplitudes on it (ranked in increasing string order) fit one workgroup's
// LDS, and the forward pass, the H-apply and the reverse sweep each run in
// one workgroup per state.  Everything a phase reads more than once (the
// strings, the rank table, the gates with their angles, the Hamiltonian's
// tables) is staged in LDS first with wide loads, so the per-gate and
// per-term steps touch no memory outside the workgroup.
//
// A gate pairs D (its annihilated qubits set, its created ones clear) with
// E = D ^ x by a Givens rotation whose sign is csign (-1)^{|D & chain|}; the
// thread holding D's rank updates both amplitudes, the pairs of one gate are
// disjoint, and one barrier separates gates.  lambda = H phi is formed on the
// sector only: output string b takes, for every subgroup of every x-group of
// H, the subgroup's term at b times phi at b ^ x when that string is in the
// sector (E and the gradient need lambda on the sector only, as phi and A_j
// phi live there).  The H-apply splits each string's subgroups over several
// threads when the workgroup has more threads than the sector has strings,
// and adds the parts in a fixed order.  The H-apply writes the energy and the
// reverse sweep the per-gate gradient sums directly (no separate reduction
// launches).  Amplitudes are real (double) or complex (double2), as the rest
// of the sector paths: the pair moves are real rotations and H is a real
// matrix.
#include <mutex>

#include "device_common.h"

namespace vqe {

constexpr int kSmallThreads = 256;   // forward pass and reverse sweep
constexpr int kSmallHxThreads = 1024;
constexpr int kSmallMaxSlices = 8;   // threads per string in the H-apply

static_assert(sizeof(GroupDesc) == 16 && sizeof(SubDesc) == 8, "descriptor sizes staged in LDS");

// A gate as the kernels use it: masks, sign, and its (cos, sin).
struct SmallGate {
    uint32_t x, pd, chain;
    float csign;
    double c, s;
};
static_assert(sizeof(SmallGate) == 32, "SmallGate layout");

__host__ __device__ inline size_t small_r16(size_t v) { return (v + 15) & ~size_t(15); }

// Threads per string in the H-apply.
__host__ __device__ inline int small_slices(int nsec) {
    const int s = kSmallHxThreads / (nsec > 0 ? nsec : 1);
    return s < 1 ? 1 : (s > kSmallMaxSlices ? kSmallMaxSlices : s);
}

// Copy nbytes (even) from global memory to LDS, both 16-byte aligned: 16-byte
// pieces with four loads per thread issued before their stores, then the
// remainder in 2-byte pieces.
template <int NT>
__device__ __forceinline__ void small_copy(void* dst, const void* src, size_t nbytes) {
    const uint4* s4 = static_cast<const uint4*>(src);
    uint4* d4 = static_cast<uint4*>(dst);
    const int n16 = int(nbytes >> 4);
    int t = threadIdx.x;
    for (; t + 3 * NT < n16; t += 4 * NT) {
        const uint4 a = s4[t], b = s4[t + NT], c = s4[t + 2 * NT], d = s4[t + 3 * NT];
        d4[t] = a;
        d4[t + NT] = b;
        d4[t + 2 * NT] = c;
        d4[t + 3 * NT] = d;
    }
    for (; t < n16; t += NT) d4[t] = s4[t];
    const int rem = int(nbytes & 15) >> 1;
    if (int(threadIdx.x) < rem) {
        const size_t o = (size_t(n16) << 3) + threadIdx.x;   // in 2-byte units
        static_cast<uint16_t*>(dst)[o] = static_cast<const uint16_t*>(src)[o];
    }
}

// Fixed-order workgroup total of NT threads: wave totals, then every thread
// adds them in wave order.  Contains barriers: every thread calls it.
template <int NT>
__device__ __forceinline__ double small_block_total(double v, double* red) {
    v = wave_total(v);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double r = 0.0;
#pragma unroll
    for (int i = 0; i < NT / 64; ++i) r += red[i];
    __syncthreads();
    return r;
}

// LDS layout (byte offsets, every region 16-byte aligned): amplitude
// vectors, H-apply partial sums, gates, Hamiltonian, rank table, strings.
struct SmallLayout {
    size_t vec, part, gates, ham, rank, str, total;
};

enum SmallPhase { kSmallFwd = 0, kSmallHx = 1, kSmallAdj = 2 };

__host__ __device__ inline SmallLayout small_layout(const SmallSpace& sp, int phase) {
    SmallLayout l;
    const size_t vbytes = size_t(sp.vbytes) * size_t(sp.nsec);   // one vector's amplitudes
    l.vec = 0;
    l.part = l.vec + (phase == kSmallAdj ? 2 : 1) * small_r16(vbytes);   // phi [, lambda]
    const int sl = small_slices(sp.nsec);
    l.gates = l.part + (phase == kSmallHx && sl > 1 ? small_r16(size_t(sl) * vbytes) : 0);
    l.ham = l.gates + (phase == kSmallHx ? 0 : sizeof(SmallGate) * size_t(sp.M));
    l.rank = l.ham + (phase == kSmallHx ? small_r16(size_t(sp.ham_lds)) : 0);
    l.str = l.rank + small_r16(2 * (size_t(1) << sp.n));
    l.total = l.str + small_r16(4 * size_t(sp.nsec));
    return l;
}

// Stage the sector's strings and the rank table into LDS.
template <int NT>
__device__ __forceinline__ void small_stage_space(const SmallSpace& sp, uint32_t* str, int16_t* rank) {
    small_copy<NT>(str, sp.str, 4 * size_t(sp.nsec));
    small_copy<NT>(rank, sp.rank, 2 * (size_t(1) << sp.n));
}

// Pair update of gate g on LDS amplitudes: psi <- U psi.
template <typename V>
__device__ __forceinline__ void small_gate(const SmallGate& g, const uint32_t* str, const int16_t* rank, int nsec,
                                           V* psi) {
    for (int t = threadIdx.x; t < nsec; t += kSmallThreads) {
        const uint32_t d = str[t];
        if ((d & g.x) != g.pd) continue;
        const int re = rank[d ^ g.x];
        const double ss = double(g.csign) * parity_sign(d & g.chain) * g.s;
        V a = psi[t], b = psi[re];
        givens(a, b, g.c, ss);
        psi[t] = a;
        psi[re] = b;
    }
}

// Forward pass: |ref> then U_M ... U_1; phi and the gates' (cos, sin) out.
template <typename V>
__global__ void __launch_bounds__(kSmallThreads) k_small_fwd(const StateDesc* __restrict__ sd, SmallSpace sp) {
    extern __shared__ __align__(16) unsigned char smem[];
    const SmallLayout L = small_layout(sp, kSmallFwd);
    const StateDesc& s = sd[blockIdx.y];
    V* psi = reinterpret_cast<V*>(smem + L.vec);
    SmallGate* gs = reinterpret_cast<SmallGate*>(smem + L.gates);
    uint32_t* str = reinterpret_cast<uint32_t*>(smem + L.str);
    int16_t* rank = reinterpret_cast<int16_t*>(smem + L.rank);
    small_stage_space<kSmallThreads>(sp, str, rank);
    for (int t = threadIdx.x; t < sp.nsec; t += kSmallThreads)
        psi[t] = t == sp.ref_rank ? vunit(V{}) : vzero<V>();
    for (int j = threadIdx.x; j < s.M; j += kSmallThreads) {
        const GateDesc g = s.gates[j];
        double sn, c;
        sincos(g.scale * s.theta[g.param], &sn, &c);
        s.cs[j] = make_double2(c, sn);
        gs[j] = SmallGate{g.x, g.pd, g.chain, float(g.csign), c, sn};
    }
    __syncthreads();
    for (int j = 0; j < s.M; ++j) {
        small_gate<V>(gs[j], str, rank, sp.nsec, psi);
        __syncthreads();
    }
    V* phi = reinterpret_cast<V*>(s.phi);
    for (int t = threadIdx.x; t < sp.nsec; t += kSmallThreads) phi[t] = psi[t];
}

// lambda = H phi on the sector, and E = Re <phi|lambda> into out_e.
template <typename V>
__global__ void __launch_bounds__(kSmallHxThreads) k_small_hx(const StateDesc* __restrict__ sd, SmallSpace sp) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double red[kSmallHxThreads / 64];
    const SmallLayout L = small_layout(sp, kSmallHx);
    const StateDesc& s = sd[blockIdx.y];
    const int nsec = sp.nsec;
    V* psi = reinterpret_cast<V*>(smem + L.vec);
    V* part = reinterpret_cast<V*>(smem + L.part);
    V* lam = reinterpret_cast<V*>(s.lam);
    uint32_t* str = reinterpret_cast<uint32_t*>(smem + L.str);
    int16_t* rank = reinterpret_cast<int16_t*>(smem + L.rank);
    small_stage_space<kSmallHxThreads>(sp, str, rank);
    small_copy<kSmallHxThreads>(psi, s.phi, sizeof(V) * size_t(nsec));
    // the state's own Hamiltonian fits the staged region when the launch has one
    const bool hlds = sp.ham_lds > 0 && small_ham_bytes(s.G, s.nsub, s.ntab) <= size_t(sp.ham_lds);
    double e = 0.0;
    if (hlds) {
        GroupDesc* groups = reinterpret_cast<GroupDesc*>(smem + L.ham);
        double* tabs = reinterpret_cast<double*>(smem + L.ham + 16 * size_t(s.G));
        SubDesc* subs = reinterpret_cast<SubDesc*>(reinterpret_cast<unsigned char*>(tabs) +
                                                   small_r16(8 * size_t(s.ntab)));
        int32_t* sgrp = reinterpret_cast<int32_t*>(reinterpret_cast<unsigned char*>(subs) +
                                                   small_r16(8 * size_t(s.nsub)));
        small_copy<kSmallHxThreads>(groups, s.groups, 16 * size_t(s.G));
        small_copy<kSmallHxThreads>(tabs, s.tabs, 8 * size_t(s.ntab));
        small_copy<kSmallHxThreads>(subs, s.subs, 8 * size_t(s.nsub));
        for (int gi = threadIdx.x; gi < s.G; gi += kSmallHxThreads) {
            const GroupDesc gd = s.groups[gi];
            for (int si = gd.sub_begin; si < gd.sub_end; ++si) sgrp[si] = gi;
        }
        __syncthreads();
        // thread (slice q, string r) takes subgroups q, q + sl, q + 2 sl, ...
        const int sl = small_slices(nsec);
        for (int i = threadIdx.x; i < sl * nsec; i += kSmallHxThreads) {
            const int r = i % nsec, q = i / nsec;
            const uint32_t b = str[r];
            V acc = vzero<V>();
            for (int si = q; si < s.nsub; si += sl) {
                const GroupDesc gd = groups[sgrp[si]];
                const uint32_t p = b ^ gd.x;
                if (p >= (1u << sp.n)) continue;
                const int rp = rank[p];
                if (rp < 0) continue;
                const SubDesc sub = subs[si];
                const double t = tabs[sub.tab + pext_pos(b, gd.pos)];
                const double d = (__popc(b & sub.w) & 1) ? -t : t;
                axpy(acc, d, psi[rp]);
            }
            if (sl > 1) {
                part[size_t(q) * nsec + r] = acc;
            } else {
                lam[r] = acc;
                e += redot(psi[r], acc);
            }
        }
        if (sl > 1) {
            __syncthreads();
            for (int r = threadIdx.x; r < nsec; r += kSmallHxThreads) {
                V acc = vzero<V>();
                for (int q = 0; q < sl; ++q) vadd(acc, part[size_t(q) * nsec + r]);
                lam[r] = acc;
                e += redot(psi[r], acc);
            }
        }
    } else {
        __syncthreads();
        for (int r = threadIdx.x; r < nsec; r += kSmallHxThreads) {
            const uint32_t b = str[r];
            V acc = vzero<V>();
            for (int gi = 0; gi < s.G; ++gi) {
                const GroupDesc gd = s.groups[gi];
                const uint32_t p = b ^ gd.x;
                if (p >= (1u << sp.n)) continue;
                const int rp = rank[p];
                if (rp < 0) continue;
                axpy(acc, group_coeff(gd, s.subs, s.tabs, b), psi[rp]);
            }
            lam[r] = acc;
            e += redot(psi[r], acc);
        }
    }
    const double tot = small_block_total<kSmallHxThreads>(e, red);
    if (threadIdx.x == 0) s.out_e[0] = tot;
}

// Reverse sweep: per gate (last first) each wave's part of Re <lambda|A_j phi>
// into LDS, then U_j^dag on phi and lambda in the same pass; the per-gate sums
// (waves added in fixed order) into out_g at the end.
template <typename V>
__global__ void __launch_bounds__(kSmallThreads) k_small_adj(const StateDesc* __restrict__ sd, SmallSpace sp) {
    constexpr int kWaves = kSmallThreads / 64;
    extern __shared__ __align__(16) unsigned char smem[];
    const SmallLayout L = small_layout(sp, kSmallAdj);
    const StateDesc& s = sd[blockIdx.y];
    V* psi = reinterpret_cast<V*>(smem + L.vec);
    V* lam = reinterpret_cast<V*>(smem + L.vec + small_r16(sizeof(V) * size_t(sp.nsec)));
    SmallGate* gs = reinterpret_cast<SmallGate*>(smem + L.gates);
    uint32_t* str = reinterpret_cast<uint32_t*>(smem + L.str);
    int16_t* rank = reinterpret_cast<int16_t*>(smem + L.rank);
    double* part = reinterpret_cast<double*>(smem + L.total);   // [M][waves] gradient partials
    small_stage_space<kSmallThreads>(sp, str, rank);
    small_copy<kSmallThreads>(psi, s.phi, sizeof(V) * size_t(sp.nsec));
    small_copy<kSmallThreads>(lam, s.lam, sizeof(V) * size_t(sp.nsec));
    for (int j = threadIdx.x; j < s.M; j += kSmallThreads) {
        const GateDesc g = s.gates[j];
        const double2 cs = s.cs[j];
        gs[j] = SmallGate{g.x, g.pd, g.chain, float(g.csign), cs.x, cs.y};
    }
    __syncthreads();
    const int w = threadIdx.x >> 6;
    for (int j = s.M - 1; j >= 0; --j) {
        const SmallGate g = gs[j];
        double acc = 0.0;
        for (int t = threadIdx.x; t < sp.nsec; t += kSmallThreads) {
            const uint32_t d = str[t];
            if ((d & g.x) != g.pd) continue;
            const int re = rank[d ^ g.x];
            const double sg = double(g.csign) * parity_sign(d & g.chain);
            V fD = psi[t], fE = psi[re], lD = lam[t], lE = lam[re];
            // A|D> = s|E>, A|E> = -s|D>: <lam|A phi> = s (lam_E^* phi_D - lam_D^* phi_E)
            acc += sg * (redot(lE, fD) - redot(lD, fE));
            const double ss = -sg * g.s;   // U^dag: rotation by -theta
            givens(fD, fE, g.c, ss);
            givens(lD, lE, g.c, ss);
            psi[t] = fD;
            psi[re] = fE;
            lam[t] = lD;
            lam[re] = lE;
        }
        acc = wave_total(acc);
        if ((threadIdx.x & 63) == 0) part[size_t(j) * kWaves + w] = acc;
        __syncthreads();
    }
    for (int j = threadIdx.x; j < s.M; j += kSmallThreads) {
        double r = 0.0;
#pragma unroll
        for (int i = 0; i < kWaves; ++i) r += part[size_t(j) * kWaves + i];
        s.out_g[j] = r;
    }
}

size_t small_lds(const SmallSpace& sp, int phase) {
    const size_t base = small_layout(sp, phase).total;
    return phase == kSmallAdj ? base + 8 * size_t(kSmallThreads / 64) * size_t(sp.M) : base;
}

// The launches' LDS (dynamic plus the H-apply's static reduction slots) must
// fit the CU's 160 KiB; beyond 64 KiB the kernels are allowed the whole of it
// (once).
int small_prepare(const SmallSpace& sp) {
    constexpr size_t kMax = size_t(160) << 10;
    size_t lds = 0;
    for (int ph = 0; ph < 3; ++ph) lds = std::max(lds, small_lds(sp, ph) + 8 * size_t(kSmallHxThreads / 64));
    if (lds > kMax) return 1;
    if (lds <= (64u << 10)) return 0;
    static std::once_flag once;
    static int rc = 0;
    std::call_once(once, [] {
        const void* fs[6] = {reinterpret_cast<const void*>(&k_small_fwd<double2>),
                             reinterpret_cast<const void*>(&k_small_hx<double2>),
                             reinterpret_cast<const void*>(&k_small_adj<double2>),
                             reinterpret_cast<const void*>(&k_small_fwd<double>),
                             reinterpret_cast<const void*>(&k_small_hx<double>),
                             reinterpret_cast<const void*>(&k_small_adj<double>)};
        for (const void* f : fs)
            if (hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, int(kMax)) != hipSuccess) rc = 1;
    });
    return rc;
}

template <typename V>
static void launch_small_t(int phase, const StateDesc* sd, int count, const SmallSpace& sp, hipStream_t st) {
    const size_t lds = small_lds(sp, phase);
    if (phase == kSmallFwd)
        hipLaunchKernelGGL(k_small_fwd<V>, dim3(1, count), dim3(kSmallThreads), lds, st, sd, sp);
    else if (phase == kSmallHx)
        hipLaunchKernelGGL(k_small_hx<V>, dim3(1, count), dim3(kSmallHxThreads), lds, st, sd, sp);
    else
        hipLaunchKernelGGL(k_small_adj<V>, dim3(1, count), dim3(kSmallThreads), lds, st, sd, sp);
}

void launch_small(int phase, const StateDesc* sd, int count, const SmallSpace& sp, hipStream_t st) {
    if (sp.vbytes == 8)
        launch_small_t<double>(phase, sd, count, sp, st);
    else
        launch_small_t<double2>(phase, sd, count, sp, st);
}

}  // namespace vqe
