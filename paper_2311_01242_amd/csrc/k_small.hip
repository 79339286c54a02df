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
// tables) is staged in LDS first, so the per-gate and per-term steps touch
// no memory outside the workgroup.
//
// A gate pairs D (its annihilated qubits set, its created ones clear) with
// E = D ^ x by a Givens rotation whose sign is csign (-1)^{|D & chain|}; the
// thread holding D's rank updates both amplitudes, the pairs of one gate are
// disjoint, and one barrier separates gates.  lambda = H phi is formed on the
// sector only: output string b takes, for every x-group of H, the group's
// coefficient at b times phi at b ^ x when that string is in the sector (E
// and the gradient need lambda on the sector only, as phi and A_j phi live
// there).  The H-apply writes the energy and the reverse sweep the per-gate
// gradient sums directly (no separate reduction launches).
#include <mutex>

#include "device_common.h"

namespace vqe {

constexpr int kSmallThreads = 256;
constexpr int kSmallWaves = kSmallThreads / 64;

static_assert(sizeof(GroupDesc) == 16 && sizeof(SubDesc) == 8, "descriptor sizes staged in LDS");

// A gate as the kernels use it: masks, sign, and its (cos, sin).
struct SmallGate {
    uint32_t x, pd, chain;
    float csign;
    double c, s;
};
static_assert(sizeof(SmallGate) == 32, "SmallGate layout");

// Fixed-order workgroup total: wave totals, then every thread adds them in
// wave order.  Contains barriers: every thread calls it.
__device__ __forceinline__ double small_block_total(double v, double* red) {
    v = wave_total(v);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double r = 0.0;
#pragma unroll
    for (int i = 0; i < kSmallWaves; ++i) r += red[i];
    __syncthreads();
    return r;
}

// Stage the sector's strings and the rank table into LDS.
__device__ __forceinline__ void small_stage_space(const SmallSpace& sp, uint32_t* str, int16_t* rank) {
    for (int t = threadIdx.x; t < sp.nsec; t += kSmallThreads) str[t] = sp.str[t];
    for (int t = threadIdx.x; t < (1 << sp.n); t += kSmallThreads) rank[t] = sp.rank[t];
}

// Pair update of gate g on LDS amplitudes: psi <- U psi (ssign = +1) or
// U^dag psi (ssign = -1).
__device__ __forceinline__ void small_gate(const SmallGate& g, double ssign, const uint32_t* str,
                                           const int16_t* rank, int nsec, double2* psi) {
    for (int t = threadIdx.x; t < nsec; t += kSmallThreads) {
        const uint32_t d = str[t];
        if ((d & g.x) != g.pd) continue;
        const int re = rank[d ^ g.x];
        const double ss = ssign * double(g.csign) * parity_sign(d & g.chain) * g.s;
        double2 a = psi[t], b = psi[re];
        givens(a, b, g.c, ss);
        psi[t] = a;
        psi[re] = b;
    }
}

// LDS layout (byte offsets, every region 8-byte aligned): amplitude vectors,
// gates, Hamiltonian (tables, groups, subgroups), strings, rank table.
struct SmallLayout {
    size_t vec, gates, ham, str, rank, total;
};

__host__ __device__ inline SmallLayout small_layout(const SmallSpace& sp, int vectors, bool gates, bool ham) {
    SmallLayout l;
    l.vec = 0;
    l.gates = l.vec + size_t(vectors) * 16 * size_t(sp.nsec);
    l.ham = l.gates + (gates ? sizeof(SmallGate) * size_t(sp.M) : 0);
    l.str = l.ham + (ham ? size_t(sp.ham_lds) : 0);
    l.rank = l.str + 4 * size_t(sp.nsec);
    l.total = l.rank + 2 * (size_t(1) << sp.n);
    l.total = (l.total + 7) & ~size_t(7);
    return l;
}

// Forward pass: |ref> then U_M ... U_1; phi and the gates' (cos, sin) out.
__global__ void __launch_bounds__(kSmallThreads) k_small_fwd(const StateDesc* __restrict__ sd, SmallSpace sp) {
    extern __shared__ __align__(16) unsigned char smem[];
    const SmallLayout L = small_layout(sp, 1, true, false);
    const StateDesc& s = sd[blockIdx.y];
    double2* psi = reinterpret_cast<double2*>(smem + L.vec);
    SmallGate* gs = reinterpret_cast<SmallGate*>(smem + L.gates);
    uint32_t* str = reinterpret_cast<uint32_t*>(smem + L.str);
    int16_t* rank = reinterpret_cast<int16_t*>(smem + L.rank);
    small_stage_space(sp, str, rank);
    for (int t = threadIdx.x; t < sp.nsec; t += kSmallThreads)
        psi[t] = make_double2(t == sp.ref_rank ? 1.0 : 0.0, 0.0);
    for (int j = threadIdx.x; j < s.M; j += kSmallThreads) {
        const GateDesc g = s.gates[j];
        double sn, c;
        sincos(g.scale * s.theta[g.param], &sn, &c);
        s.cs[j] = make_double2(c, sn);
        gs[j] = SmallGate{g.x, g.pd, g.chain, float(g.csign), c, sn};
    }
    __syncthreads();
    for (int j = 0; j < s.M; ++j) {
        small_gate(gs[j], 1.0, str, rank, sp.nsec, psi);
        __syncthreads();
    }
    for (int t = threadIdx.x; t < sp.nsec; t += kSmallThreads) s.phi[t] = psi[t];
}

// lambda = H phi on the sector, and E = Re <phi|lambda> into out_e.
__device__ __forceinline__ void small_hx_body(const StateDesc& s, const SmallSpace& sp, const GroupDesc* groups,
                                              const SubDesc* subs, const double* tabs, const uint32_t* str,
                                              const int16_t* rank, const double2* psi, double* red) {
    double e = 0.0;
    for (int t = threadIdx.x; t < sp.nsec; t += kSmallThreads) {
        const uint32_t b = str[t];
        double lr = 0.0, li = 0.0;
        for (int gi = 0; gi < s.G; ++gi) {
            const GroupDesc gd = groups[gi];
            const uint32_t p = b ^ gd.x;
            if (p >= (1u << sp.n)) continue;
            const int rp = rank[p];
            if (rp < 0) continue;
            const double d = group_coeff(gd, subs, tabs, b);
            const double2 f = psi[rp];
            lr += d * f.x;
            li += d * f.y;
        }
        s.lam[t] = make_double2(lr, li);
        e += psi[t].x * lr + psi[t].y * li;
    }
    const double tot = small_block_total(e, red);
    if (threadIdx.x == 0) s.out_e[0] = tot;
}

__global__ void __launch_bounds__(kSmallThreads) k_small_hx(const StateDesc* __restrict__ sd, SmallSpace sp) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double red[kSmallWaves];
    const SmallLayout L = small_layout(sp, 1, false, true);
    const StateDesc& s = sd[blockIdx.y];
    double2* psi = reinterpret_cast<double2*>(smem + L.vec);
    uint32_t* str = reinterpret_cast<uint32_t*>(smem + L.str);
    int16_t* rank = reinterpret_cast<int16_t*>(smem + L.rank);
    small_stage_space(sp, str, rank);
    for (int t = threadIdx.x; t < sp.nsec; t += kSmallThreads) psi[t] = s.phi[t];
    // the state's own Hamiltonian fits the staged region when the launch has one
    const bool hlds = sp.ham_lds > 0 && small_ham_bytes(s.G, s.nsub, s.ntab) <= size_t(sp.ham_lds);
    double* tabs = reinterpret_cast<double*>(smem + L.ham);
    GroupDesc* groups = reinterpret_cast<GroupDesc*>(tabs + s.ntab);
    SubDesc* subs = reinterpret_cast<SubDesc*>(groups + s.G);
    if (hlds) {
        for (int t = threadIdx.x; t < s.ntab; t += kSmallThreads) tabs[t] = s.tabs[t];
        for (int t = threadIdx.x; t < s.G; t += kSmallThreads) groups[t] = s.groups[t];
        for (int t = threadIdx.x; t < s.nsub; t += kSmallThreads) subs[t] = s.subs[t];
    }
    __syncthreads();
    if (hlds)
        small_hx_body(s, sp, groups, subs, tabs, str, rank, psi, red);
    else
        small_hx_body(s, sp, s.groups, s.subs, s.tabs, str, rank, psi, red);
}

// Reverse sweep: per gate (last first) each wave's part of Re <lambda|A_j phi>
// into LDS, then U_j^dag on phi and lambda in the same pass; the per-gate sums
// (waves added in fixed order) into out_g at the end.
__global__ void __launch_bounds__(kSmallThreads) k_small_adj(const StateDesc* __restrict__ sd, SmallSpace sp) {
    extern __shared__ __align__(16) unsigned char smem[];
    const SmallLayout L = small_layout(sp, 2, true, false);
    const StateDesc& s = sd[blockIdx.y];
    double2* psi = reinterpret_cast<double2*>(smem + L.vec);
    double2* lam = psi + sp.nsec;
    SmallGate* gs = reinterpret_cast<SmallGate*>(smem + L.gates);
    uint32_t* str = reinterpret_cast<uint32_t*>(smem + L.str);
    int16_t* rank = reinterpret_cast<int16_t*>(smem + L.rank);
    double* part = reinterpret_cast<double*>(smem + L.total);   // [M][waves] gradient partials
    small_stage_space(sp, str, rank);
    for (int t = threadIdx.x; t < sp.nsec; t += kSmallThreads) {
        psi[t] = s.phi[t];
        lam[t] = s.lam[t];
    }
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
            double2 fD = psi[t], fE = psi[re], lD = lam[t], lE = lam[re];
            // A|D> = s|E>, A|E> = -s|D>: <lam|A phi> = s (lam_E^* phi_D - lam_D^* phi_E)
            acc += sg * ((lE.x * fD.x + lE.y * fD.y) - (lD.x * fE.x + lD.y * fE.y));
            const double ss = -sg * g.s;   // U^dag: rotation by -theta
            givens(fD, fE, g.c, ss);
            givens(lD, lE, g.c, ss);
            psi[t] = fD;
            psi[re] = fE;
            lam[t] = lD;
            lam[re] = lE;
        }
        acc = wave_total(acc);
        if ((threadIdx.x & 63) == 0) part[size_t(j) * kSmallWaves + w] = acc;
        __syncthreads();
    }
    for (int j = threadIdx.x; j < s.M; j += kSmallThreads) {
        double r = 0.0;
#pragma unroll
        for (int i = 0; i < kSmallWaves; ++i) r += part[size_t(j) * kSmallWaves + i];
        s.out_g[j] = r;
    }
}

size_t small_lds(const SmallSpace& sp, int phase) {
    if (phase == 0) return small_layout(sp, 1, true, false).total;
    if (phase == 1) return small_layout(sp, 1, false, true).total;
    return small_layout(sp, 2, true, false).total + 8 * size_t(kSmallWaves) * size_t(sp.M);
}

// The launches' LDS must fit the CU's 160 KiB; beyond 64 KiB the kernels are
// allowed the whole of it (once).
int small_prepare(const SmallSpace& sp) {
    constexpr size_t kMax = size_t(160) << 10;
    size_t lds = 0;
    for (int ph = 0; ph < 3; ++ph) lds = std::max(lds, small_lds(sp, ph) + 8 * kSmallWaves);
    if (lds > kMax) return 1;
    if (lds <= (64u << 10)) return 0;
    static std::once_flag once;
    static int rc = 0;
    std::call_once(once, [] {
        const void* fs[3] = {reinterpret_cast<const void*>(&k_small_fwd), reinterpret_cast<const void*>(&k_small_hx),
                             reinterpret_cast<const void*>(&k_small_adj)};
        for (const void* f : fs)
            if (hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, int(kMax)) != hipSuccess) rc = 1;
    });
    return rc;
}

void launch_small(int phase, const StateDesc* sd, int count, const SmallSpace& sp, hipStream_t st) {
    const size_t lds = small_lds(sp, phase);
    if (phase == 0)
        hipLaunchKernelGGL(k_small_fwd, dim3(1, count), dim3(kSmallThreads), lds, st, sd, sp);
    else if (phase == 1)
        hipLaunchKernelGGL(k_small_hx, dim3(1, count), dim3(kSmallThreads), lds, st, sd, sp);
    else
        hipLaunchKernelGGL(k_small_adj, dim3(1, count), dim3(kSmallThreads), lds, st, sd, sp);
}

}  // namespace vqe
