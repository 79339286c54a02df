// H-apply kernels: lambda = H phi and the expectation Re <phi|lambda>
// (Sec. 2.1.1, Eq. 1) for H = sum_k c_k P_k grouped by x-mask.
//
// For an x-group g the folded terms act as
//   lambda[b'] += psi[b' ^ x_g] * D_g(b'),
//   D_g(b')     = sum_{s in sub(g)} (-1)^{popcount(b' & w_s)} tab_s[pext(b', x_g)],
// so one gather of psi[b' ^ x_g] serves every z-mask of the group.
//
//  k_hx_dense   every output index, every group (any state)
//  k_hx_sector  only outputs in the (N, S_z) sector of the reference (every
//               number- and spin-conserving circuit stays there, and H maps the
//               sector to itself).  Outputs are tiled by their low L bits; for
//               each x_hi = x >> L batch of groups the partner tile's in-sector
//               amplitudes are staged compressed in LDS, indexed by the
//               combinatorial rank of their alpha and beta occupation strings.
#include "device_common.h"

namespace vqe {

__global__ void __launch_bounds__(kBlock) k_hx_dense(const StateDesc* __restrict__ sd, uint64_t N,
                                                     int write_lam) {
    __shared__ double red[kBlock / 64];
    const StateDesc& s = sd[blockIdx.y];
    const double2* __restrict__ phi = s.phi;
    const GroupDesc* __restrict__ groups = s.groups;
    const int G = s.G;
    double acc = 0.0;
    for (uint64_t b = blockIdx.x * uint64_t(blockDim.x) + threadIdx.x; b < N;
         b += uint64_t(gridDim.x) * blockDim.x) {
        const uint32_t b32 = uint32_t(b);
        double lr = 0.0, li = 0.0;
        for (int gi = 0; gi < G; ++gi) {
            const GroupDesc gd = groups[gi];
            const double2 p = phi[b ^ gd.x];
            const double d = group_coeff(gd, s.subs, s.tabs, b32);
            lr += d * p.x;
            li += d * p.y;
        }
        if (write_lam) s.lam[b] = make_double2(lr, li);
        const double2 q = phi[b];
        acc += q.x * lr + q.y * li;
    }
    const double r = block_sum(acc, red);
    if (threadIdx.x == 0) s.part_e[blockIdx.x] = r;
}

// Bits 0, 2, 4, ... of v packed into bits 0, 1, 2, ... (v < 2^14).
__device__ __forceinline__ uint32_t compact_even(uint32_t v) {
    v &= 0x5555u;
    v = (v | (v >> 1)) & 0x3333u;
    v = (v | (v >> 2)) & 0x0F0Fu;
    v = (v | (v >> 4)) & 0x00FFu;
    return v;
}

constexpr int kMaxStage = 1225;   // C(7,3) * C(7,4): largest class of a 14-bit tile
constexpr int kStagePer = (kMaxStage + kBlock - 1) / kBlock;

// PACKED: phi and lambda hold only the sector, block h = b >> L from base[h]
// in the same (alpha rank, beta rank) order as the tile here; otherwise they
// are full 2^n vectors.
template <bool PACKED>
__global__ void __launch_bounds__(kBlock) k_hx_sector(const StateDesc* __restrict__ sd,
                                                      HxPlan plan,
                                                      const HxTables* __restrict__ tabsrc,
                                                      const int32_t* __restrict__ base) {
    __shared__ double2 stage[kMaxStage];      // partner tile, in-sector amplitudes by rank
    __shared__ double tch[kChunkTabs];        // the chunk's coefficient tables
    __shared__ GroupDesc gch[kChunkGroups];   // the chunk's groups (chunk-local sub ranges)
    __shared__ SubDesc sch[kChunkSubs];       // the chunk's subgroups (chunk-local tables)
    __shared__ HxTables T;
    __shared__ double red[kBlock / 64];
    {   // copy the rank/unrank tables into LDS
        const uint32_t* src = reinterpret_cast<const uint32_t*>(tabsrc);
        uint32_t* dst = reinterpret_cast<uint32_t*>(&T);
        for (int i = threadIdx.x; i < int(sizeof(HxTables) / 4); i += kBlock) dst[i] = src[i];
    }
    __syncthreads();
    const StateDesc& s = sd[blockIdx.y];
    const double2* __restrict__ phi = s.phi;
    const double* __restrict__ tabs = s.tabs;
    const int L = plan.L;
    const uint32_t lowmask = (1u << L) - 1u;
    const uint32_t ohi = uint32_t(blockIdx.x) << L;
    const int kA = plan.na - __popc(ohi & 0x55555555u);
    const int kB = plan.nb - __popc(ohi & 0xAAAAAAAAu);
    if (kA < 0 || kA > T.La || kB < 0 || kB > T.Lb) {   // no in-sector output here
        if (threadIdx.x == 0) s.part_e[blockIdx.x] = 0.0;
        return;
    }
    const int cB = T.offB[kB + 1] - T.offB[kB];
    const int cnt = (T.offA[kA + 1] - T.offA[kA]) * cB;
    uint32_t lo[kHxOuts];
    double lr[kHxOuts], li[kHxOuts];
#pragma unroll
    for (int u = 0; u < kHxOuts; ++u) {
        const int k = threadIdx.x + u * kBlock;
        lo[u] = (k < cnt) ? uint32_t(T.unA[T.offA[kA] + k / cB] | T.unB[T.offB[kB] + k % cB]) : 0u;
        lr[u] = li[u] = 0.0;
    }
    uint32_t staged = 0xffffffffu;   // x_hi whose partner tile is in `stage`
    int kA2 = 0, kB2 = 0, cB2 = 1;
    for (int c = 0; c < s.nb; ++c) {
        const HxChunk ck = s.chunks[c];
        if (ck.xhi != staged) {
            const uint32_t phi_hi = ohi ^ (ck.xhi << L);
            const int a2 = plan.na - __popc(phi_hi & 0x55555555u);
            const int b2 = plan.nb - __popc(phi_hi & 0xAAAAAAAAu);
            if (a2 < 0 || a2 > T.La || b2 < 0 || b2 > T.Lb) {   // partner tile empty: skip batch
                while (c + 1 < s.nb && s.chunks[c + 1].xhi == ck.xhi) ++c;
                continue;
            }
            kA2 = a2;
            kB2 = b2;
            cB2 = T.offB[kB2 + 1] - T.offB[kB2];
            const int cnt2 = (T.offA[kA2 + 1] - T.offA[kA2]) * cB2;
            double2 v[kStagePer];
#pragma unroll
            for (int k = 0; k < kStagePer; ++k) {
                const int i = threadIdx.x + k * kBlock;
                if (i < cnt2) {
                    if (PACKED)
                        v[k] = phi[int64_t(base[phi_hi >> L]) + i];
                    else
                        v[k] = phi[phi_hi | T.unA[T.offA[kA2] + i / cB2] | T.unB[T.offB[kB2] + i % cB2]];
                }
            }
            __syncthreads();   // everyone done with the previous stage
#pragma unroll
            for (int k = 0; k < kStagePer; ++k) {
                const int i = threadIdx.x + k * kBlock;
                if (i < cnt2) stage[i] = v[k];
            }
            staged = ck.xhi;
        } else {
            __syncthreads();   // everyone done with the previous chunk
        }
        // stage the chunk's descriptors and tables
        const int ng = ck.cg1 - ck.cg0, ns = ck.cs1 - ck.cs0, nt = ck.t1 - ck.t0;
        for (int i = threadIdx.x; i < ng; i += kBlock) gch[i] = s.cgroups[ck.cg0 + i];
        for (int i = threadIdx.x; i < ns; i += kBlock) sch[i] = s.csubs[ck.cs0 + i];
        for (int i = threadIdx.x; i < nt; i += kBlock) tch[i] = tabs[ck.t0 + i];
        __syncthreads();
        for (int gi = 0; gi < ng; ++gi) {
            const GroupDesc gd = gch[gi];
            const uint32_t xlo = gd.x & lowmask;
            double2 p[kHxOuts];
            uint32_t tb[kHxOuts];
            bool ok[kHxOuts];
            bool any = false;
#pragma unroll
            for (int u = 0; u < kHxOuts; ++u) {
                const int k = threadIdx.x + u * kBlock;
                const uint32_t lp = lo[u] ^ xlo;
                ok[u] = (k < cnt) && __popc(lp & 0x5555u) == kA2 && __popc(lp & 0xAAAAu) == kB2;
                p[u] = make_double2(0.0, 0.0);
                tb[u] = 0;
                if (ok[u]) {
                    const int idx = int(T.rankA[compact_even(lp)]) * cB2 +
                                    int(T.rankB[compact_even(lp >> 1)]);
                    p[u] = stage[idx];
                    tb[u] = pext_pos(ohi | lo[u], gd.pos);
                    any = true;
                }
            }
            if (!__ballot(any)) continue;   // wave-uniform skip
            double d[kHxOuts];
#pragma unroll
            for (int u = 0; u < kHxOuts; ++u) d[u] = 0.0;
            for (int si = gd.sub_begin; si < gd.sub_end; ++si) {
                const SubDesc sub = sch[si];
#pragma unroll
                for (int u = 0; u < kHxOuts; ++u) {
                    const double t = tch[sub.tab + tb[u]];
                    d[u] += (__popc((ohi | lo[u]) & sub.w) & 1) ? -t : t;
                }
            }
#pragma unroll
            for (int u = 0; u < kHxOuts; ++u) {
                if (ok[u]) {
                    lr[u] += d[u] * p[u].x;
                    li[u] += d[u] * p[u].y;
                }
            }
        }
    }
    double acc = 0.0;
    const int64_t obase = PACKED ? int64_t(base[blockIdx.x]) : 0;
#pragma unroll
    for (int u = 0; u < kHxOuts; ++u) {
        const int k = threadIdx.x + u * kBlock;
        if (k < cnt) {
            const int64_t b = PACKED ? obase + k : int64_t(ohi | lo[u]);
            s.lam[b] = make_double2(lr[u], li[u]);
            const double2 q = phi[b];
            acc += q.x * lr[u] + q.y * li[u];
        }
    }
    const double r = block_sum(acc, red);
    if (threadIdx.x == 0) s.part_e[blockIdx.x] = r;
}

// Sector H-apply on the packed layout.  Same tiling as k_hx_sector (output
// tile = block h, partner block h ^ x_hi staged in LDS).  Thread t owns the
// outputs k = t * kHxOuts + u; each output's low alpha and beta bits are
// kept as compact 7-bit strings, and the partner's position within the
// staged block comes from two class rank tables that also flag a partner of
// the wrong electron count (negative index), so no separate sector test is
// needed.  Group and subgroup fields are read into scalar registers (they
// are the same for all lanes).
__global__ void __launch_bounds__(kBlock) k_hx_packed(const StateDesc* __restrict__ sd, HxPlan plan,
                                                      const HxTables* __restrict__ tabsrc,
                                                      const int32_t* __restrict__ base) {
    __shared__ double2 stage[kMaxStage];
    __shared__ double tch[kChunkTabs];
    __shared__ GroupDesc gch[kChunkGroups];
    __shared__ SubDesc sch[kChunkSubs];
    __shared__ HxTables T;
    __shared__ RankK R;
    __shared__ double red[kBlock / 64];
    {
        const uint32_t* src = reinterpret_cast<const uint32_t*>(tabsrc);
        uint32_t* dst = reinterpret_cast<uint32_t*>(&T);
        for (int i = threadIdx.x; i < int(sizeof(HxTables) / 4); i += kBlock) dst[i] = src[i];
        const uint32_t* srk = reinterpret_cast<const uint32_t*>(
            reinterpret_cast<const char*>(tabsrc) + kRankKOffset);
        uint32_t* drk = reinterpret_cast<uint32_t*>(&R);
        for (int i = threadIdx.x; i < int(sizeof(RankK) / 4); i += kBlock) drk[i] = srk[i];
    }
    __syncthreads();
    const StateDesc& s = sd[blockIdx.y];
    const double2* __restrict__ phi = s.phi;
    const double* __restrict__ tabs = s.tabs;
    const int L = plan.L;
    const uint32_t ohi = uint32_t(blockIdx.x) << L;
    const int kA = plan.na - __popc(ohi & 0x55555555u);
    const int kB = plan.nb - __popc(ohi & 0xAAAAAAAAu);
    if (kA < 0 || kA > T.La || kB < 0 || kB > T.Lb) {   // empty block
        if (threadIdx.x == 0) s.part_e[blockIdx.x] = 0.0;
        return;
    }
    const int cB = T.offB[kB + 1] - T.offB[kB];
    const int cnt = (T.offA[kA + 1] - T.offA[kA]) * cB;
    uint32_t sv[kHxOuts], ca[kHxOuts], cb[kHxOuts];
    double lr[kHxOuts], li[kHxOuts];
    // a slot past the block's end works on a copy of entry 0 and is not written
#pragma unroll
    for (int u = 0; u < kHxOuts; ++u) {
        const int k = threadIdx.x * kHxOuts + u;
        const int kc = (k < cnt) ? k : 0;
        const uint32_t lo = uint32_t(T.unA[T.offA[kA] + kc / cB] | T.unB[T.offB[kB] + kc % cB]);
        sv[u] = ohi | lo;
        ca[u] = compact_even(lo);
        cb[u] = compact_even(lo >> 1);
        lr[u] = li[u] = 0.0;
    }
    // waves whose outputs all lie past the block's end only help with staging
    const bool wave_live = __ballot(int(threadIdx.x) * kHxOuts < cnt) != 0;
    uint32_t staged = 0xffffffffu;   // x_hi whose partner block is in `stage`
    int cB2 = 1, kA2 = 0, kB2 = 0;
    for (int c = 0; c < s.nb; ++c) {
        const HxChunk ck = s.chunks[c];
        if (ck.xhi != staged) {
            const uint32_t hp = uint32_t(blockIdx.x) ^ ck.xhi;
            const uint32_t phi_hi = hp << L;
            const int a2 = plan.na - __popc(phi_hi & 0x55555555u);
            const int b2 = plan.nb - __popc(phi_hi & 0xAAAAAAAAu);
            if (a2 < 0 || a2 > T.La || b2 < 0 || b2 > T.Lb) {   // partner block empty: skip batch
                while (c + 1 < s.nb && s.chunks[c + 1].xhi == ck.xhi) ++c;
                continue;
            }
            kA2 = a2;
            kB2 = b2;
            cB2 = T.offB[b2 + 1] - T.offB[b2];
            const int cnt2 = (T.offA[a2 + 1] - T.offA[a2]) * cB2;
            const double* src = reinterpret_cast<const double*>(phi + base[hp]);
            double vr[kStagePer], vi[kStagePer];
#pragma unroll
            for (int k = 0; k < kStagePer; ++k) {   // clamped: every load is in the block
                const int i = min(int(threadIdx.x) + k * kBlock, cnt2 - 1);
                vr[k] = src[2 * i];
                vi[k] = src[2 * i + 1];
            }
            __syncthreads();   // everyone done with the previous stage
#pragma unroll
            for (int k = 0; k < kStagePer; ++k) {
                const int i = threadIdx.x + k * kBlock;
                if (i < cnt2) stage[i] = make_double2(vr[k], vi[k]);
            }
            staged = ck.xhi;
        } else {
            __syncthreads();   // everyone done with the previous chunk
        }
        const int ng = ck.cg1 - ck.cg0, ns = ck.cs1 - ck.cs0, nt = ck.t1 - ck.t0;
        for (int i = threadIdx.x; i < ng; i += kBlock) gch[i] = s.cgroups[ck.cg0 + i];
        for (int i = threadIdx.x; i < ns; i += kBlock) sch[i] = s.csubs[ck.cs0 + i];
        for (int i = threadIdx.x; i < nt; i += kBlock) tch[i] = tabs[ck.t0 + i];
        __syncthreads();
        if (!wave_live) continue;
        const int16_t* ra = R.a[kA2];
        const int16_t* rb = R.b[kB2];
        for (int gi = 0; gi < ng; ++gi) {
            const uint32_t x = __builtin_amdgcn_readfirstlane(gch[gi].x);
            if ((__popc(x & 0x55555555u) | __popc(x & 0xAAAAAAAAu)) & 1)
                continue;   // changes N_alpha or N_beta: no in-sector pair
            const uint32_t pos = __builtin_amdgcn_readfirstlane(gch[gi].pos);
            const int sb = __builtin_amdgcn_readfirstlane(gch[gi].sub_begin);
            const int se = __builtin_amdgcn_readfirstlane(gch[gi].sub_end);
            const uint32_t xl = x & ((1u << L) - 1u);
            const uint32_t xa = compact_even(xl), xb = compact_even(xl >> 1);
            int idx[kHxOuts];
            bool any = false;
#pragma unroll
            for (int u = 0; u < kHxOuts; ++u) {
                idx[u] = int(ra[ca[u] ^ xa]) * cB2 + int(rb[cb[u] ^ xb]);
                any |= idx[u] >= 0;
            }
            if (!__ballot(any)) continue;   // wave-uniform skip
            // table positions (bit 31 of an output string is 0: n < 32)
            const uint32_t q0 = (pos >> 3) & 31, q1 = (pos >> 8) & 31, q2 = (pos >> 13) & 31,
                           q3 = (pos >> 18) & 31;
            double2 p[kHxOuts];
            uint32_t ti[kHxOuts];
#pragma unroll
            for (int u = 0; u < kHxOuts; ++u) {
                ti[u] = __builtin_amdgcn_ubfe(sv[u], q0, 1) | (__builtin_amdgcn_ubfe(sv[u], q1, 1) << 1) |
                        (__builtin_amdgcn_ubfe(sv[u], q2, 1) << 2) |
                        (__builtin_amdgcn_ubfe(sv[u], q3, 1) << 3);
                p[u] = (idx[u] >= 0) ? stage[idx[u]] : make_double2(0.0, 0.0);
            }
            double d[kHxOuts];
#pragma unroll
            for (int u = 0; u < kHxOuts; ++u) d[u] = 0.0;
            for (int si = sb; si < se; ++si) {
                const uint32_t w = __builtin_amdgcn_readfirstlane(sch[si].w);
                const int toff = __builtin_amdgcn_readfirstlane(sch[si].tab);
#pragma unroll
                for (int u = 0; u < kHxOuts; ++u) {
                    // (-1)^{|b & w|} applied as a flip of the sign bit
                    const double t = tch[toff + ti[u]];
                    const uint32_t flip = uint32_t(__popc(sv[u] & w)) << 31;
                    d[u] += __hiloint2double(__double2hiint(t) ^ int(flip), __double2loint(t));
                }
            }
#pragma unroll
            for (int u = 0; u < kHxOuts; ++u) {
                lr[u] += d[u] * p[u].x;   // p = 0 where the pair is not in the sector
                li[u] += d[u] * p[u].y;
            }
        }
    }
    double acc = 0.0;
    double2* out = s.lam + base[blockIdx.x];
    const double2* own = phi + base[blockIdx.x];
#pragma unroll
    for (int u = 0; u < kHxOuts; ++u) {
        const int k = threadIdx.x * kHxOuts + u;
        if (k < cnt) {
            out[k] = make_double2(lr[u], li[u]);
            const double2 q = own[k];
            acc += q.x * lr[u] + q.y * li[u];
        }
    }
    const double r = block_sum(acc, red);
    if (threadIdx.x == 0) s.part_e[blockIdx.x] = r;
}

void launch_hx_dense(const StateDesc* sd, int count, uint64_t N, int nblk, int write_lam,
                     hipStream_t st) {
    hipLaunchKernelGGL(k_hx_dense, dim3(nblk, count), dim3(kBlock), 0, st, sd, N, write_lam);
}

void launch_hx_sector(const StateDesc* sd, int count, const HxPlan& plan, const HxTables* tabs,
                      hipStream_t st) {
    hipLaunchKernelGGL(k_hx_sector<false>, dim3(plan.ntiles, count), dim3(kBlock), 0, st, sd, plan,
                       tabs, nullptr);
}

void launch_hx_packed(const StateDesc* sd, int count, const HxPlan& plan, const HxTables* tabs,
                      const int32_t* base, hipStream_t st) {
    hipLaunchKernelGGL(k_hx_packed, dim3(plan.ntiles, count), dim3(kBlock), 0, st, sd, plan, tabs,
                       base);
}

}  // namespace vqe
