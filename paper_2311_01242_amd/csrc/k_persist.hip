// Persistent gate passes over a whole batch of packed states (the batched
// evaluation of many states of uneven qubit counts, Sec. 2.1.1 Eq. 1 and its
// adjoint gradient): one launch applies every run of every state of every
// size class, forward or reverse.
//
// Work items are (state, run, live tile) triples in per-XCD queues built on
// the host; the workgroups of a launch (one wave each) read the hardware id
// of the XCD they run on and take items from that XCD's queue through an
// atomic head counter, so every item of a state runs on one XCD and its tiles
// pass from run to run through that XCD's L2.  An item may start once all
// tiles of the state's earlier runs (in pass order) are done: it waits until
// the state's completion counter reaches the item's `need`.  Items are queued
// run by run, so an item only ever waits on items dequeued before it, held by
// running workgroups: no deadlock for any grid size.  Every wait is bounded;
// a wait that gives up sets its queue's error flag (read by the host) and
// ends the workgroup, and the other waits of that queue see the flag and end
// too.
//
// Coherence inside an XCD: tiles are written with plain stores (L1 is
// write-through), the writer waits for its stores to be acknowledged before
// it bumps the counter with a device-scope atomic (executed in the XCD's
// L2), and readers poll the counter and stage tiles with loads that bypass
// L1 (device scope), so they read what L2 holds.
//
// Inside an item one wave applies the run's gates to the tile staged in LDS:
// the pairs of a gate are disjoint, the wave's LDS operations execute in
// issue order, so no barrier is needed between gates; each lane holds up to
// PMAX pair entries of the gate in registers (the next gate's are loaded
// while the current gate runs), reads all its pairs' amplitudes, rotates
// them and writes them back.  The reverse sweep also forms the gate's
// Re <lambda|A_j phi> partial of the tile (fixed-order wave total).
#include "device_common.h"

namespace vqe {

constexpr int kPqBatch = 1;   // items per queue-head atomic (8 was slower: a run's tiles then finish one after another)

__device__ __forceinline__ void wave_lds_fence() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// 16-byte load that misses in L1 (device scope): reads the XCD's L2.
__device__ __forceinline__ double2 ld_l2(__amdgpu_buffer_rsrc_t r, uint32_t byte_off) {
    typedef int v4i __attribute__((ext_vector_type(4)));
    const v4i v = __builtin_amdgcn_raw_buffer_load_b128(r, byte_off, 0, 16 /* sc1 */);
    return make_double2(__hiloint2double(v.y, v.x), __hiloint2double(v.w, v.z));
}

__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc_of(const void* base, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000);
}

__device__ __forceinline__ int32_t ld_counter(const int32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint32_t xcc_id() {
    // hwreg(HW_REG_XCC_ID, 0, 16)
    return __builtin_amdgcn_s_getreg(20 | (0 << 6) | (15 << 11));
}

// Copy of c consecutive amplitudes (both vectors of the reverse sweep) from
// global memory into LDS, 8 per lane in flight per pass: buffer loads that
// miss L1 and read 0 past the block's end (no branch around the loads).
template <int VEC>
__device__ __forceinline__ void stage_block(const double2* phi, const double2* lam, int c, double2* shp,
                                            double2* shl, int lane) {
    const __amdgpu_buffer_rsrc_t rp = rsrc_of(phi, uint32_t(c) * 16u);
    const __amdgpu_buffer_rsrc_t rl = rsrc_of(lam, uint32_t(c) * 16u);
    for (int k0 = 0; k0 < c; k0 += 8 * 64) {
        double2 vp[8], vl[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const uint32_t off = uint32_t(k0 + lane + 64 * u) * 16u;
            vp[u] = ld_l2(rp, off);
            if (VEC == 2) vl[u] = ld_l2(rl, off);
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int k = k0 + lane + 64 * u;
            if (k < c) {
                shp[k] = vp[u];
                if (VEC == 2) shl[k] = vl[u];
            }
        }
    }
}

__device__ __forceinline__ void wait_vm0() { __builtin_amdgcn_s_waitcnt(0x0f70); }   // vmcnt(0)

// What one item needs, loaded once it is dequeued.
struct PqTile {
    PqItem item;
    PackedRun run;
    const PackedGate* pg;
    double2* phi;
    double2* lam;
    const double2* cs;       // the state's (cos, sin) per gate
    double* part_g;
    int32_t gstride;
    TileBlocks tb;
    const uint32_t* lbase;   // the tile class's pair lists
    int stride;
    bool empty;
};

__device__ __forceinline__ void load_tile(const PqArgs& a, const HxTables& T, int idx, PqTile& d) {
    d.item = ldc(a.items + idx);
    const PqRun& R = a.runs[d.item.run];
    d.run = ldc(&R.r);
    d.pg = ldc(&R.pg);
    const int32_t* base = ldc(&R.base);
    const StateDesc& s = a.sd[d.item.state];
    d.phi = s.phi;
    d.lam = s.lam;
    d.cs = s.cs;
    d.part_g = s.part_g;
    d.gstride = s.gstride;
    const int o = d.run.live ? ldc(d.run.live + d.item.tile) : d.item.tile;
    tile_blocks(T, d.run, o, base, d.tb);
    d.empty = d.tb.nE == 0;
    const int2 lc = d.empty ? make_int2(0, 0) : ldc(d.run.info + d.tb.cls);
    d.lbase = d.run.ent + lc.x;
    d.stride = lc.y;
}

// Bounded wait until the item's state has `need` finished tiles; false when
// it gave up (its queue's error flag is then set) or the flag was already set.
__device__ __forceinline__ bool wait_dep(const PqArgs& a, int q, const PqItem& it, int spin_limit, int lane) {
    if (it.need <= 0) return true;
    int polls = 0;
    for (;;) {
        if (ld_counter(a.done + it.state) >= it.need) return true;
        if (ld_counter(a.err + q) != 0 || ++polls > spin_limit) break;
        __builtin_amdgcn_s_sleep(2);
    }
    if (lane == 0) __hip_atomic_store(a.err + q, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return false;
}

__device__ __forceinline__ void publish(const PqArgs& a, int state, int lane) {
    if (lane == 0) __hip_atomic_fetch_add(a.done + state, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Stage an item: its tile (both vectors of the reverse sweep) and the
// per-gate parameters of the tile.
template <int VEC>
__device__ __forceinline__ void stage(const PqTile& d, double2* shp, double2* shl, double2* gpar, int lane) {
#pragma unroll
    for (int b = 0; b < kMaxTileBlocks; ++b) {
        if (b >= d.run.nblk) break;
        const int c = (b + 1 < d.run.nblk ? d.tb.off[b + 1] : d.tb.nE) - d.tb.off[b];
        if (c > 0)
            stage_block<VEC>(d.phi + d.tb.gb[b], d.lam + d.tb.gb[b], c, shp + d.tb.off[b], shl + d.tb.off[b],
                             lane);
    }
    const int ng = d.run.g1 - d.run.g0;
    for (int j = lane; j < ng; j += 64) {
        const PackedGate g = d.pg[j];
        const double2 cs = d.cs[d.run.g0 + j];
        const double sgn = g.csign * parity_sign((d.tb.hbase << d.run.L) & g.chhi);
        gpar[2 * j] = make_double2(cs.x, sgn * cs.y);
        gpar[2 * j + 1] = make_double2(sgn, 0.0);
    }
}

// Pair entries of gate t (pass order) of the tile for this lane: slot p
// holds list position lane + 64 p.  Positions past the list re-read its last
// entry and gates past the run re-read the run's last gate, so that every
// call issues the same PMAX loads with no branch and no use of the result
// (the compiler then waits for each ring slot alone, where it is used);
// apply_gate ignores slots at positions past the list.
template <int PMAX>
__device__ __forceinline__ void load_entries(uint32_t (&e)[PMAX], const PqTile& d, int t, int ng, bool fwd,
                                             int lane) {
    const int tc = t < ng ? t : ng - 1;
    const uint32_t* l = d.lbase + size_t(fwd ? tc : ng - 1 - tc) * d.stride;
    const int last = max(d.stride - 1, 0);
#pragma unroll
    for (int p = 0; p < PMAX; ++p) e[p] = ldg32(l + min(lane + 64 * p, last));
}

// One gate of the tile: the lane's pairs in e (and, for lists longer than
// 64 PMAX, the rest read one at a time); the reverse sweep also stores the
// gate's tile partial of Re <lambda|A_j phi>.
template <int VEC, int PMAX, bool OVF>
__device__ __forceinline__ void apply_gate(const PqTile& d, int jl, const uint32_t (&e_in)[PMAX],
                                           double2* shp, double2* shl, const double2* gpar, double* gsum,
                                           int lane) {
    constexpr bool fwd = (VEC == 1);
    // the entries are first used here: the empty asm keeps the compiler from
    // hoisting their decoding (and the wait for their loads) above the
    // previous gates
    uint32_t e[PMAX];
#pragma unroll
    for (int p = 0; p < PMAX; ++p) {
        e[p] = e_in[p];
        __asm__ volatile("" : "+v"(e[p]));
    }
    const double2 cs = gpar[2 * jl];            // (cos, sgn sin)
    const double sgn_hi = gpar[2 * jl + 1].x;  // the tile's part of the sign
    double acc = 0.0;
    double2 fD[PMAX], fE[PMAX], lD[PMAX], lE[PMAX];
    bool on[PMAX];
#pragma unroll
    for (int p = 0; p < PMAX; ++p) on[p] = (lane + 64 * p < d.stride) && e[p] != kPairNone;
#pragma unroll
    for (int p = 0; p < PMAX; ++p) {
        if (on[p]) {
            const int k = int(e[p] & kEntMask), ie = int((e[p] >> kEntBits) & kEntMask);
            fD[p] = shp[k];
            fE[p] = shp[ie];
            if (VEC == 2) {
                lD[p] = shl[k];
                lE[p] = shl[ie];
            }
        }
    }
#pragma unroll
    for (int p = 0; p < PMAX; ++p) {
        if (on[p]) {
            const int k = int(e[p] & kEntMask), ie = int((e[p] >> kEntBits) & kEntMask);
            const bool neg = (e[p] >> kEntParity) & 1u;
            const double ss = neg ? -cs.y : cs.y;
            if (fwd) {
                givens(fD[p], fE[p], cs.x, ss);
            } else {
                const double sg_t = neg ? -sgn_hi : sgn_hi;
                acc += sg_t * ((lE[p].x * fD[p].x + lE[p].y * fD[p].y) - (lD[p].x * fE[p].x + lD[p].y * fE[p].y));
                givens(fD[p], fE[p], cs.x, -ss);
                givens(lD[p], lE[p], cs.x, -ss);
                shl[k] = lD[p];
                shl[ie] = lE[p];
            }
            shp[k] = fD[p];
            shp[ie] = fE[p];
        }
    }
    for (int i = lane + 64 * PMAX; OVF && i < d.stride; i += 64) {
        const uint32_t x = ldg32(d.lbase + size_t(jl) * d.stride + i);
        if (x == kPairNone) break;
        const int k = int(x & kEntMask), ie = int((x >> kEntBits) & kEntMask);
        const bool neg = (x >> kEntParity) & 1u;
        const double ss = neg ? -cs.y : cs.y;
        double2 dd = shp[k], ff = shp[ie];
        if (fwd) {
            givens(dd, ff, cs.x, ss);
        } else {
            double2 ld = shl[k], le = shl[ie];
            const double sg_t = neg ? -sgn_hi : sgn_hi;
            acc += sg_t * ((le.x * dd.x + le.y * dd.y) - (ld.x * ff.x + ld.y * ff.y));
            givens(dd, ff, cs.x, -ss);
            givens(ld, le, cs.x, -ss);
            shl[k] = ld;
            shl[ie] = le;
        }
        shp[k] = dd;
        shp[ie] = ff;
    }
    if (!fwd) {
        acc = wave_total(acc);
        if (lane == 0) gsum[jl] = acc;
    }
    wave_lds_fence();
}

// The gates of a staged tile, in pass order, with the pair entries of the
// next three gates in flight (a ring of four register sets, refilled right
// after each gate, the same loads on every path).  The reverse sweep's tile
// partials collect in LDS and go out after the last gate.
template <int VEC, int PMAX, bool OVF>
__device__ __forceinline__ void run_gates(const PqTile& d, double2* shp, double2* shl, const double2* gpar,
                                          double* gsum, int lane) {
    constexpr bool fwd = (VEC == 1);
    const int ng = d.run.g1 - d.run.g0;
    uint32_t r0[PMAX], r1[PMAX], r2[PMAX], r3[PMAX];
    // issued in ring order (the scheduling barriers keep them so), as the
    // refills in the loop are
    load_entries(r0, d, 0, ng, fwd, lane);
    __builtin_amdgcn_sched_barrier(0);
    load_entries(r1, d, 1, ng, fwd, lane);
    __builtin_amdgcn_sched_barrier(0);
    load_entries(r2, d, 2, ng, fwd, lane);
    __builtin_amdgcn_sched_barrier(0);
    load_entries(r3, d, 3, ng, fwd, lane);
    __builtin_amdgcn_sched_barrier(0);
    int t = 0;
    for (; t + 4 <= ng; t += 4) {
        apply_gate<VEC, PMAX, OVF>(d, fwd ? t : ng - 1 - t, r0, shp, shl, gpar, gsum, lane);
        load_entries(r0, d, t + 4, ng, fwd, lane);
        apply_gate<VEC, PMAX, OVF>(d, fwd ? t + 1 : ng - 2 - t, r1, shp, shl, gpar, gsum, lane);
        load_entries(r1, d, t + 5, ng, fwd, lane);
        apply_gate<VEC, PMAX, OVF>(d, fwd ? t + 2 : ng - 3 - t, r2, shp, shl, gpar, gsum, lane);
        load_entries(r2, d, t + 6, ng, fwd, lane);
        apply_gate<VEC, PMAX, OVF>(d, fwd ? t + 3 : ng - 4 - t, r3, shp, shl, gpar, gsum, lane);
        load_entries(r3, d, t + 7, ng, fwd, lane);
    }
    if (t < ng) apply_gate<VEC, PMAX, OVF>(d, fwd ? t : ng - 1 - t, r0, shp, shl, gpar, gsum, lane);
    if (t + 1 < ng) apply_gate<VEC, PMAX, OVF>(d, fwd ? t + 1 : ng - 2 - t, r1, shp, shl, gpar, gsum, lane);
    if (t + 2 < ng) apply_gate<VEC, PMAX, OVF>(d, fwd ? t + 2 : ng - 3 - t, r2, shp, shl, gpar, gsum, lane);
    if (!fwd)
        for (int jl = lane; jl < ng; jl += 64)
            d.part_g[size_t(d.run.g0 + jl) * d.gstride + d.item.tile] = gsum[jl];
}

template <int VEC, int PMAX, bool OVF>
__global__ void __launch_bounds__(64) k_pq(PqArgs a) {
    extern __shared__ double2 sh[];
    __shared__ HxTables T;
    const int lane = threadIdx.x;
    {
        const uint32_t* src = reinterpret_cast<const uint32_t*>(a.tabs);
        uint32_t* dst = reinterpret_cast<uint32_t*>(&T);
        for (int i = lane; i < int(sizeof(HxTables) / 4); i += 64) dst[i] = src[i];
    }
    wave_lds_fence();
    const int q = ldc(a.qmap + (xcc_id() & (kPqMaxXcc - 1)));
    if (q < 0) return;
    const int i0 = ldc(a.qoff + q), n_items = ldc(a.qoff + q + 1) - i0;
    const int spin_limit = ldc(a.ctl);
    double2* shp = sh;
    double2* shl = sh + a.cap;
    double2* gpar = sh + size_t(VEC) * a.cap;
    double* gsum = reinterpret_cast<double*>(gpar + 2 * a.max_ng);
    // items are taken kPqBatch at a time (one atomic per batch); the atomic
    // for the next batch is issued when the current batch's last item starts,
    // and its result is read after that item's gates
    auto take = [&]() {
        int v = 0;
        if (lane == 0) v = __hip_atomic_fetch_add(a.head + q, kPqBatch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return v;
    };
    int cur = __builtin_amdgcn_readfirstlane(take());
    if (cur >= n_items) return;
    int end = min(cur + kPqBatch, n_items);
    PqTile d;
    load_tile(a, T, i0 + cur, d);
    if (!wait_dep(a, q, d.item, spin_limit, lane)) return;
    if (!d.empty) stage<VEC>(d, shp, shl, gpar, lane);
    int pending = -1;   // state of a finished item whose completion is not yet published
    for (;;) {
        const bool last = cur + 1 >= end;
        const int ticket = last ? take() : 0;
        wait_vm0();                  // this tile staged; the previous tile's stores acknowledged
        if (pending >= 0) publish(a, pending, lane);
        pending = -1;
        wave_lds_fence();
        if (!d.empty) {
            run_gates<VEC, PMAX, OVF>(d, shp, shl, gpar, gsum, lane);
            const int nE = d.tb.nE;
            for (int k = lane; k < nE; k += 64) {
                const int64_t gi = tile_global(d.tb, d.run.nblk, k);
                stg2(d.phi + gi, shp[k]);
                if (VEC == 2) stg2(d.lam + gi, shl[k]);
            }
        } else if (VEC == 2) {   // an empty tile: zero gradient partials
            const int ng = d.run.g1 - d.run.g0;
            for (int jl = lane; jl < ng; jl += 64)
                d.part_g[size_t(d.run.g0 + jl) * d.gstride + d.item.tile] = 0.0;
        }
        pending = d.item.state;
        if (last) {
            cur = __builtin_amdgcn_readfirstlane(ticket);
            if (cur >= n_items) break;
            end = min(cur + kPqBatch, n_items);
        } else {
            ++cur;
        }
        load_tile(a, T, i0 + cur, d);
        if (d.item.need > 0 && ld_counter(a.done + d.item.state) < d.item.need) {
            // it must wait: publish the finished item first (it may be the one awaited)
            wait_vm0();
            publish(a, pending, lane);
            pending = -1;
            if (!wait_dep(a, q, d.item, spin_limit, lane)) return;
        }
        // the LDS reads of the stores above have completed before their
        // stores issued; the next tile may overwrite LDS
        wave_lds_fence();
        if (!d.empty) stage<VEC>(d, shp, shl, gpar, lane);
    }
    wait_vm0();
    if (pending >= 0) publish(a, pending, lane);
}

__global__ void k_pq_reset(int32_t* p, int n) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0;
}

// Raw XCC id of each workgroup of a probe launch.
__global__ void k_xcc_probe(int32_t* out) {
    if (threadIdx.x == 0) out[blockIdx.x] = int32_t(xcc_id());
}

using PqKernel = void (*)(PqArgs);

// pmax 1, 2, 4, 8: pair slots per lane; 9: eight slots and a loop for the rest
template <int VEC>
static PqKernel pq_kernel(int pmax) {
    switch (pmax) {
        case 1: return &k_pq<VEC, 1, false>;
        case 2: return &k_pq<VEC, 2, false>;
        case 4: return &k_pq<VEC, 4, false>;
        case 8: return &k_pq<VEC, 8, false>;
        default: return &k_pq<VEC, 8, true>;
    }
}

int pq_pmax_for(int max_stride) {
    const int per_lane = (max_stride + 63) / 64;
    return per_lane <= 1 ? 1 : per_lane <= 2 ? 2 : per_lane <= 4 ? 4 : per_lane <= 8 ? 8 : 9;
}

int pq_prepare(int vec, int pmax, size_t lds_bytes, int* blocks_per_cu) {
    const void* f = reinterpret_cast<const void*>(vec == 1 ? pq_kernel<1>(pmax) : pq_kernel<2>(pmax));
    if (lds_bytes > (64u << 10) &&
        hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, int(lds_bytes)) != hipSuccess)
        return 1;
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, f, 64, lds_bytes) != hipSuccess || nb < 1) return 1;
    *blocks_per_cu = nb;
    return 0;
}

void launch_pq(int vec, int pmax, const PqArgs& a, int grid, size_t lds_bytes, hipStream_t st) {
    if (vec == 1)
        hipLaunchKernelGGL(pq_kernel<1>(pmax), dim3(grid), dim3(64), lds_bytes, st, a);
    else
        hipLaunchKernelGGL(pq_kernel<2>(pmax), dim3(grid), dim3(64), lds_bytes, st, a);
}

void launch_pq_reset(int32_t* p, int n, hipStream_t st) {
    hipLaunchKernelGGL(k_pq_reset, dim3(std::max(1, std::min(64, (n + 255) / 256))), dim3(256), 0, st, p, n);
}

void launch_xcc_probe(int32_t* out, int blocks, hipStream_t st) {
    hipLaunchKernelGGL(k_xcc_probe, dim3(blocks), dim3(64), 0, st, out);
}

}  // namespace vqe
