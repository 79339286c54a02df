// Ansatz kernels on the packed sector layout (Sec. 2.1.2; the objective of
// Sec. 2.1.1, Eq. 1, and its gradient by the reverse sweep).
//
// Every UCCSD gate conserves the alpha and beta electron counts, so a state
// prepared from the reference |HF> has nonzero amplitudes only in the
// reference's (N, S_z) sector.  The packed layout stores exactly those
// amplitudes: strings b are grouped in blocks by their high bits h = b >> L,
// block h holds the in-sector strings with that high part ordered by
// (rank of the low alpha string, rank of the low beta string) among strings
// of their popcounts, and blocks follow each other in increasing h from
// base[h].  Empty blocks take no space.  The reference is entry 0.
//
// L is at least the number of electrons, so the reference lies in block 0.
// A gate pairs D (annihilated orbitals occupied, created ones empty) with
// E = D ^ x.  Consecutive gates whose high orbitals (the annihilated and
// created ones above the block bits) fit a window of at most 4 high bits form
// a run, applied tile by tile: a tile is the set of blocks whose high parts
// agree outside the window (those the run's gates pair), staged in LDS one
// after the other, all the run's gates applied, written back.  For UCCSD on
// the reference the occupied orbitals are low, so D and E differ in the
// high bits of the created orbitals only; generalised excitations may also
// annihilate high orbitals.
#include <type_traits>
#include <utility>

#include "device_common.h"

namespace vqe {

// Calls f(std::integral_constant<int, i>) for i = 0 .. N-1 in order (the
// bodies see i as a constant).
template <typename F, int... I>
__device__ __forceinline__ void unroll_each(F&& f, std::integer_sequence<int, I...>) {
    (f(std::integral_constant<int, I>{}), ...);
}
template <int N, typename F>
__device__ __forceinline__ void unroll_n(F&& f) {
    unroll_each(f, std::make_integer_sequence<int, N>{});
}

template <typename V>
__global__ void k_packed_hf(const StateDesc* __restrict__ sd, int64_t size) {
    const StateDesc& s = sd[blockIdx.y];
    V* phi = reinterpret_cast<V*>(s.phi);
    for (int64_t k = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; k < size;
         k += int64_t(gridDim.x) * blockDim.x)
        nt_store(phi + k, k == 0 ? vunit(V{}) : vzero<V>());
}

// VEC = 1: forward pass on phi.  VEC = 2: reverse sweep on phi and lambda
// with per-gate, per-tile partials of Re <lambda|A_j phi> (A_j = T_j - T_j^dag).
// V: amplitude type (double2, or double for real states).
// Tile entry k (blocks one after the other) is staged by thread k % BS
// (2 EPT BS covers the largest tile of the run); a gate's pairs come from the
// run's precomputed list for the tile's class, one pair per thread per pass.
// The tile's geometry is its host-built descriptor (one scalar read), so the
// tile loads, the gate parameters and the first list entries are all in
// flight together before the first wait.
template <int VEC, int BS, int EPT, typename V>
__global__ void __launch_bounds__(BS) k_prun(const StateDesc* __restrict__ sd, PackedRun run,
                                             const PackedGate* __restrict__ pg) {
    extern __shared__ double2 sh[];
    constexpr int kRedGates = 8;                            // gates per batch of wave totals
    constexpr int kListAhead = 4;                           // list prefetch distance (gates)
    static_assert(kRedGates % kListAhead == 0, "a batch of wave totals starts at slot 0");
    __shared__ double red[2][VEC == 2 ? kRedGates : 1][BS / 64];   // wave totals of the last two batches
    __shared__ double gsum[VEC == 2 ? kMaxRunGates : 1];   // per-gate tile totals
    const StateDesc& s = sd[blockIdx.y];
    // both passes cover the run's live tiles only (all of them without a list);
    // gradient partials go to the tile's position in the launch
    const TileDesc tb = ldc(run.tdesc + blockIdx.x);
    const int po = int(blockIdx.x);
    const int tid = threadIdx.x;
    if (tb.nE == 0) {   // an empty tile: zero gradient partials
        if (VEC == 2)
            for (int jl = tid; jl < run.g1 - run.g0; jl += BS)
                s.part_g[size_t(run.g0 + jl) * s.gstride + po] = 0.0;
        return;
    }
    const int nE = tb.nE;
    const uint32_t hb0 = tb.hbase << run.L;
    V* shp = reinterpret_cast<V*>(sh);
    V* shl = shp + nE;
    // the reverse sweep on real amplitudes keeps (phi, lambda) of an entry
    // side by side, so that a pair's four values take two 16-byte LDS reads
    // and two writes
    constexpr bool kPL = VEC == 2 && std::is_same<V, double>::value;
    double2* shpl = sh;
    const bool fwd = (VEC == 1);
    const int ng = run.g1 - run.g0;
    const int cls = tb.cls;
    // the tile class's pair lists: gate j's list at lbase + j * stride, padded
    // with kPairNone.  Each thread's first entry of a gate is loaded kListAhead
    // gates ahead (the first kListAhead before the tile loads) into slot
    // t % kListAhead of eq; the gate loops are unrolled so that every slot
    // index is a constant, so a gate waits only for its own entry's load and
    // the list reads' latency overlaps kListAhead gate steps
    const int2 lc = ldc(run.info + cls);
    const uint32_t* lbase = run.ent + lc.x;
    const int stride = lc.y;
    // the loads go through a buffer resource bounded to the class's lists and
    // are issued unconditionally for a clamped gate (reads past the lists
    // return 0); a slot is checked only when its gate takes it (a thread past
    // the list's length has no entry), so the compiler can wait for that
    // slot's load alone while the later ones stay in flight
    const __amdgpu_buffer_rsrc_t lrs = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<uint32_t*>(lbase), 0, int(uint32_t(ng) * uint32_t(stride) * 4u), 0x00020000);
    const bool has_slot = tid < stride;
    auto list_first = [&](int j) -> uint32_t {   // raw: the thread's first entry of gate j
        const int jc = j < 0 ? 0 : (j >= ng ? ng - 1 : j);
        return __builtin_amdgcn_raw_buffer_load_b32(lrs, uint32_t(jc * stride + tid) * 4u, 0, 0);
    };
    uint32_t eq[kListAhead];
#pragma unroll
    for (int d = 0; d < kListAhead; ++d) eq[d] = list_first(fwd ? d : ng - 1 - d);
    // per-gate parameters of this tile after the tile (2 double2 per gate):
    // (cos, sgn sin) and (sgn, 0), sgn the gate's pair sign from the tile's
    // high bits outside the window (the window's part is in each entry);
    // staged once; the first is read by broadcast in the gate loop, the
    // second (reverse sweep) applied to the gate's tile total at the end
    double2* gpar = sh + (size_t(VEC) * run.max_entries * sizeof(V) + 15) / 16;
    // the state index of each staged entry, kept for the write-back
    int gix[2 * EPT];
    {   // all loads first (clamped into the tile), then the LDS stores
        V vp[2 * EPT], vl[2 * EPT];
#pragma unroll
        for (int u = 0; u < 2 * EPT; ++u) {
            gix[u] = tile_index(tb, run.nblk, min(tid + BS * u, nE - 1));
            vp[u] = ldgv(reinterpret_cast<const V*>(s.phi) + gix[u]);
            if (VEC == 2) vl[u] = ldgv(reinterpret_cast<const V*>(s.lam) + gix[u]);
        }
        for (int j = tid; j < ng; j += BS) {
            const PackedGate g = pg[j];
            const double2 cs = s.cs[run.g0 + j];
            const double sgn = g.csign * parity_sign(hb0 & g.chhi);
            gpar[2 * j] = make_double2(cs.x, sgn * cs.y);
            gpar[2 * j + 1] = make_double2(sgn, 0.0);
        }
        // unconditional stores (a clamped slot rewrites the last entry with its
        // own value), so that every load is waited for on every path
#pragma unroll
        for (int u = 0; u < 2 * EPT; ++u) {
            const int k = min(tid + BS * u, nE - 1);
            if constexpr (kPL) {
                shpl[k] = make_double2(vp[u], vl[u]);
            } else {
                shp[k] = vp[u];
                if (VEC == 2) shl[k] = vl[u];
            }
        }
    }
    __syncthreads();
    // forward pass: the next gate's (cos, sgn sin) is read at the start of the
    // current gate, so that only pair data follows the barrier (measured: the
    // forward runs 4% faster, the reverse sweep, which reads the sign too, 5%
    // slower, so it reads its parameters after the barrier)
    double2 cs_ahead = gpar[0];
    // one gate: its pairs (one per thread per pass), returning the thread's
    // part of the reverse sweep's Re <lambda|A_j phi>; the slot's entry for
    // gate t + kListAhead is loaded meanwhile.  LONG (a list longer than the
    // block): the thread's later entries are read in the gate itself; the
    // gate loops are built separately for the two cases, so that the common
    // one has no other list reads than the slots'
    auto gate_step = [&](int t, auto slot, auto long_tag) -> double {
        constexpr int q = decltype(slot)::value;   // t % kListAhead
        constexpr bool LONG = decltype(long_tag)::value;
        const int jl = fwd ? t : ng - 1 - t;
        const int jn = fwd ? jl + kListAhead : jl - kListAhead;
        const uint32_t ecur = has_slot ? eq[q] : kPairNone;
        const double2 cs = VEC == 1 ? cs_ahead : gpar[2 * jl];   // (cos, sgn sin)
        const double ssin = cs.y;
        if (VEC == 1) cs_ahead = gpar[2 * (jl + 1 < ng ? jl + 1 : jl)];
        double acc = 0.0;
        for (int i = tid; i < (LONG ? stride : tid + 1); i += BS) {
            const uint32_t e = (i == tid) ? ecur : ldg32(lbase + size_t(jl) * stride + i);
            if (e == kPairNone) break;   // the padding: the rest of the list is padding too
            const int k = int(e & kEntMask), ie = int((e >> kEntBits) & kEntMask);
            const double ss = ((e >> kEntParity) & 1u) ? -ssin : ssin;
            if (fwd) {
                V d = shp[k], f = shp[ie];
                givens(d, f, cs.x, ss);
                shp[k] = d;
                shp[ie] = f;
            } else {
                V fD, fE, lD, lE;
                if constexpr (kPL) {
                    const double2 pD = shpl[k], pE = shpl[ie];
                    fD = pD.x;
                    lD = pD.y;
                    fE = pE.x;
                    lE = pE.y;
                } else {
                    fD = shp[k];
                    fE = shp[ie];
                    lD = shl[k];
                    lE = shl[ie];
                }
                // <lam| A phi> with A|D> = s|E>, A|E> = -s|D> (s = ss / sin)
                // the entry's part of the sign here; the tile's (a factor of
                // +-1 common to the gate) when the tile's total is stored
                const double dv = redot(lE, fD) - redot(lD, fE);
                acc += ((e >> kEntParity) & 1u) ? -dv : dv;
                givens(fD, fE, cs.x, -ss);   // U^dag: rotation by -theta
                givens(lD, lE, cs.x, -ss);
                if constexpr (kPL) {
                    shpl[k] = make_double2(fD, lD);
                    shpl[ie] = make_double2(fE, lE);
                } else {
                    shp[k] = fD;
                    shp[ie] = fE;
                    shl[k] = lD;
                    shl[ie] = lE;
                }
            }
        }
        // the slot's next entry, issued once this gate's entry is dead (so
        // that it can take the same register)
        eq[q] = list_first(jn);
        __syncthreads();
        return acc;
    };
    // Whole rounds of slots (and whole batches of wave totals) run without
    // per-gate bounds, so every one issues the same loads and a gate waits for
    // its own slot only; the last, partial one checks each gate.
    if (fwd) {
        auto gates = [&](auto long_tag) {
            int t0 = 0;
            for (; t0 + kListAhead <= ng; t0 += kListAhead)
                unroll_n<kListAhead>([&](auto slot) {
                    (void)gate_step(t0 + decltype(slot)::value, slot, long_tag);
                });
            unroll_n<kListAhead>([&](auto slot) {
                if (t0 + decltype(slot)::value < ng) (void)gate_step(t0 + decltype(slot)::value, slot, long_tag);
            });
        };
        if (stride > BS) gates(std::true_type{});
        else gates(std::false_type{});
    } else {
        // the wave totals of kRedGates consecutive gates are taken together
        // after them (wave_totals8: off the per-gate barrier path); thread
        // u < kRedGates adds the waves of gate u of the previous batch once a
        // barrier has passed since they were written
        static_assert(kRedGates == 8, "wave_totals8 takes eight gates");
        auto batch = [&](int t0, auto long_tag, auto full_tag) {
            constexpr bool FULL = decltype(full_tag)::value;
            double acc[kRedGates];
            unroll_n<kRedGates>([&](auto uu) {
                constexpr int u = decltype(uu)::value;
                acc[u] = 0.0;
                if (FULL || t0 + u < ng) {
                    acc[u] = gate_step(t0 + u, std::integral_constant<int, u % kListAhead>{}, long_tag);
                    if (u == 0 && t0 > 0 && tid < kRedGates) {
                        const int tp = t0 - kRedGates + tid;
                        double v = 0.0;
#pragma unroll
                        for (int w = 0; w < BS / 64; ++w) v += red[(t0 / kRedGates - 1) & 1][tid][w];
                        gsum[ng - 1 - tp] = v;
                    }
                }
            });
            const double tot = wave_totals8(acc, tid & 63);
            if ((tid & 7) == 0) red[(t0 / kRedGates) & 1][(tid & 63) >> 3][tid >> 6] = tot;
        };
        auto gates = [&](auto long_tag) {
            int t0 = 0;
            for (; t0 + kRedGates <= ng; t0 += kRedGates) batch(t0, long_tag, std::true_type{});
            if (t0 < ng) batch(t0, long_tag, std::false_type{});
        };
        if (stride > BS) gates(std::true_type{});
        else gates(std::false_type{});
        __syncthreads();
        {
            const int t0 = (ng - 1) / kRedGates * kRedGates;   // the last batch
            if (tid < kRedGates && t0 + tid < ng) {
                double v = 0.0;
#pragma unroll
                for (int w = 0; w < BS / 64; ++w) v += red[(t0 / kRedGates) & 1][tid][w];
                gsum[ng - 1 - (t0 + tid)] = v;
            }
        }
        __syncthreads();
        for (int jl = tid; jl < ng; jl += BS)
            s.part_g[size_t(run.g0 + jl) * s.gstride + po] = gsum[jl] * gpar[2 * jl + 1].x;
    }
#pragma unroll
    for (int u = 0; u < 2 * EPT; ++u) {
        const int k = tid + BS * u;
        if (k < nE) {
            if constexpr (kPL) {
                const double2 pl = shpl[k];
                stgv(reinterpret_cast<double*>(s.phi) + gix[u], pl.x);
                stgv(reinterpret_cast<double*>(s.lam) + gix[u], pl.y);
            } else {
                stgv(reinterpret_cast<V*>(s.phi) + gix[u], shp[k]);
                if (VEC == 2) stgv(reinterpret_cast<V*>(s.lam) + gix[u], shl[k]);
            }
        }
    }
}

// Zero-angle reverse sweep of a gate pool (ADAPT-VQE pool gradients): every
// gate at angle 0 is the identity, so phi and lambda are only read and the
// gates are independent.  One launch covers every (run, tile): block b works
// on tile b - blk0[r] of run r = blk_run[b]; after staging the tile, each
// wave takes whole gates (w, w + BS/64, ...) and its 64 lanes split the
// gate's pair list, so a gate's tile partial of Re <lambda|A_j phi> is one
// wave total, stored without a block barrier.
template <int BS, int EPT, typename V>
__global__ void __launch_bounds__(BS) k_ppool(const StateDesc* __restrict__ sd,
                                              const PackedRun* __restrict__ runs,
                                              const int32_t* __restrict__ blk_run,
                                              const int32_t* __restrict__ blk0,
                                              const PackedGate* __restrict__ pg_all,
                                              const HxTables* __restrict__ tabsrc,
                                              const int32_t* __restrict__ base) {
    extern __shared__ double2 sh[];
    __shared__ HxTables T;
    {
        const uint32_t* src = reinterpret_cast<const uint32_t*>(tabsrc);
        uint32_t* dst = reinterpret_cast<uint32_t*>(&T);
        for (int i = threadIdx.x; i < int(sizeof(HxTables) / 4); i += BS) dst[i] = src[i];
    }
    __syncthreads();
    const StateDesc& s = sd[blockIdx.y];
    const int r = ldc(blk_run + blockIdx.x);
    const PackedRun run = ldc(runs + r);
    const int o = int(blockIdx.x) - ldc(blk0 + r);
    const int tid = threadIdx.x, lane = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int ng = run.g1 - run.g0;
    TileBlocks tb;
    tile_blocks(T, run, o, base, tb);
    if (tb.nE == 0) {
        for (int jl = tid; jl < ng; jl += BS) s.part_g[size_t(run.g0 + jl) * s.gstride + o] = 0.0;
        return;
    }
    const int nE = tb.nE;
    const uint32_t hb0 = tb.hbase << run.L;
    V* shp = reinterpret_cast<V*>(sh);
    V* shl = shp + nE;
    {
        V vp[2 * EPT], vl[2 * EPT];
#pragma unroll
        for (int u = 0; u < 2 * EPT; ++u) {
            const int k = min(tid + BS * u, nE - 1);
            const int64_t gi = tile_global(tb, run.nblk, k);
            vp[u] = ldgv(reinterpret_cast<const V*>(s.phi) + gi);
            vl[u] = ldgv(reinterpret_cast<const V*>(s.lam) + gi);
        }
#pragma unroll
        for (int u = 0; u < 2 * EPT; ++u) {
            const int k = min(tid + BS * u, nE - 1);
            shp[k] = vp[u];
            shl[k] = vl[u];
        }
    }
    __syncthreads();
    const int cls = tb.cls;
    const PackedGate* pg = pg_all + run.g0;
    const int2 lc = ldc(run.info + cls);
    for (int jl = w; jl < ng; jl += BS / 64) {
        const uint32_t* lst = run.ent + lc.x + size_t(jl) * lc.y;
        const PackedGate g = ldc(pg + jl);
        const double sgn_hi = g.csign * parity_sign(hb0 & g.chhi);
        double acc = 0.0;
        for (int i = lane; i < lc.y; i += 64) {
            const uint32_t e = ldg32(lst + i);
            if (e == kPairNone) break;
            const int k = int(e & kEntMask), ie = int((e >> kEntBits) & kEntMask);
            const double sg_t = ((e >> kEntParity) & 1u) ? -sgn_hi : sgn_hi;
            const V fD = shp[k], fE = shp[ie], lD = shl[k], lE = shl[ie];
            acc += sg_t * (redot(lE, fD) - redot(lD, fE));
        }
        acc = wave_total(acc);
        if (lane == 0) s.part_g[size_t(run.g0 + jl) * s.gstride + o] = acc;
    }
}

// Launch shapes (threads per tile, entries per thread).
#define VQE_PACKED_SHAPES(X)                                                                  \
    X(64, 1) X(64, 2) X(64, 4) X(64, 8) X(256, 1) X(256, 2) X(256, 3) X(256, 5) X(512, 1)     \
    X(512, 2) X(512, 3) X(1024, 1) X(1024, 2)

struct PShape {
    int bs, ept;
};
#define VQE_SHAPE_ENTRY(B, E) {B, E},
constexpr PShape kPShapes[] = {VQE_PACKED_SHAPES(VQE_SHAPE_ENTRY)};
#undef VQE_SHAPE_ENTRY
constexpr int kNumPShapes = int(sizeof(kPShapes) / sizeof(kPShapes[0]));

int packed_shape(int max_block, int min_threads) {
    int best = -1;
    for (int pass = 0; pass < 2 && best < 0; ++pass)   // second pass: any thread count
        for (int i = 0; i < kNumPShapes; ++i) {
            const PShape& p = kPShapes[i];
            if ((pass == 0 && p.bs < min_threads) || p.bs * p.ept < max_block) continue;
            if (best < 0 || p.bs * p.ept < kPShapes[best].bs * kPShapes[best].ept) best = i;
        }
    return best;
}

int packed_shape_threads(int shape) { return kPShapes[shape].bs; }

using PackedLauncher = void (*)(const StateDesc*, int, const PackedRun&, const PackedGate*, hipStream_t);

template <int VEC, int BS, int EPT, typename V>
static void launch_one(const StateDesc* sd, int count, const PackedRun& run, const PackedGate* pg,
                       hipStream_t st) {
    // the tile's amplitudes (16-byte aligned), then 2 double2 per gate
    const size_t lds = (size_t(run.max_entries) * VEC * sizeof(V) + 15) / 16 * 16 +
                       2 * size_t(run.g1 - run.g0) * sizeof(double2);
    const int nx = run.live ? run.nlive : run.ntiles;
    if (nx == 0) return;   // a run with no live tile: nothing to do, no partials
    hipLaunchKernelGGL((k_prun<VEC, BS, EPT, V>), dim3(nx, count), dim3(BS), lds, st, sd, run, pg);
}

#define VQE_FWD_ENTRY(B, E) &launch_one<1, B, E, double2>,
#define VQE_ADJ_ENTRY(B, E) &launch_one<2, B, E, double2>,
#define VQE_FWD_REAL(B, E) &launch_one<1, B, E, double>,
#define VQE_ADJ_REAL(B, E) &launch_one<2, B, E, double>,
static const PackedLauncher kFwdLaunch[] = {VQE_PACKED_SHAPES(VQE_FWD_ENTRY)};
static const PackedLauncher kAdjLaunch[] = {VQE_PACKED_SHAPES(VQE_ADJ_ENTRY)};
static const PackedLauncher kFwdLaunchR[] = {VQE_PACKED_SHAPES(VQE_FWD_REAL)};
static const PackedLauncher kAdjLaunchR[] = {VQE_PACKED_SHAPES(VQE_ADJ_REAL)};
#undef VQE_FWD_ENTRY
#undef VQE_ADJ_ENTRY
#undef VQE_FWD_REAL
#undef VQE_ADJ_REAL

void launch_packed_run(const StateDesc* sd, int count, const PackedRun& run, const PackedGate* pg,
                       bool adjoint, bool real, hipStream_t st) {
    if (adjoint)
        (real ? kAdjLaunchR : kAdjLaunch)[run.shape_adj](sd, count, run, pg, st);
    else
        (real ? kFwdLaunchR : kFwdLaunch)[run.shape](sd, count, run, pg, st);
}

using PoolLauncher = void (*)(const StateDesc*, int, const PoolSweep&, const HxTables*,
                              const int32_t*, hipStream_t);

template <int BS, int EPT, typename V>
static void launch_pool_one(const StateDesc* sd, int count, const PoolSweep& ps,
                            const HxTables* tabs, const int32_t* base, hipStream_t st) {
    hipLaunchKernelGGL((k_ppool<BS, EPT, V>), dim3(ps.nblk, count), dim3(BS), ps.lds, st, sd, ps.runs,
                       ps.blk_run, ps.blk0, ps.gates, tabs, base);
}

#define VQE_POOL_ENTRY(B, E) &launch_pool_one<B, E, double2>,
#define VQE_POOL_REAL(B, E) &launch_pool_one<B, E, double>,
static const PoolLauncher kPoolLaunch[] = {VQE_PACKED_SHAPES(VQE_POOL_ENTRY)};
static const PoolLauncher kPoolLaunchR[] = {VQE_PACKED_SHAPES(VQE_POOL_REAL)};
#undef VQE_POOL_ENTRY
#undef VQE_POOL_REAL

void launch_pool_sweep(const StateDesc* sd, int count, const PoolSweep& ps, const HxTables* tabs,
                       const int32_t* base, bool real, hipStream_t st) {
    if (ps.nblk > 0) (real ? kPoolLaunchR : kPoolLaunch)[ps.shape](sd, count, ps, tabs, base, st);
}

void launch_packed_hf(const StateDesc* sd, int count, int64_t size, bool real, hipStream_t st) {
    const int nblk = blocks_for(uint64_t(size));
    if (real)
        hipLaunchKernelGGL(k_packed_hf<double>, dim3(nblk, count), dim3(kBlock), 0, st, sd, size);
    else
        hipLaunchKernelGGL(k_packed_hf<double2>, dim3(nblk, count), dim3(kBlock), 0, st, sd, size);
}

int packed_enable_lds(size_t bytes) {
    hipError_t e = hipSuccess;
    auto set = [&](const void* f) {
        hipError_t r = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, int(bytes));
        if (r != hipSuccess) e = r;
    };
#define VQE_SET_ENTRY(B, E)                                                 \
    set(reinterpret_cast<const void*>(&k_prun<1, B, E, double2>));          \
    set(reinterpret_cast<const void*>(&k_prun<2, B, E, double2>));          \
    set(reinterpret_cast<const void*>(&k_ppool<B, E, double2>));            \
    set(reinterpret_cast<const void*>(&k_prun<1, B, E, double>));           \
    set(reinterpret_cast<const void*>(&k_prun<2, B, E, double>));           \
    set(reinterpret_cast<const void*>(&k_ppool<B, E, double>));
    VQE_PACKED_SHAPES(VQE_SET_ENTRY)
#undef VQE_SET_ENTRY
    return e == hipSuccess ? 0 : 1;
}

}  // namespace vqe
