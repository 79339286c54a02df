// Host glue of the device path: device copies of Hamiltonians and ansatz
// programs, launch plans, workspaces, the batched HIP-graph evaluation and
// the device-side C-ABI entry points.  Kernels live in k_gates.hip and
// k_hamiltonian.hip.
//
// One evaluation of E(theta) and dE/dtheta (Sec. 2.1.1, Eq. 1; UCCSD of
// Sec. 2.1.2) is the launch sequence
//   angles -> |HF> -> forward gate steps -> H-apply + energy partials
//          -> reverse gate steps (adjoint) -> energy and gradient reductions.
// Forward and reverse gate steps are fused tile passes over runs of
// excitations (or single per-gate launches for explicit Pauli rotations).
// The H-apply is restricted to the (N, S_z) sector of the reference whenever
// every gate conserves both counts; for UCCSD programs the whole evaluation
// then runs on the packed sector layout (k_packed.hip), which stores only the
// in-sector amplitudes.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <memory>
#include <tuple>

#include "device_common.h"

namespace vqe {

int enable_large_lds(size_t bytes);   // k_gates.hip

#define HIPCHK(expr)                                                                        \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess)                                                               \
            return fail(VQE_EDEVICE, std::string("HIP error in ") + #expr + ": " +         \
                                         hipGetErrorString(e_));                            \
    } while (0)

// ------------------------------------------------------------------ tuning

// Launch parameters of one (qubit count, batched or single) configuration.
struct Tuning {
    int64_t fwd_budget;   // LDS bytes of a forward run tile
    int64_t adj_budget;   // LDS bytes of a reverse run tile (phi + lambda)
    int L;                // low-bit tile of the sector H-apply
    int fwd_threads = 64; // packed layout: least threads per forward run tile
    int adj_threads = 64; // packed layout: least threads per reverse run tile
    int tile_cap = 0;     // packed layout: entries per run tile (0: two of the largest blocks)
};

static std::mutex g_tune_mu;
static std::map<std::pair<int, int>, Tuning> g_tune;   // (n, batched) -> override
static std::map<std::pair<int, int>, std::pair<int, int>> g_threads;   // -> run threads
static std::map<std::pair<int, int>, int> g_tile_cap;   // -> entries per run tile

static Tuning default_tuning(int n, bool batched) {
    Tuning t;
    t.fwd_budget = (n >= 22) ? (128 << 10) : (64 << 10);
    t.adj_budget = (n >= 21) ? (128 << 10) : (64 << 10);
    int L = std::min(n, kHxMaxL);
    if (!batched) {
        // a single state: 12 block bits (the packed layout raises L to n_e when
        // that is more) and 256-thread run tiles, measured best or within 1.5%
        // of the best for single UCCSD states of 16 to 24 qubits (8-27% faster
        // than the batch defaults there)
        L = std::min(n, 12);
        t.fwd_threads = t.adj_threads = 256;
    }
    t.L = L;
    return t;
}

static Tuning tuning_for(int n, bool batched) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune.find({n, batched ? 1 : 0});
    Tuning t = default_tuning(n, batched);   // an override replaces the budgets and L only
    if (it != g_tune.end()) {
        t.fwd_budget = it->second.fwd_budget;
        t.adj_budget = it->second.adj_budget;
        t.L = it->second.L;
    }
    auto th = g_threads.find({n, batched ? 1 : 0});
    if (th != g_threads.end()) {
        t.fwd_threads = th->second.first;
        t.adj_threads = th->second.second;
    }
    auto tc = g_tile_cap.find({n, batched ? 1 : 0});
    if (tc != g_tile_cap.end()) t.tile_cap = tc->second;
    return t;
}

// ------------------------------------------------------------ device copies

struct AnsatzPlan {
    int64_t fwd_budget = 0, adj_budget = 0;
    // step: kind 0 = fused run (index into runs), kind 1 = single gate (gate index)
    std::vector<std::pair<int, int>> fwd_steps, adj_steps;
    std::vector<RunDesc> fwd_runs, adj_runs;
    std::vector<int> fwd_off, adj_off;   // TileGate offset per run
    TileGate* d_fwd_tg = nullptr;
    TileGate* d_adj_tg = nullptr;
    std::vector<int32_t> gcnt;           // gradient partials per gate
    int32_t* d_gcnt = nullptr;
    int32_t gstride = 1;
    size_t max_lds = 0;
    // algorithmic traffic of one evaluation (bytes) from the tile geometry
    double fwd_bytes = 0.0, adj_bytes = 0.0;
};

// String-product H-apply plan of a Hamiltonian (groups sorted into classes
// by the alpha part of their flip mask; see k_hx_ci.hip).
struct CiSpace;

// Row-move groups of a Hamiltonian (host) and their per-row lists for one
// alpha-string space (device).
struct RowMoveGroup {
    uint32_t xa = 0, tba = 0, wa = 0, wb = 0;
    std::vector<double> tab;   // by alpha pattern of the table positions
};
struct RowMoves {
    CiRowMove* d_rm = nullptr;
    int32_t* d_off = nullptr;
};
struct ColMoveGroup {
    uint32_t xb = 0, tbb = 0, wa = 0, wb = 0;   // tbb: compact beta table positions (mask)
    std::vector<double> tab;                    // by beta pattern of the table positions
};
struct ColMoves {
    CiColMove* d_cm = nullptr;
    int ncm = 0;
};
struct BetaHopGroup {
    int pair = 0;                           // pair index of its two beta orbitals
    uint32_t xb = 0, lo = 0, hi = 0, wa0 = 0, wb0 = 0;
    double S[4] = {0, 0, 0, 0};             // by beta pattern (bit 0: orbital lo)
    std::vector<double> Tb, Ta;             // -2 T_t, [orbital][4]
};
struct BetaHops {
    CiBetaHop* d_bh = nullptr;
    int nbh = 0;
};
struct AlphaHopGroup {
    int pair = 0;                           // pair index of its two alpha orbitals
    uint32_t xa = 0, lo = 0, hi = 0, wa0 = 0, wb0 = 0;
    double S[4] = {0, 0, 0, 0};             // by alpha pattern (bit 0: orbital lo)
    std::vector<double> Ta, Tb;             // -2 T_t, [orbital][4]
};
struct AlphaHops {
    CiAlphaHop* d_ah = nullptr;
    int32_t* d_off = nullptr;
    double* d_b = nullptr;
};
// The diagonal group in occupation form: K + sum_t L_t n_t + sum_{t<u} Q_tu n_t n_u
// (its Z_t and Z_t Z_u strings with Z = 1 - 2n), and its row and column parts
// for one string space.
struct DiagForm {
    bool on = false;
    double K = 0.0;
    std::vector<double> L, Q;   // [n], [n][n] (t < u)
};
struct DiagParts {
    double* d_row = nullptr;
    double* d_col = nullptr;
};

struct CiHam {
    std::vector<RowMoveGroup> rmg;
    std::map<const CiSpace*, RowMoves*> rm;        // by string space
    std::vector<ColMoveGroup> cmg;
    std::map<const CiSpace*, ColMoves*> cm;
    std::vector<BetaHopGroup> bhg;
    double* d_hopa = nullptr;                      // alpha tables of the beta hops
    std::map<const CiSpace*, BetaHops*> bh;
    std::vector<AlphaHopGroup> ahg;
    std::map<const CiSpace*, AlphaHops*> ah;
    DiagForm diag;
    double* d_dgx = nullptr;                       // alpha-beta pair coefficients [alpha][16]
    std::map<const CiSpace*, DiagParts*> dg;
    CiChunk* chunks = nullptr;
    CiGroup* groups = nullptr;
    CiSub* subs = nullptr;
    double* tabs = nullptr;
    int nchunks = 0;
    int ob = 0;   // beta orbitals the pair records are laid out for
    CiPairClass* pcls = nullptr;
    CiPairRec* precs = nullptr;
    CiGroup* rgroups = nullptr;
    CiSub* rsubs = nullptr;
    double* ptabs = nullptr;
    double2* pcoef = nullptr;   // pair coefficients by class, alpha pattern and pair
    int npcls = 0;
    bool psplit = false;   // pair records' beta sign masks split (see StateDesc::ci_psplit)
};

struct DevHam {
    GroupDesc* groups = nullptr;
    SubDesc* subs = nullptr;
    double* tabs = nullptr;
    std::map<int, struct HxWork*> work;   // L -> sector H-apply work list
    CiHam* ci = nullptr;
};

// Launch plan of an ansatz on the packed sector layout with block bits L.
struct PackedPlan {
    int L = 0;
    std::vector<PackedRun> runs;
    std::vector<int> off;             // PackedGate offset per run
    PackedGate* d_gates = nullptr;
    int2* d_info = nullptr;           // pair-list index: {offset, stride} per run and class
    uint32_t* d_ent = nullptr;        // pair lists
    int32_t* d_live = nullptr;        // live tiles of the runs that have a list
    TileDesc* d_tdesc = nullptr;      // launched tiles of each run, in launch order
    std::vector<int32_t> gcnt;        // gradient partials per gate (tiles of its run)
    int32_t* d_gcnt = nullptr;
    int32_t* d_gcnt_live = nullptr;   // the same for the reverse sweep (live tiles of its run)
    int32_t gstride = 1;
    size_t max_lds = 0;
    int max_entries = 0;              // largest tile (entries per vector)
    int max_stride = 0;               // longest padded pair list of a gate in a tile
    int max_gates = 0;                // longest run
    std::vector<double> run_work;     // per run: live-tile entries x gates (load balance)
    double fwd_bytes = 0.0, adj_bytes = 0.0;   // algorithmic traffic of one evaluation
    // single-launch zero-angle sweep (built on first use as a pool)
    PackedRun* d_runs = nullptr;
    int32_t* d_blk = nullptr;    // run of each block, then the first block of each run
    PoolSweep sweep{};
    double sweep_bytes = 0.0;    // phi and lambda entries of every live tile, read once
    double pairs = 0.0;          // pair updates of one pass over the gates (live tiles)
};

struct DevAnsatz {
    GateDesc* gates = nullptr;
    std::map<std::pair<int64_t, int64_t>, AnsatzPlan*> plans;
    std::map<std::tuple<int, int, int, int>, PackedPlan*> packed;   // by (L, fwd, adj threads, tile cap)
};

static int current_device(int* dev) {
    HIPCHK(hipGetDevice(dev));
    return VQE_OK;
}

template <class T>
static int upload(T** dst, const T* src, size_t count) {
    *dst = nullptr;
    if (count == 0) return VQE_OK;
    HIPCHK(hipMalloc(dst, count * sizeof(T)));
    HIPCHK(hipMemcpy(*dst, src, count * sizeof(T), hipMemcpyHostToDevice));
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
    int rc = upload(&d->groups, H->groups.data(), H->groups.size());
    if (!rc) rc = upload(&d->subs, H->subs.data(), H->subs.size());
    if (!rc) rc = upload(&d->tabs, H->tabs.data(), H->tabs.size());
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

// Work list of the sector H-apply for tile bits L: the groups (sorted by x,
// hence by x >> L) cut into chunks that fit the kernel's LDS buffers.
struct HxWork {
    HxChunk* chunks = nullptr;
    GroupDesc* cgroups = nullptr;
    SubDesc* csubs = nullptr;
    int count = 0;
};

static int ham_chunks(const vqe_hamiltonian* H, DevHam* d, int L, HxWork** out) {
    std::lock_guard<std::mutex> lk(H->mu);
    auto it = d->work.find(L);
    if (it != d->work.end()) {
        *out = it->second;
        return VQE_OK;
    }
    std::vector<HxChunk> ch;
    std::vector<GroupDesc> cg;
    std::vector<SubDesc> cs;
    HxChunk cur{};
    bool open = false;
    auto close = [&]() {
        if (open) {
            cur.cg1 = int32_t(cg.size());
            cur.cs1 = int32_t(cs.size());
            ch.push_back(cur);
        }
        open = false;
    };
    for (size_t gi = 0; gi < H->groups.size(); ++gi) {
        const GroupDesc& g = H->groups[gi];
        const uint32_t xhi = g.x >> L;
        const int ts = 1 << (g.pos & 7);
        int si = g.sub_begin;
        while (si < g.sub_end) {
            if (open && (cur.xhi != xhi || int(cg.size()) - cur.cg0 >= kChunkGroups ||
                         int(cs.size()) - cur.cs0 >= kChunkSubs ||
                         H->subs[si].tab + ts - cur.t0 > kChunkTabs))
                close();
            if (!open) {
                cur = HxChunk{};
                cur.cg0 = int32_t(cg.size());
                cur.cs0 = int32_t(cs.size());
                cur.t0 = H->subs[si].tab;
                cur.t1 = cur.t0;
                cur.xhi = xhi;
                open = true;
            }
            GroupDesc lg = g;
            lg.sub_begin = int32_t(cs.size()) - cur.cs0;
            // as many of this group's subgroups as fit the open chunk
            while (si < g.sub_end && int(cs.size()) - cur.cs0 < kChunkSubs &&
                   H->subs[si].tab + ts - cur.t0 <= kChunkTabs) {
                cs.push_back(SubDesc{H->subs[si].w, H->subs[si].tab - cur.t0});
                cur.t1 = H->subs[si].tab + ts;
                ++si;
            }
            lg.sub_end = int32_t(cs.size()) - cur.cs0;
            if (lg.sub_end > lg.sub_begin) cg.push_back(lg);
            if (si < g.sub_end) close();   // continue this group in a new chunk
        }
    }
    close();
    auto* w = new HxWork();
    w->count = int(ch.size());
    int rc = upload(&w->chunks, ch.data(), ch.size());
    if (!rc) rc = upload(&w->cgroups, cg.data(), cg.size());
    if (!rc) rc = upload(&w->csubs, cs.data(), cs.size());
    if (rc) {
        (void)hipFree(w->chunks);
        (void)hipFree(w->cgroups);
        (void)hipFree(w->csubs);
        delete w;
        return rc;
    }
    d->work[L] = w;
    *out = w;
    return VQE_OK;
}

static uint32_t pext_host(uint32_t v, uint32_t mask) {
    uint32_t out = 0;
    int k = 0;
    for (int q = 0; q < 32; ++q)
        if ((mask >> q) & 1u) out |= ((v >> q) & 1u) << k++;
    return out;
}

// Greedy split of the gate list into fused runs: consecutive excitations with
// the same created orbitals (key) whose tile of `vectors` statevectors fits
// `budget` LDS bytes.  The tile's inner bits always include the lowest three
// qubits (minus key bits) so that loads and stores move whole 128-byte lines.
static void plan_direction(const vqe_ansatz* A, int64_t budget, int vectors,
                           std::vector<std::pair<int, int>>& steps, std::vector<RunDesc>& runs,
                           std::vector<int>& offs, std::vector<TileGate>& tgs, double& bytes) {
    const int n = A->n;
    const uint32_t full = (n == 32) ? 0xffffffffu : ((1u << n) - 1u);
    const int64_t M = int64_t(A->gates.size());
    bytes = 0.0;
    auto tile_bytes = [&](uint32_t inner) {
        return (int64_t(2) << __builtin_popcount(inner)) * int64_t(sizeof(double2)) * vectors;
    };
    auto rot_bytes = [&](uint32_t inner) {   // a Pauli-rotation tile: 2^m amplitudes
        return (int64_t(1) << __builtin_popcount(inner)) * int64_t(sizeof(double2)) * vectors;
    };
    int64_t j = 0;
    while (j < M) {
        const GateDesc& g = A->gates[j];
        if (g.type != kExcitation) {
            // consecutive rotations whose flip masks fit one tile of the budget
            const uint32_t low3 = std::min<uint32_t>(7u, full);
            uint32_t inner = g.x | low3;
            if (rot_bytes(inner) > budget || __builtin_popcount(inner) > 14) {
                steps.push_back({1, int(j)});
                bytes += 2.0 * vectors * double(sizeof(double2)) * double(uint64_t(1) << n);
                ++j;
                continue;
            }
            int64_t j2 = j + 1;
            while (j2 < M && A->gates[j2].type != kExcitation && j2 - j < kMaxRunGates) {
                const uint32_t cand = inner | A->gates[j2].x;
                if (rot_bytes(cand) > budget || __builtin_popcount(cand) > 14) break;
                inner = cand;
                ++j2;
            }
            for (int q = 0; q < n; ++q) {
                const uint32_t bit = 1u << q;
                if (inner & bit) continue;
                if (rot_bytes(inner | bit) > budget || __builtin_popcount(inner | bit) > 14) break;
                inner |= bit;
            }
            RunDesc r{};
            r.g0 = int32_t(j);
            r.g1 = int32_t(j2);
            r.inner = inner;
            r.key = 0;
            r.outer = full & ~inner;
            r.m = __builtin_popcount(inner);
            r.contiguous = (inner == ((1u << r.m) - 1u)) ? 1 : 0;
            r.ntiles = int32_t(1u << __builtin_popcount(r.outer));
            r.kind = 1;
            offs.push_back(int(tgs.size()));
            for (int64_t k = j; k < j2; ++k) {
                const GateDesc& h = A->gates[k];
                TileGate t{};
                t.xr = pext_host(h.x, inner);
                t.pdr = pext_host(h.chain, inner);
                t.chr = uint32_t(__builtin_popcount(h.x & h.chain) & 3);
                t.chain_out = h.chain & r.outer;
                t.csign = 1.0;
                tgs.push_back(t);
            }
            steps.push_back({0, int(runs.size())});
            runs.push_back(r);
            bytes += 2.0 * double(rot_bytes(inner)) * double(r.ntiles);
            j = j2;
            continue;
        }
        const uint32_t key = g.x & ~g.pd;
        const uint32_t low = std::min<uint32_t>(7u, full) & ~key;
        uint32_t inner = (g.pd | low) & ~key;
        int64_t j2 = j + 1;
        while (j2 < M) {
            const GateDesc& h = A->gates[j2];
            if (h.type != kExcitation || (h.x & ~h.pd) != key || j2 - j >= kMaxRunGates) break;
            const uint32_t cand = inner | h.pd;
            if (tile_bytes(cand) > budget) break;
            inner = cand;
            ++j2;
        }
        // grow the tile with the lowest free qubits up to the budget: the same
        // total traffic in fewer, larger tiles with longer contiguous chunks
        for (int q = 0; q < n; ++q) {
            const uint32_t bit = 1u << q;
            if ((inner | key) & bit) continue;
            if (tile_bytes(inner | bit) > budget) break;
            inner |= bit;
        }
        RunDesc r{};
        r.g0 = int32_t(j);
        r.g1 = int32_t(j2);
        r.inner = inner;
        r.key = key;
        r.outer = full & ~inner & ~key;
        r.m = __builtin_popcount(inner);
        r.contiguous = (inner == ((1u << r.m) - 1u)) ? 1 : 0;
        r.ntiles = int32_t(1u << __builtin_popcount(r.outer));
        offs.push_back(int(tgs.size()));
        for (int64_t k = j; k < j2; ++k) {
            const GateDesc& h = A->gates[k];
            TileGate t{};
            t.xr = pext_host(h.pd, inner);
            t.pdr = t.xr;
            t.chr = pext_host(h.chain & inner, inner);
            t.chain_out = h.chain & r.outer;
            t.csign = h.csign;
            tgs.push_back(t);
        }
        steps.push_back({0, int(runs.size())});
        runs.push_back(r);
        bytes += 2.0 * double(tile_bytes(inner)) * double(r.ntiles);   // read + write every tile
        j = j2;
    }
}

static int get_plan(const vqe_ansatz* A, DevAnsatz* da, const Tuning& tn, AnsatzPlan** out) {
    std::lock_guard<std::mutex> lk(A->mu);
    auto key = std::make_pair(tn.fwd_budget, tn.adj_budget);
    auto it = da->plans.find(key);
    if (it != da->plans.end()) {
        *out = it->second;
        return VQE_OK;
    }
    auto* p = new AnsatzPlan();
    p->fwd_budget = tn.fwd_budget;
    p->adj_budget = tn.adj_budget;
    std::vector<TileGate> tf, ta;
    plan_direction(A, tn.fwd_budget, 1, p->fwd_steps, p->fwd_runs, p->fwd_off, tf, p->fwd_bytes);
    plan_direction(A, tn.adj_budget, 2, p->adj_steps, p->adj_runs, p->adj_off, ta, p->adj_bytes);
    const int n = A->n;
    const uint64_t N = uint64_t(1) << n;
    p->fwd_bytes += double(sizeof(double2)) * double(N);   // |HF> write
    p->gcnt.assign(A->gates.size(), 1);
    int32_t gstride = 1;
    for (auto& st : p->adj_steps) {
        if (st.first == 0) {
            const RunDesc& r = p->adj_runs[st.second];
            for (int k = r.g0; k < r.g1; ++k) p->gcnt[k] = r.ntiles;
            gstride = std::max(gstride, r.ntiles);
        } else {
            const int nb = blocks_for(N >> 1);
            p->gcnt[st.second] = nb;
            gstride = std::max(gstride, nb);
        }
    }
    p->gstride = gstride;
    // tiles: 2^(m+1) amplitudes for excitation runs, 2^m for rotation runs
    for (auto& r : p->fwd_runs)
        p->max_lds = std::max(p->max_lds, (size_t(r.kind == 1 ? 1 : 2) << r.m) * sizeof(double2));
    for (auto& r : p->adj_runs)
        p->max_lds = std::max(p->max_lds, (size_t(r.kind == 1 ? 1 : 2) << r.m) * sizeof(double2) * 2);
    int rc = upload(&p->d_fwd_tg, tf.data(), tf.size());
    if (!rc) rc = upload(&p->d_adj_tg, ta.data(), ta.size());
    if (!rc) rc = upload(&p->d_gcnt, p->gcnt.data(), p->gcnt.size());
    if (!rc && p->max_lds > (64u << 10) && enable_large_lds(p->max_lds) != 0)
        rc = fail(VQE_EDEVICE, "could not enable " + std::to_string(p->max_lds) + " bytes of LDS");
    if (rc) {
        (void)hipFree(p->d_fwd_tg);
        (void)hipFree(p->d_adj_tg);
        (void)hipFree(p->d_gcnt);
        delete p;
        return rc;
    }
    da->plans[key] = p;
    *out = p;
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
    if (int rc = upload(&d->gates, A->gates.data(), A->gates.size())) {
        delete d;
        return rc;
    }
    A->dev[dev] = d;
    *out = d;
    return VQE_OK;
}

// Rank/unrank tables of the sector H-apply, one per (device, L).
static std::mutex g_hxt_mu;
static std::map<std::pair<int, int>, HxTables*> g_hxt;

static void fill_tables(int L, HxTables& T) {
    std::memset(&T, 0, sizeof(T));
    T.L = L;
    T.La = (L + 1) / 2;
    T.Lb = L / 2;
    auto build = [](int bits, int shift, int32_t* off, uint16_t* un, uint8_t* rank) {
        int pos = 0;
        for (int k = 0; k <= bits; ++k) {
            off[k] = pos;
            int r = 0;
            for (uint32_t s = 0; s < (1u << bits); ++s) {
                if (__builtin_popcount(s) != k) continue;
                uint32_t spread = 0;
                for (int i = 0; i < bits; ++i)
                    if ((s >> i) & 1u) spread |= 1u << (2 * i + shift);
                un[pos++] = uint16_t(spread);
                rank[s] = uint8_t(r++);
            }
        }
        for (int k = bits + 1; k <= 8; ++k) off[k] = pos;
    };
    build(T.La, 0, T.offA, T.unA, T.rankA);
    build(T.Lb, 1, T.offB, T.unB, T.rankB);
}

static const HxTables* host_tables(int L) {
    static std::mutex mu;
    static std::map<int, HxTables> cache;
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find(L);
    if (it == cache.end()) {
        HxTables T;
        fill_tables(L, T);
        it = cache.emplace(L, T).first;
    }
    return &it->second;
}

static int hx_tables(int L, HxTables** out) {
    int dev;
    if (int rc = current_device(&dev)) return rc;
    std::lock_guard<std::mutex> lk(g_hxt_mu);
    auto it = g_hxt.find({dev, L});
    if (it != g_hxt.end()) {
        *out = it->second;
        return VQE_OK;
    }
    // HxTables followed by the class rank tables (RankK) at kRankKOffset
    std::vector<char> buf(kRankKOffset + sizeof(RankK), 0);
    HxTables& T = *reinterpret_cast<HxTables*>(buf.data());
    fill_tables(L, T);
    RankK& R = *reinterpret_cast<RankK*>(buf.data() + kRankKOffset);
    for (int k = 0; k < 8; ++k)
        for (uint32_t v = 0; v < 128; ++v) {
            const bool inA = v < (1u << T.La), inB = v < (1u << T.Lb);
            R.a[k][v] = int16_t((inA && __builtin_popcount(v) == k) ? T.rankA[v] : kRankMiss);
            R.b[k][v] = int16_t((inB && __builtin_popcount(v) == k) ? T.rankB[v] : kRankMiss);
        }
    char* dptr = nullptr;
    if (int rc = upload(&dptr, buf.data(), buf.size())) return rc;
    HxTables* d = reinterpret_cast<HxTables*>(dptr);
    g_hxt[{dev, L}] = d;
    *out = d;
    return VQE_OK;
}

// ---------------------------------------------------------- packed layout

// Block sizes and offsets of the packed sector layout of (n, ne) with block
// bits L: block h holds C(La, kA) C(Lb, kB) amplitudes, kA and kB being the
// electrons the reference leaves to the low bits after h's own.
struct PackedLayout {
    int n = 0, na = 0, nb = 0, L = 0;
    int64_t size = 0;                    // in-sector amplitudes
    std::vector<int32_t> base, bsize;    // per block h < 2^(n - L)
    int32_t* d_base = nullptr;
    int32_t* d_perm = nullptr;           // block order -> string-product order (or null)
};

// The run kernels' descriptor of tile o of run r (host side of the block
// geometry the pair lists were built with: block sizes from the popcount
// tables, block starts from the layout's base offsets).
static TileDesc host_tile_desc(const HxTables& T, const PackedRun& r, int o, const std::vector<int32_t>& base) {
    TileDesc d{};
    uint32_t hb = 0, bits = r.free_hi, v = uint32_t(o);
    while (bits) {   // pdep(o, free_hi)
        const uint32_t low = bits & (~bits + 1u);
        if (v & 1u) hb |= low;
        v >>= 1;
        bits &= bits - 1;
    }
    d.hbase = hb;
    const uint32_t hbg = hb << r.L;
    const int ca = __builtin_popcount(hbg & 0x55555555u), cb = __builtin_popcount(hbg & 0xAAAAAAAAu);
    d.cls = ca * r.cls_b + cb;
    int acc = 0;
    for (int b = 0; b < kMaxTileBlocks; ++b) {
        d.off[b] = acc;
        d.delta[b] = -acc;
        if (b < r.nblk) {
            const uint32_t sg = r.blk[b] << r.L;
            const int kA = r.na - ca - __builtin_popcount(sg & 0x55555555u);
            const int kB = r.nb - cb - __builtin_popcount(sg & 0xAAAAAAAAu);
            if (kA >= 0 && kA <= T.La && kB >= 0 && kB <= T.Lb) {
                d.delta[b] = base[hb | r.blk[b]] - acc;
                acc += (T.offA[kA + 1] - T.offA[kA]) * (T.offB[kB + 1] - T.offB[kB]);
            }
        }
    }
    d.nE = acc <= r.max_entries ? acc : 0;
    return d;
}

static std::mutex g_lay_mu;
static std::map<std::tuple<int, int, int, int>, PackedLayout*> g_lay;   // (dev, n, ne, L)

static int64_t binom(int n, int k) {
    if (k < 0 || k > n) return 0;
    int64_t r = 1;
    for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
    return r;
}

static int packed_layout(int n, int ne, int L, PackedLayout** out) {
    int dev;
    if (int rc = current_device(&dev)) return rc;
    std::lock_guard<std::mutex> lk(g_lay_mu);
    const auto key = std::make_tuple(dev, n, ne, L);
    auto it = g_lay.find(key);
    if (it != g_lay.end()) {
        *out = it->second;
        return VQE_OK;
    }
    auto* lay = new PackedLayout();
    lay->n = n;
    lay->na = (ne + 1) / 2;
    lay->nb = ne / 2;
    lay->L = L;
    const int La = (L + 1) / 2, Lb = L / 2;
    const uint32_t nblocks = 1u << (n - L);
    lay->base.resize(nblocks);
    lay->bsize.resize(nblocks);
    int64_t pos = 0;
    for (uint32_t h = 0; h < nblocks; ++h) {
        const uint32_t hb = h << L;
        const int kA = lay->na - __builtin_popcount(hb & 0x55555555u);
        const int kB = lay->nb - __builtin_popcount(hb & 0xAAAAAAAAu);
        const int64_t c = binom(La, kA) * binom(Lb, kB);
        lay->base[h] = int32_t(pos);
        lay->bsize[h] = int32_t(c);
        pos += c;
    }
    lay->size = pos;
    if (pos != binom((n + 1) / 2, lay->na) * binom(n / 2, lay->nb) || pos > INT32_MAX) {
        delete lay;
        return fail(VQE_EINVAL, "packed layout: sector size mismatch");
    }
    if (int rc = upload(&lay->d_base, lay->base.data(), lay->base.size())) {
        delete lay;
        return rc;
    }
    g_lay[key] = lay;
    *out = lay;
    return VQE_OK;
}

// ------------------------------------------------------ string-product order

static uint32_t compact_even_host(uint32_t v) {   // bits 0, 2, 4, ... -> 0, 1, 2, ...
    uint32_t out = 0;
    for (int i = 0; i < 16; ++i) out |= ((v >> (2 * i)) & 1u) << i;
    return out;
}

// Alpha and beta strings of (n, ne) with their rank tables.
struct CiSpace {
    int oa = 0, ob = 0, NA = 0, NB = 0;
    std::vector<uint32_t> sa, sb;
    std::vector<int32_t> rank_a;
    std::vector<int16_t> rank_b;
    uint32_t* d_sa = nullptr;
    uint32_t* d_sb = nullptr;
    int32_t* d_rank_a = nullptr;
    int16_t* d_rank_b = nullptr;
    int npairs = 0, e1 = 0;
    uint32_t* d_plist = nullptr;
    CiArgs args() const {
        CiArgs a{};
        a.sa = d_sa;
        a.sb = d_sb;
        a.rank_a = d_rank_a;
        a.rank_b = d_rank_b;
        a.plist = d_plist;
        a.na_str = NA;
        a.nb_str = NB;
        a.ob = ob;
        a.npairs = npairs;
        a.nsplit = 1;
        a.e1 = e1;
        return a;
    }
};

// Index of the beta pair (p < q) among the pairs of ob orbitals, lexicographic.
static int pair_index(int p, int q, int ob) { return p * ob - p * (p + 1) / 2 + (q - p - 1); }

constexpr int kCiMaxBits = 13;    // alpha / beta orbitals of the string-product path
constexpr int kCiMaxCols = 1024;  // beta strings per row (16 per lane)

static std::mutex g_cis_mu;
static std::map<std::tuple<int, int, int>, CiSpace*> g_cis;   // (dev, n, ne)

static int ci_space(int n, int ne, CiSpace** out) {
    int dev;
    if (int rc = current_device(&dev)) return rc;
    std::lock_guard<std::mutex> lk(g_cis_mu);
    const auto key = std::make_tuple(dev, n, ne);
    auto it = g_cis.find(key);
    if (it != g_cis.end()) {
        *out = it->second;
        return VQE_OK;
    }
    auto* c = new CiSpace();
    c->oa = (n + 1) / 2;
    c->ob = n / 2;
    const int na = (ne + 1) / 2, nb = ne / 2;
    c->rank_a.assign(size_t(1) << c->oa, -1);
    c->rank_b.assign(size_t(1) << c->ob, int16_t(-1));
    for (uint32_t v = 0; v < (1u << c->oa); ++v)
        if (__builtin_popcount(v) == na) {
            c->rank_a[v] = int32_t(c->sa.size());
            c->sa.push_back(v);
        }
    for (uint32_t v = 0; v < (1u << c->ob); ++v)
        if (__builtin_popcount(v) == nb) {
            c->rank_b[v] = int16_t(c->sb.size());
            c->sb.push_back(v);
        }
    c->NA = int(c->sa.size());
    c->NB = int(c->sb.size());
    // beta-pair lists: for each column, the pairs with one orbital occupied
    c->npairs = c->ob * (c->ob - 1) / 2;
    c->e1 = nb * (c->ob - nb);
    std::vector<uint32_t> plist(size_t(c->e1) * size_t(c->NB));
    for (int ib = 0; ib < c->NB; ++ib) {
        const uint32_t b = c->sb[ib];
        int e = 0;
        for (int p = 0; p < c->ob; ++p)
            for (int q = p + 1; q < c->ob; ++q) {
                const int bp = (b >> p) & 1, bq = (b >> q) & 1;
                if (bp == bq) continue;
                const int16_t r = c->rank_b[b ^ (1u << p) ^ (1u << q)];
                const uint32_t between = ((1u << q) - 1u) & ~((2u << p) - 1u);   // orbitals p+1 .. q-1
                // byte offsets (of an 8-byte amplitude, of an 8-byte coefficient)
                // so that the kernel adds them to its LDS bases as they are
                plist[size_t(e) * c->NB + ib] = uint32_t(r) * 8u |
                                                (uint32_t(2 * pair_index(p, q, c->ob) + bq) * 8u << 16) |
                                                (uint32_t(__builtin_popcount(b & between) & 1) << 31);
                ++e;
            }
    }
    int rc = upload(&c->d_sa, c->sa.data(), c->sa.size());
    if (!rc && !plist.empty()) rc = upload(&c->d_plist, plist.data(), plist.size());
    if (!rc) rc = upload(&c->d_sb, c->sb.data(), c->sb.size());
    if (!rc) rc = upload(&c->d_rank_a, c->rank_a.data(), c->rank_a.size());
    if (!rc) rc = upload(&c->d_rank_b, c->rank_b.data(), c->rank_b.size());
    if (rc) {
        (void)hipFree(c->d_sa);
        (void)hipFree(c->d_sb);
        (void)hipFree(c->d_rank_a);
        (void)hipFree(c->d_rank_b);
        (void)hipFree(c->d_plist);
        delete c;
        return rc;
    }
    g_cis[key] = c;
    *out = c;
    return VQE_OK;
}

// Block order -> string-product order of a packed layout.
static int layout_perm(PackedLayout* lay, const CiSpace& cs, const HxTables& T) {
    if (lay->d_perm) return VQE_OK;
    std::vector<int32_t> perm(size_t(lay->size));
    const uint32_t nblocks = uint32_t(lay->base.size());
    for (uint32_t h = 0; h < nblocks; ++h) {
        if (lay->bsize[h] == 0) continue;
        const uint32_t hb = h << lay->L;
        const int kA = lay->na - __builtin_popcount(hb & 0x55555555u);
        const int kB = lay->nb - __builtin_popcount(hb & 0xAAAAAAAAu);
        const int cB = T.offB[kB + 1] - T.offB[kB];
        for (int k = 0; k < lay->bsize[h]; ++k) {
            const uint32_t b = hb | T.unA[T.offA[kA] + k / cB] | T.unB[T.offB[kB] + k % cB];
            const int32_t ra = cs.rank_a[compact_even_host(b)];
            const int32_t rb = cs.rank_b[compact_even_host(b >> 1)];
            if (ra < 0 || rb < 0) return fail(VQE_EINVAL, "string-product order: string outside the sector");
            perm[size_t(lay->base[h]) + k] = ra * cs.NB + rb;
        }
    }
    return upload(&lay->d_perm, perm.data(), perm.size());
}

// Groups, subgroups and re-indexed tables of the string-product H-apply,
// from the folded group structure.  Groups that change N_alpha or N_beta are
// left out (they pair no two sector states).  Classes (equal alpha flip
// mask xa) with groups that flip two beta orbitals and have one subgroup
// become beta-pair classes; every other group goes to the generic list, cut
// into LDS-sized chunks.
static int ci_ham(const vqe_hamiltonian* H, DevHam* d, CiHam** out) {
    std::lock_guard<std::mutex> lk(H->mu);
    if (d->ci) {
        *out = d->ci;
        return VQE_OK;
    }
    const int ob = H->n / 2;
    const int npairs = ob * (ob - 1) / 2;
    struct G {
        uint32_t xa, xb;
        size_t gi;
    };
    std::vector<G> order;
    for (size_t gi = 0; gi < H->groups.size(); ++gi) {
        const uint32_t x = H->groups[gi].x;
        if ((__builtin_popcount(x & 0x55555555u) | __builtin_popcount(x & 0xAAAAAAAAu)) & 1) continue;
        order.push_back(G{compact_even_host(x), compact_even_host(x >> 1), gi});
    }
    std::stable_sort(order.begin(), order.end(), [](const G& a, const G& b) {
        return a.xa != b.xa ? a.xa < b.xa : a.xb < b.xb;
    });
    // table layout of a group: alpha and beta positions and their original table bits
    struct Layout {
        int k, ka, kb, pa[4], pb[4], slot_a[4], slot_b[4];
    };
    auto layout = [](const GroupDesc& gd) {
        Layout l{};
        l.k = int(gd.pos & 7);
        for (int i = 0; i < l.k; ++i) {
            const int q = int((gd.pos >> (3 + 5 * i)) & 31);
            if (q % 2 == 0) {
                l.pa[l.ka] = q / 2;
                l.slot_a[l.ka++] = i;
            } else {
                l.pb[l.kb] = q / 2;
                l.slot_b[l.kb++] = i;
            }
        }
        return l;
    };
    auto push_table = [&](const Layout& l, const SubDesc& sd, std::vector<double>& t) {
        for (int e = 0; e < (1 << l.k); ++e) {   // new index e = alpha pattern | beta pattern << ka
            uint32_t old = 0;
            for (int i = 0; i < l.ka; ++i)
                if ((e >> i) & 1) old |= 1u << l.slot_a[i];
            for (int i = 0; i < l.kb; ++i)
                if ((e >> (l.ka + i)) & 1) old |= 1u << l.slot_b[i];
            t.push_back(H->tabs[size_t(sd.tab) + old]);
        }
    };
    auto pair_eligible = [&](const G& o) {
        const GroupDesc& gd = H->groups[o.gi];
        const Layout l = layout(gd);
        return __builtin_popcount(o.xb) == 2 && gd.sub_end - gd.sub_begin == 1 &&
               l.k == __builtin_popcount(H->groups[o.gi].x) && ob >= 2;
    };
    auto make_group = [&](const G& o, const Layout& l, int col_only) {
        CiGroup g{};
        g.xa = o.xa;
        g.xb = o.xb;
        for (int i = 0; i < l.ka; ++i) g.tba |= 1u << l.pa[i];
        for (int i = 0; i < 4; ++i) g.tbb |= uint32_t(i < l.kb ? l.pb[i] : 31) << (5 * i);
        g.meta = (__builtin_popcount(o.xa) / 2) | (l.ka << 8) | (col_only << 16);
        return g;
    };
    // Linear form of a group (4 or more subgroups whose masks all differ from
    // one of them, w0, by at most one orbital): tables S, then -2 T_t per
    // alpha and per beta orbital (see CiGroup).
    const int oa_all = (H->n + 1) / 2;
    auto linear_form = [&](const GroupDesc& gd, const Layout& l, std::vector<double>& t,
                           CiGroup& g) -> bool {
        if (gd.sub_end - gd.sub_begin < 4) return false;
        for (int c = gd.sub_begin; c < gd.sub_end; ++c) {
            const uint32_t w0 = H->subs[c].w;
            bool ok = true;
            for (int si = gd.sub_begin; si < gd.sub_end && ok; ++si)
                ok = __builtin_popcount(H->subs[si].w ^ w0) <= 1;
            if (!ok) continue;
            const int nt = 1 << l.k;
            std::vector<double> T(size_t(1 + oa_all + ob) * nt, 0.0);
            uint32_t ma = 0, mb = 0;
            for (int si = gd.sub_begin; si < gd.sub_end; ++si) {
                std::vector<double> one;
                push_table(l, H->subs[si], one);
                for (int e = 0; e < nt; ++e) T[size_t(e)] += one[size_t(e)];
                const uint32_t dq = H->subs[si].w ^ w0;
                if (!dq) continue;
                const int q = __builtin_ctz(dq);
                const int slot = (q % 2 == 0) ? 1 + q / 2 : 1 + oa_all + q / 2;
                if (q % 2 == 0)
                    ma |= 1u << (q / 2);
                else
                    mb |= 1u << (q / 2);
                for (int e = 0; e < nt; ++e) T[size_t(slot) * nt + e] += -2.0 * one[size_t(e)];
            }
            t.insert(t.end(), T.begin(), T.end());
            g.meta |= 1 << 17;
            g.wa = compact_even_host(w0);
            g.wb = compact_even_host(w0 >> 1);
            g.s0 = int32_t(ma);
            g.s1 = int32_t(mb);
            g.pad[0] = nt | (oa_all << 8);
            return true;
        }
        return false;
    };
    // groups that flip alpha orbitals only, with one subgroup over all their
    // flip bits: listed per row (CiRowMove) instead of visited by every row
    auto row_move = [&](const G& o) {
        const GroupDesc& gd = H->groups[o.gi];
        const Layout l = layout(gd);
        return o.xb == 0 && o.xa != 0 && gd.sub_end - gd.sub_begin == 1 &&
               l.k == __builtin_popcount(H->groups[o.gi].x);
    };
    // and the same for beta orbitals only: listed per column (CiColMove)
    auto col_move = [&](const G& o) {
        const GroupDesc& gd = H->groups[o.gi];
        const Layout l = layout(gd);
        return o.xa == 0 && o.xb != 0 && gd.sub_end - gd.sub_begin == 1 &&
               l.k == __builtin_popcount(H->groups[o.gi].x);
    };
    // linear groups flipping two beta orbitals only: column lists with a per-row
    // alpha part (CiBetaHop)
    auto beta_hop = [&](const G& o, BetaHopGroup* out) {
        const GroupDesc& gd = H->groups[o.gi];
        const Layout l = layout(gd);
        if (o.xa != 0 || __builtin_popcount(o.xb) != 2 || l.k != 2 || l.kb != 2) return false;
        for (int c = gd.sub_begin; c < gd.sub_end; ++c) {
            const uint32_t w0 = H->subs[c].w;
            bool ok = true;
            for (int si = gd.sub_begin; si < gd.sub_end && ok; ++si)
                ok = __builtin_popcount(H->subs[si].w ^ w0) <= 1;
            if (!ok) continue;
            BetaHopGroup r{};
            r.xb = o.xb;
            r.lo = uint32_t(__builtin_ctz(o.xb));
            r.hi = uint32_t(31 - __builtin_clz(o.xb));
            r.pair = pair_index(int(r.lo), int(r.hi), ob);
            r.wa0 = compact_even_host(w0);
            r.wb0 = compact_even_host(w0 >> 1);
            r.Tb.assign(size_t(ob) * 4, 0.0);
            r.Ta.assign(size_t(oa_all) * 4, 0.0);
            for (int si = gd.sub_begin; si < gd.sub_end; ++si) {
                std::vector<double> one;
                push_table(l, H->subs[si], one);   // by beta pattern (ka = 0)
                for (int e = 0; e < 4; ++e) r.S[e] += one[size_t(e)];
                const uint32_t dq = H->subs[si].w ^ w0;
                if (!dq) continue;
                const int q = __builtin_ctz(dq);
                std::vector<double>& T = (q % 2 == 0) ? r.Ta : r.Tb;
                for (int e = 0; e < 4; ++e) T[size_t(q / 2) * 4 + e] += -2.0 * one[size_t(e)];
            }
            *out = std::move(r);
            return true;
        }
        return false;
    };
    // the diagonal group, when it holds only one- and two-orbital Z strings
    DiagForm dform;
    auto diag_form = [&](const G& o) {
        if (o.xa != 0 || o.xb != 0) return false;
        const GroupDesc& gd = H->groups[o.gi];
        if ((gd.pos & 7) != 0) return false;
        for (int si = gd.sub_begin; si < gd.sub_end; ++si)
            if (__builtin_popcount(H->subs[si].w) > 2) return false;
        const int n = H->n;
        dform.on = true;
        dform.L.assign(size_t(n), 0.0);
        dform.Q.assign(size_t(n) * n, 0.0);
        for (int si = gd.sub_begin; si < gd.sub_end; ++si) {
            const uint32_t w = H->subs[si].w;
            const double cc = H->tabs[size_t(H->subs[si].tab)];
            dform.K += cc;
            if (!w) continue;
            const int t = __builtin_ctz(w);
            dform.L[size_t(t)] += -2.0 * cc;
            if (__builtin_popcount(w) == 2) {
                const int u = 31 - __builtin_clz(w);
                dform.L[size_t(u)] += -2.0 * cc;
                dform.Q[size_t(t) * n + u] += 4.0 * cc;
            }
        }
        return true;
    };
    // linear groups flipping two alpha orbitals only: row lists with a per-column
    // beta part (CiAlphaHop)
    const int pairs_a = oa_all * (oa_all - 1) / 2;
    auto alpha_hop = [&](const G& o, AlphaHopGroup* out) {
        const GroupDesc& gd = H->groups[o.gi];
        const Layout l = layout(gd);
        if (o.xb != 0 || __builtin_popcount(o.xa) != 2 || l.k != 2 || l.ka != 2) return false;
        for (int c = gd.sub_begin; c < gd.sub_end; ++c) {
            const uint32_t w0 = H->subs[c].w;
            bool ok = true;
            for (int si = gd.sub_begin; si < gd.sub_end && ok; ++si)
                ok = __builtin_popcount(H->subs[si].w ^ w0) <= 1;
            if (!ok) continue;
            AlphaHopGroup r{};
            r.xa = o.xa;
            r.lo = uint32_t(__builtin_ctz(o.xa));
            r.hi = uint32_t(31 - __builtin_clz(o.xa));
            r.pair = pair_index(int(r.lo), int(r.hi), oa_all);
            r.wa0 = compact_even_host(w0);
            r.wb0 = compact_even_host(w0 >> 1);
            r.Ta.assign(size_t(oa_all) * 4, 0.0);
            r.Tb.assign(size_t(std::max(ob, 1)) * 4, 0.0);
            for (int si = gd.sub_begin; si < gd.sub_end; ++si) {
                std::vector<double> one;
                push_table(l, H->subs[si], one);   // by alpha pattern (kb = 0)
                for (int e = 0; e < 4; ++e) r.S[e] += one[size_t(e)];
                const uint32_t dq = H->subs[si].w ^ w0;
                if (!dq) continue;
                const int q = __builtin_ctz(dq);
                std::vector<double>& T = (q % 2 == 0) ? r.Ta : r.Tb;
                for (int e = 0; e < 4; ++e) T[size_t(q / 2) * 4 + e] += -2.0 * one[size_t(e)];
            }
            *out = std::move(r);
            return true;
        }
        return false;
    };
    std::vector<RowMoveGroup> rmg;
    std::vector<ColMoveGroup> cmg;
    std::vector<BetaHopGroup> bhg;
    std::vector<AlphaHopGroup> ahg;
    {
        std::vector<G> kept;
        for (const G& o : order) {
            if (diag_form(o)) continue;
            AlphaHopGroup agp;
            if (pairs_a > 0 && alpha_hop(o, &agp)) {
                ahg.push_back(std::move(agp));
                continue;
            }
            BetaHopGroup bg;
            if (beta_hop(o, &bg)) {
                bhg.push_back(std::move(bg));
                continue;
            }
            if (col_move(o)) {
                const GroupDesc& gd = H->groups[o.gi];
                const Layout l = layout(gd);
                ColMoveGroup r{};
                r.xb = o.xb;
                for (int i = 0; i < l.kb; ++i) r.tbb |= 1u << l.pb[i];
                const SubDesc& sd = H->subs[gd.sub_begin];
                r.wa = compact_even_host(sd.w);
                r.wb = compact_even_host(sd.w >> 1);
                push_table(l, sd, r.tab);
                cmg.push_back(std::move(r));
                continue;
            }
            if (!row_move(o)) {
                kept.push_back(o);
                continue;
            }
            const GroupDesc& gd = H->groups[o.gi];
            const Layout l = layout(gd);
            RowMoveGroup r{};
            r.xa = o.xa;
            for (int i = 0; i < l.ka; ++i) r.tba |= 1u << l.pa[i];
            const SubDesc& sd = H->subs[gd.sub_begin];
            r.wa = compact_even_host(sd.w);
            r.wb = compact_even_host(sd.w >> 1);
            push_table(l, sd, r.tab);
            rmg.push_back(std::move(r));
        }
        order.swap(kept);
    }
    std::map<uint32_t, int> is_pair;   // xa -> the class has a beta-pair group
    for (const G& o : order)
        if (pair_eligible(o)) is_pair[o.xa] = 1;
    // ---- beta-pair classes
    std::vector<CiPairClass> pcls;
    bool psplit = true;   // every class's records share one beta chain mask beyond their own pair
    std::vector<CiPairRec> precs;
    std::vector<CiGroup> rgrp;
    std::vector<CiSub> rsub;
    std::vector<double> ptab;
    for (size_t i = 0; i < order.size();) {
        size_t j = i;
        while (j < order.size() && order[j].xa == order[i].xa) ++j;
        if (is_pair.count(order[i].xa)) {
            CiPairClass pc{};
            pc.xa = order[i].xa;
            pc.half = __builtin_popcount(pc.xa) / 2;
            pc.rec0 = int32_t(precs.size());
            precs.resize(precs.size() + size_t(npairs), CiPairRec{-1, 0u, 0u, 0});
            pc.rest0 = int32_t(rgrp.size());
            uint32_t known = 0;   // bits of the class mask fixed by some record
            for (size_t t = i; t < j; ++t) {
                const G& o = order[t];
                const GroupDesc& gd = H->groups[o.gi];
                const Layout l = layout(gd);
                if (pair_eligible(o)) {
                    const int p = __builtin_ctz(o.xb), q = 31 - __builtin_clz(o.xb);
                    CiPairRec& r = precs[size_t(pc.rec0 + pair_index(p, q, ob))];
                    const SubDesc& sd = H->subs[gd.sub_begin];
                    r.tab = int32_t(ptab.size());
                    r.wa = compact_even_host(sd.w);
                    r.wb = compact_even_host(sd.w >> 1);
                    r.ka = l.ka | (p << 8) | (q << 16);
                    push_table(l, sd, ptab);
                    // the record's mask must be (orbitals strictly between p and q)
                    // ^ (the class mask off p and q): bits p, q of the class mask
                    // cancel in the kernel (a listed column has exactly one of them)
                    const uint32_t between = ((1u << q) - 1u) & ~((2u << p) - 1u);
                    const uint32_t pq = (1u << p) | (1u << q), m = r.wb ^ between;
                    if ((m & pq) != 0 || ((m ^ pc.wbc) & known & ~pq) != 0) psplit = false;
                    pc.wbc |= m & ~known & ~pq;
                    known |= ~pq;
                } else {
                    CiGroup g = make_group(o, l, 0);
                    std::vector<double> lt;
                    if (linear_form(gd, l, lt, g)) {
                        g.tab = int32_t(ptab.size());
                        ptab.insert(ptab.end(), lt.begin(), lt.end());
                        rgrp.push_back(g);
                        continue;
                    }
                    g.s0 = int32_t(rsub.size());
                    for (int si = gd.sub_begin; si < gd.sub_end; ++si) {
                        const SubDesc& sd = H->subs[si];
                        CiSub cs{};
                        cs.wa = compact_even_host(sd.w);
                        cs.wb = compact_even_host(sd.w >> 1);
                        cs.tab = int32_t(ptab.size());
                        push_table(l, sd, ptab);
                        rsub.push_back(cs);
                    }
                    g.s1 = int32_t(rsub.size());
                    g.wa = rsub[size_t(g.s0)].wa;
                    g.wb = rsub[size_t(g.s0)].wb;
                    g.tab = rsub[size_t(g.s0)].tab;
                    rgrp.push_back(g);
                }
            }
            pc.rest1 = int32_t(rgrp.size());
            pcls.push_back(pc);
        }
        i = j;
    }
    // ---- generic groups (the other classes), chunked
    std::map<uint32_t, int> col_only;   // xa -> every group of the class has xb = 0
    for (const G& o : order) {
        if (is_pair.count(o.xa)) continue;
        auto it = col_only.find(o.xa);
        if (it == col_only.end()) it = col_only.emplace(o.xa, 1).first;
        if (o.xb != 0) it->second = 0;
    }
    std::vector<CiChunk> chunks;
    std::vector<CiGroup> grp;
    std::vector<CiSub> sub;
    std::vector<double> tab;
    CiChunk cur{};
    bool open = false;
    auto close = [&]() {
        if (open) {
            cur.g1 = int32_t(grp.size());
            cur.s1 = int32_t(sub.size());
            cur.t1 = int32_t(tab.size());
            chunks.push_back(cur);
        }
        open = false;
    };
    for (const G& o : order) {
        if (is_pair.count(o.xa)) continue;
        const GroupDesc& gd = H->groups[o.gi];
        const Layout l = layout(gd);
        const int nt = 1 << l.k;
        const CiGroup g = make_group(o, l, col_only[o.xa]);
        {   // a linear group: one unit of (1 + oa + ob) nt table entries
            CiGroup lg = g;
            std::vector<double> lt;
            if (linear_form(gd, l, lt, lg)) {
                if (open && (int(grp.size()) - cur.g0 >= kCiChunkGroups ||
                             int(tab.size()) - cur.t0 + int(lt.size()) > kCiChunkTabs))
                    close();
                if (!open) {
                    cur = CiChunk{};
                    cur.g0 = int32_t(grp.size());
                    cur.s0 = int32_t(sub.size());
                    cur.t0 = int32_t(tab.size());
                    open = true;
                }
                lg.tab = int32_t(tab.size()) - cur.t0;
                tab.insert(tab.end(), lt.begin(), lt.end());
                grp.push_back(lg);
                continue;
            }
        }
        int si = gd.sub_begin;
        while (si < gd.sub_end) {
            if (open && (int(grp.size()) - cur.g0 >= kCiChunkGroups ||
                         int(sub.size()) - cur.s0 >= kCiChunkSubs ||
                         int(tab.size()) - cur.t0 + nt > kCiChunkTabs))
                close();
            if (!open) {
                cur = CiChunk{};
                cur.g0 = int32_t(grp.size());
                cur.s0 = int32_t(sub.size());
                cur.t0 = int32_t(tab.size());
                open = true;
            }
            CiGroup lg = g;
            lg.s0 = int32_t(sub.size()) - cur.s0;
            // as many of this group's subgroups as fit the open chunk
            while (si < gd.sub_end && int(sub.size()) - cur.s0 < kCiChunkSubs &&
                   int(tab.size()) - cur.t0 + nt <= kCiChunkTabs) {
                const SubDesc& sd = H->subs[si];
                CiSub cs{};
                cs.wa = compact_even_host(sd.w);
                cs.wb = compact_even_host(sd.w >> 1);
                cs.tab = int32_t(tab.size()) - cur.t0;
                std::vector<double> t1;
                push_table(l, sd, t1);
                tab.insert(tab.end(), t1.begin(), t1.end());
                sub.push_back(cs);
                ++si;
            }
            lg.s1 = int32_t(sub.size()) - cur.s0;
            if (lg.s1 > lg.s0) {
                const CiSub& first = sub[size_t(cur.s0 + lg.s0)];
                lg.wa = first.wa;
                lg.wb = first.wb;
                lg.tab = first.tab;
                grp.push_back(lg);
            }
            if (si < gd.sub_end) close();   // continue this group in a new chunk
        }
    }
    close();
    if (chunks.empty()) chunks.push_back(CiChunk{});   // nothing generic: one empty chunk
    // the pair coefficients of every class for every alpha pattern of its flipped
    // alpha orbitals (patterns 1 and 2 of the beta pair), from the tables; with
    // psplit, each carries the class mask's bit at the pair orbital the output
    // occupies (p for the first, q for the second)
    std::vector<double2> pcoef;
    for (CiPairClass& pc : pcls) {
        const int ka = __builtin_popcount(pc.xa);
        pc.coef0 = int32_t(pcoef.size());
        for (uint32_t ta = 0; ta < (1u << ka); ++ta)
            for (int jp = 0; jp < npairs; ++jp) {
                const CiPairRec& r = precs[size_t(pc.rec0 + jp)];
                double c1 = 0.0, c2 = 0.0;
                if (r.tab >= 0) {
                    const int rka = r.ka & 0xff, p = (r.ka >> 8) & 0xff, q = (r.ka >> 16) & 0xff;
                    c1 = ptab[size_t(r.tab) + (ta | (1u << rka))];
                    c2 = ptab[size_t(r.tab) + (ta | (2u << rka))];
                    if (psplit && ((pc.wbc >> p) & 1u)) c1 = -c1;
                    if (psplit && ((pc.wbc >> q) & 1u)) c2 = -c2;
                }
                pcoef.push_back(make_double2(c1, c2));
            }
    }
    auto* c = new CiHam();
    c->nchunks = int(chunks.size());
    c->ob = ob;
    c->npcls = int(pcls.size());
    c->psplit = psplit;
    c->rmg.swap(rmg);
    c->cmg.swap(cmg);
    std::vector<double> hopa(size_t(std::max(npairs, 1)) * 16 * 2, 0.0);
    for (const BetaHopGroup& g : bhg)
        for (int t = 0; t < oa_all && t < 16; ++t)
            for (int pi = 0; pi < 2; ++pi)
                hopa[(size_t(g.pair) * 16 + t) * 2 + pi] = g.Ta[size_t(t) * 4 + pi + 1];
    c->bhg.swap(bhg);
    c->ahg.swap(ahg);
    std::vector<double> dgx;
    if (dform.on) {
        const int n = H->n;
        dgx.assign(16 * 16, 0.0);
        for (int t = 0; t < oa_all; ++t)
            for (int u = 0; u < ob; ++u) {
                const int qa = 2 * t, qb = 2 * u + 1;
                dgx[size_t(t) * 16 + u] = dform.Q[size_t(std::min(qa, qb)) * n + std::max(qa, qb)];
            }
    }
    c->diag = std::move(dform);
    int rc = upload(&c->d_hopa, hopa.data(), hopa.size());
    if (!rc && !dgx.empty()) rc = upload(&c->d_dgx, dgx.data(), dgx.size());
    if (!rc) rc = upload(&c->chunks, chunks.data(), chunks.size());
    if (!rc) rc = upload(&c->groups, grp.data(), grp.size());
    if (!rc) rc = upload(&c->subs, sub.data(), sub.size());
    if (!rc) rc = upload(&c->tabs, tab.data(), tab.size());
    if (!rc) rc = upload(&c->pcls, pcls.data(), pcls.size());
    if (!rc) rc = upload(&c->precs, precs.data(), precs.size());
    if (!rc) rc = upload(&c->rgroups, rgrp.data(), rgrp.size());
    if (!rc) rc = upload(&c->rsubs, rsub.data(), rsub.size());
    if (!rc) rc = upload(&c->ptabs, ptab.data(), ptab.size());
    if (!rc) rc = upload(&c->pcoef, pcoef.data(), pcoef.size());
    if (rc) {
        (void)hipFree(c->chunks);
        (void)hipFree(c->groups);
        (void)hipFree(c->subs);
        (void)hipFree(c->tabs);
        (void)hipFree(c->pcls);
        (void)hipFree(c->precs);
        (void)hipFree(c->rgroups);
        (void)hipFree(c->rsubs);
        (void)hipFree(c->ptabs);
        (void)hipFree(c->pcoef);
        (void)hipFree(c->d_hopa);
        (void)hipFree(c->d_dgx);
        delete c;
        return rc;
    }
    d->ci = c;
    *out = c;
    return VQE_OK;
}

// Smallest block-bit count for which every gate of A can run on the packed
// layout (all excitations, annihilated orbitals in the low bits) and the
// reference of ne electrons is entry 0 (block 0), or -1.
static int packed_min_L(const vqe_ansatz* A, int ne) {
    if (A->n > 31) return -1;   // the packed H-apply relies on bit 31 of a string being 0
    for (const GateDesc& g : A->gates) {
        if (g.type != kExcitation || g.pd == 0) return -1;
        const uint32_t key = g.x & ~g.pd;
        if (__builtin_popcount(g.pd & 0x55555555u) != __builtin_popcount(key & 0x55555555u) ||
            __builtin_popcount(g.pd & 0xAAAAAAAAu) != __builtin_popcount(key & 0xAAAAAAAAu))
            return -1;
    }
    return std::max(1, ne);   // the reference in block 0
}

static int packed_plan(const vqe_ansatz* A, DevAnsatz* da, const PackedLayout& lay,
                       const Tuning& tn, PackedPlan** out) {
    std::lock_guard<std::mutex> lk(A->mu);
    const auto pkey = std::make_tuple(lay.L, tn.fwd_threads, tn.adj_threads, tn.tile_cap);
    auto it = da->packed.find(pkey);
    if (it != da->packed.end()) {
        *out = it->second;
        return VQE_OK;
    }
    const int n = A->n, L = lay.L;
    const uint32_t hmask = (1u << (n - L)) - 1u, lowmask = (1u << L) - 1u;
    const int64_t M = int64_t(A->gates.size());
    const HxTables& T = *host_tables(L);
    auto* p = new PackedPlan();
    p->L = L;
    p->gcnt.assign(size_t(M), 1);
    std::vector<PackedGate> pg;
    std::vector<int2> info;       // per run and first-block class: {offset, stride}
    std::vector<uint32_t> ent;    // pair lists
    std::vector<size_t> info0;    // offset of each run's info table
    // blocks that may hold a nonzero amplitude in the forward pass: first the
    // reference's (entry 0, the lowest nonempty block), then every block of a
    // tile that had one
    std::vector<char> nz(size_t(hmask) + 1, 0);
    for (uint32_t h = 0; h <= hmask; ++h)
        if (lay.bsize[h] > 0) {
            nz[h] = 1;
            break;
        }
    std::vector<int32_t> live_all;
    std::vector<std::pair<size_t, size_t>> live_of;   // per run: {offset, count}
    std::vector<TileDesc> tdesc;                      // launched tiles of every run
    std::vector<size_t> tdesc0;                       // per run: its first descriptor
    if (lay.size >= (int64_t(1) << 31)) {
        delete p;
        return fail(VQE_ERANGE, "packed layout: state too large for 32-bit tile offsets");
    }
    constexpr size_t kNoList = ~size_t(0);
    // tile-size limit of a run (entries per vector): the tuning's, else at
    // least kDefaultTileCap and two of the layout's largest blocks (a tile of
    // one block pair).  Measured on a single 24-qubit state with the run
    // kernels' 256 threads: caps of 2400 and 3200 entries 2.23-2.24 ms per
    // energy + gradient, 800-1600 entries 2.48-2.52 ms, two largest blocks 2.53
    constexpr int64_t kDefaultTileCap = 2400;
    int32_t maxblk = 1;
    for (int32_t b : lay.bsize) maxblk = std::max(maxblk, b);
    const int64_t cap = std::min<int64_t>(
        tn.tile_cap > 0 ? tn.tile_cap : std::max<int64_t>(2 * int64_t(maxblk), kDefaultTileCap), kMaxTileEntries);
    // block patterns (within window W) that the gates [j0, j1) pair: D blocks
    // hold the gate's high annihilated bits and none of its high created ones,
    // E blocks the reverse, with any combination of the window's other bits
    auto used_patterns = [&](int64_t j0, int64_t j1, uint32_t W) {
        uint32_t mask = 0;   // bit i: pattern pdep(i, W)
        const int nw = __builtin_popcount(W);
        for (int i = 0; i < (1 << nw); ++i) {
            uint32_t s_ = 0, bits = W, v = uint32_t(i);
            while (bits) {
                const uint32_t low = bits & (~bits + 1u);
                if (v & 1u) s_ |= low;
                v >>= 1;
                bits &= bits - 1;
            }
            for (int64_t k = j0; k < j1; ++k) {
                const GateDesc& h = A->gates[size_t(k)];
                const uint32_t dg = (h.pd >> L) & hmask, kg = ((h.x & ~h.pd) >> L) & hmask;
                const uint32_t part = s_ & (dg | kg);
                if (part == dg || part == kg) {
                    mask |= 1u << i;
                    break;
                }
            }
        }
        return mask;
    };
    auto pattern = [&](uint32_t W, int i) {
        uint32_t s_ = 0, bits = W, v = uint32_t(i);
        while (bits) {
            const uint32_t low = bits & (~bits + 1u);
            if (v & 1u) s_ |= low;
            v >>= 1;
            bits &= bits - 1;
        }
        return s_;
    };
    std::map<std::pair<uint32_t, uint32_t>, int64_t> tile_memo;   // (W, used mask) -> largest tile
    auto largest_tile = [&](uint32_t W, uint32_t umask) {
        auto key = std::make_pair(W, umask);
        auto it2 = tile_memo.find(key);
        if (it2 != tile_memo.end()) return it2->second;
        const uint32_t free_ = hmask & ~W;
        const int nf = __builtin_popcount(free_), nw = __builtin_popcount(W);
        int64_t best = 0;
        for (uint32_t o = 0; o < (1u << nf); ++o) {
            const uint32_t base = pattern(free_, int(o));
            int64_t sum = 0;
            for (int i = 0; i < (1 << nw); ++i)
                if (umask >> i & 1u) sum += lay.bsize[base | pattern(W, i)];
            best = std::max(best, sum);
        }
        tile_memo[key] = best;
        return best;
    };
    const int nAhi = __builtin_popcount((hmask << L) & 0x55555555u);   // alpha high qubits
    const int nBhi = __builtin_popcount((hmask << L) & 0xAAAAAAAAu);
    int64_t j = 0;
    while (j < M) {
        // grow the run: gate j2 joins while the window stays within 4 bits, the
        // largest tile within cap entries and the run within kMaxRunGates gates
        uint32_t W = 0, umask = 0;
        int64_t j2 = j;
        while (j2 < M && j2 - j < kMaxRunGates) {
            const GateDesc& h = A->gates[size_t(j2)];
            const uint32_t W2 = W | ((h.pd >> L) & hmask) | (((h.x & ~h.pd) >> L) & hmask);
            if (__builtin_popcount(W2) > 4) break;
            const uint32_t u2 = used_patterns(j, j2 + 1, W2);
            if (j2 > j && largest_tile(W2, u2) > cap) break;
            W = W2;
            umask = u2;
            ++j2;
        }
        PackedRun r{};
        r.g0 = int32_t(j);
        r.g1 = int32_t(j2);
        r.W = W;
        r.free_hi = hmask & ~W;
        r.ntiles = int32_t(1u << __builtin_popcount(r.free_hi));
        r.L = L;
        r.na = lay.na;
        r.nb = lay.nb;
        r.nblk = 0;
        for (int i = 0; i < (1 << __builtin_popcount(W)); ++i)
            if (umask >> i & 1u) r.blk[r.nblk++] = pattern(W, i);
        const int nAf = __builtin_popcount((r.free_hi << L) & 0x55555555u);
        const int nBf = __builtin_popcount((r.free_hi << L) & 0xAAAAAAAAu);
        (void)nAhi;
        (void)nBhi;
        r.cls_b = nBf + 1;
        r.ncls = (nAf + 1) * (nBf + 1);
        int maxe = 1;
        int64_t moved = 0, moved_live = 0;
        const size_t live0 = live_all.size();
        std::vector<char> used(size_t(r.ncls), 0);   // classes of nonempty tiles
        std::vector<int64_t> live_cls(size_t(r.ncls), 0);   // live tiles per class
        for (int32_t o = 0; o < r.ntiles; ++o) {
            const uint32_t base = pattern(r.free_hi, o);
            int nE = 0;
            bool any_nz = false;
            for (int b = 0; b < r.nblk; ++b) {
                const int c = lay.bsize[base | r.blk[b]];
                nE += c;
                if (c > 0 && nz[base | r.blk[b]]) any_nz = true;
            }
            if (nE == 0) continue;
            maxe = std::max(maxe, nE);
            moved += nE;
            if (any_nz) {   // the run's gates leave a tile of zero blocks zero
                live_all.push_back(o);
                moved_live += nE;
                const uint32_t hl = base << L;
                ++live_cls[size_t(__builtin_popcount(hl & 0x55555555u) * r.cls_b +
                                  __builtin_popcount(hl & 0xAAAAAAAAu))];
                for (int b = 0; b < r.nblk; ++b)
                    if (lay.bsize[base | r.blk[b]] > 0) nz[base | r.blk[b]] = 1;
            }
            const uint32_t hb = base << L;
            used[size_t(__builtin_popcount(hb & 0x55555555u) * r.cls_b +
                        __builtin_popcount(hb & 0xAAAAAAAAu))] = 1;
        }
        if (maxe > kMaxTileEntries) {
            delete p;
            return fail(VQE_EINVAL, "packed layout: tile too large for the pair lists");
        }
        info0.push_back(info.size());
        // pair lists per (gate, class); laid out per class with every gate's
        // list padded to the class's longest (kPairNone), so that gate g's list
        // starts at offset + g * stride and needs no per-gate descriptor
        const int64_t ng = j2 - j;
        const int ncl = r.ncls;
        std::vector<std::vector<uint32_t>> lists(size_t(ng) * size_t(ncl));
        for (int cls = 0; cls < ncl; ++cls) {
            if (!used[size_t(cls)]) continue;
            const int ca = cls / r.cls_b, cb = cls % r.cls_b;
            // the class's block shapes: (alpha, beta) electrons left to the low bits
            int kA[kMaxTileBlocks], kB[kMaxTileBlocks], cnt[kMaxTileBlocks], off[kMaxTileBlocks];
            int acc = 0;
            for (int b = 0; b < r.nblk; ++b) {
                const uint32_t sb = r.blk[b] << L;
                kA[b] = lay.na - ca - __builtin_popcount(sb & 0x55555555u);
                kB[b] = lay.nb - cb - __builtin_popcount(sb & 0xAAAAAAAAu);
                const bool ok = kA[b] >= 0 && kA[b] <= T.La && kB[b] >= 0 && kB[b] <= T.Lb;
                cnt[b] = ok ? (T.offA[kA[b] + 1] - T.offA[kA[b]]) * (T.offB[kB[b] + 1] - T.offB[kB[b]]) : 0;
                off[b] = acc;
                acc += cnt[b];
            }
            for (int64_t k = j; k < j2; ++k) {
                const GateDesc& h = A->gates[size_t(k)];
                const uint32_t pd = h.pd & lowmask, klo = (h.x & ~h.pd) & lowmask, chlo = h.chain & lowmask;
                const size_t list_before = lists[size_t(k - j) * ncl + cls].size();
                const uint32_t dg = (h.pd >> L) & hmask, kg = ((h.x & ~h.pd) >> L) & hmask;
                std::vector<uint32_t>& lst = lists[size_t(k - j) * ncl + cls];
                for (int b = 0; b < r.nblk; ++b) {
                    if ((r.blk[b] & (dg | kg)) != dg || cnt[b] == 0) continue;   // D blocks
                    const uint32_t se = r.blk[b] ^ dg ^ kg;
                    int be = -1;
                    for (int b2 = 0; b2 < r.nblk; ++b2)
                        if (r.blk[b2] == se) be = b2;
                    if (be < 0 || cnt[be] == 0) continue;
                    const uint32_t par_hi = uint32_t(__builtin_popcount((r.blk[b] << L) & h.chain & ~lowmask) & 1);
                    const int cB0 = T.offB[kB[b] + 1] - T.offB[kB[b]];
                    const int cB1 = T.offB[kB[be] + 1] - T.offB[kB[be]];
                    for (int e = 0; e < cnt[b]; ++e) {   // D entries of the block, rank order
                        const uint32_t rd = uint32_t(T.unA[T.offA[kA[b]] + e / cB0] | T.unB[T.offB[kB[b]] + e % cB0]);
                        if ((rd & (pd | klo)) != pd) continue;
                        const uint32_t re = rd ^ pd ^ klo;
                        const int ie = off[be] + int(T.rankA[compact_even_host(re)]) * cB1 +
                                       int(T.rankB[compact_even_host(re >> 1)]);
                        const uint32_t par = (uint32_t(__builtin_popcount(rd & chlo)) + par_hi) & 1u;
                        lst.push_back(uint32_t(off[b] + e) | (uint32_t(ie) << kEntBits) | (par << kEntParity));
                    }
                }
                // pair updates of the gate over the run's live tiles of this class
                p->pairs += double(lists[size_t(k - j) * ncl + cls].size() - list_before) * double(live_cls[size_t(cls)]);
            }
        }
        for (int cls = 0; cls < ncl; ++cls) {
            int2 rec = make_int2(int(ent.size()), 0);
            if (used[size_t(cls)]) {
                size_t stride = 0;
                for (int64_t g = 0; g < ng; ++g) stride = std::max(stride, lists[size_t(g) * ncl + cls].size());
                for (int64_t g = 0; g < ng; ++g) {
                    const std::vector<uint32_t>& lst = lists[size_t(g) * ncl + cls];
                    ent.insert(ent.end(), lst.begin(), lst.end());
                    ent.insert(ent.end(), stride - lst.size(), kPairNone);
                }
                rec.y = int(stride);
                p->max_stride = std::max(p->max_stride, int(stride));
            }
            info.push_back(rec);
        }
        if (ent.size() > size_t(1) << 31) {
            delete p;
            return fail(VQE_ERANGE, "packed layout: pair lists too large");
        }
        r.shape = packed_shape((maxe + 1) / 2, tn.fwd_threads);
        r.shape_adj = packed_shape((maxe + 1) / 2, tn.adj_threads);
        r.max_entries = maxe;
        if (r.shape < 0 || r.shape_adj < 0) {
            delete p;
            return fail(VQE_EINVAL, "packed layout: tile too large for the run kernels");
        }
        p->off.push_back(int(pg.size()));
        for (int64_t k = j; k < j2; ++k) {
            const GateDesc& h = A->gates[size_t(k)];
            PackedGate q{};
            q.pd = h.pd;
            q.klo = (h.x & ~h.pd) & lowmask;
            q.chlo = h.chain & lowmask;
            q.chhi = h.chain & ~lowmask;
            q.csign = h.csign;
            pg.push_back(q);
            p->gcnt[size_t(k)] = r.ntiles;
        }
        p->gstride = std::max(p->gstride, r.ntiles);
        p->max_lds = std::max(p->max_lds, (size_t(maxe) * 2 + 2 * size_t(ng)) * sizeof(double2));
        p->max_entries = std::max(p->max_entries, maxe);
        p->max_gates = std::max(p->max_gates, int(ng));
        p->run_work.push_back(double(moved_live) * double(ng));
        if (live_all.size() - live0 == size_t(r.ntiles)) {   // every tile: no list
            live_all.resize(live0);
            live_of.emplace_back(live0, kNoList);
        } else {
            live_of.emplace_back(live0, live_all.size() - live0);
        }
        tdesc0.push_back(tdesc.size());
        if (live_of.back().second == kNoList)
            for (int32_t o = 0; o < r.ntiles; ++o) tdesc.push_back(host_tile_desc(T, r, o, lay.base));
        else
            for (size_t i = live0; i < live_all.size(); ++i) tdesc.push_back(host_tile_desc(T, r, live_all[i], lay.base));
        p->fwd_bytes += 2.0 * double(sizeof(double2)) * double(moved_live);
        p->adj_bytes += 4.0 * double(sizeof(double2)) * double(moved_live);   // live tiles, as the forward
        p->sweep_bytes += 2.0 * double(sizeof(double2)) * double(moved);
        p->runs.push_back(r);
        j = j2;
    }
    p->fwd_bytes += double(sizeof(double2)) * double(lay.size);   // |HF> write
    int rc = upload(&p->d_gates, pg.data(), pg.size());
    if (!rc) rc = upload(&p->d_gcnt, p->gcnt.data(), p->gcnt.size());
    if (!rc) rc = upload(&p->d_info, info.data(), info.size());
    if (!rc) rc = upload(&p->d_ent, ent.data(), ent.size());
    if (!rc) rc = upload(&p->d_live, live_all.data(), live_all.size());
    if (!rc) rc = upload(&p->d_tdesc, tdesc.data(), tdesc.size());
    std::vector<int32_t> gcnt_live(p->gcnt);
    if (!rc)
        for (size_t r = 0; r < p->runs.size(); ++r) {
            p->runs[r].info = p->d_info + info0[r];
            p->runs[r].ent = p->d_ent;
            const bool listed = live_of[r].second != kNoList && p->d_live != nullptr;
            p->runs[r].live = listed ? p->d_live + live_of[r].first : nullptr;
            p->runs[r].nlive = listed ? int32_t(live_of[r].second) : p->runs[r].ntiles;
            p->runs[r].tdesc = p->d_tdesc + tdesc0[r];
            for (int k = p->runs[r].g0; k < p->runs[r].g1; ++k) gcnt_live[size_t(k)] = p->runs[r].nlive;
        }
    if (!rc) rc = upload(&p->d_gcnt_live, gcnt_live.data(), gcnt_live.size());
    if (!rc && p->max_lds > (64u << 10) && packed_enable_lds(p->max_lds) != 0)
        rc = fail(VQE_EDEVICE, "could not enable " + std::to_string(p->max_lds) + " bytes of LDS");
    if (rc) {
        (void)hipFree(p->d_gates);
        (void)hipFree(p->d_gcnt);
        (void)hipFree(p->d_info);
        (void)hipFree(p->d_ent);
        (void)hipFree(p->d_live);
        (void)hipFree(p->d_tdesc);
        (void)hipFree(p->d_gcnt_live);
        delete p;
        return rc;
    }
    da->packed[pkey] = p;
    *out = p;
    return VQE_OK;
}

// Per-row lists of the row moves for the alpha strings of `cs`.
static int ci_rowmoves(const vqe_hamiltonian* H, CiHam* c, const CiSpace& cs, RowMoves** out) {
    std::lock_guard<std::mutex> lk(H->mu);
    const CiSpace* key = &cs;
    auto it = c->rm.find(key);
    if (it != c->rm.end()) {
        *out = it->second;
        return VQE_OK;
    }
    std::vector<CiRowMove> rm;
    std::vector<int32_t> off;
    for (int ia = 0; ia < cs.NA; ++ia) {
        off.push_back(int32_t(rm.size()));
        const uint32_t a = cs.sa[size_t(ia)];
        for (const RowMoveGroup& g : c->rmg) {
            if (2 * __builtin_popcount(a & g.xa) != __builtin_popcount(g.xa)) continue;
            uint32_t pat = 0;   // a's bits at the table positions, in ascending order
            int k = 0;
            for (uint32_t m = g.tba; m; m &= m - 1, ++k)
                pat |= ((a >> __builtin_ctz(m)) & 1u) << k;
            const double sg = (__builtin_popcount(a & g.wa) & 1) ? -1.0 : 1.0;
            CiRowMove e{};
            e.coef = sg * g.tab[size_t(pat)];
            e.partner = cs.rank_a[size_t(a ^ g.xa)];
            e.wb = g.wb;
            if (e.partner < 0 || e.coef == 0.0) continue;
            rm.push_back(e);
        }
    }
    off.push_back(int32_t(rm.size()));
    auto* r = new RowMoves();
    int rc = upload(&r->d_off, off.data(), off.size());
    if (!rc && !rm.empty()) rc = upload(&r->d_rm, rm.data(), rm.size());
    if (rc) {
        (void)hipFree(r->d_off);
        (void)hipFree(r->d_rm);
        delete r;
        return rc;
    }
    c->rm[key] = r;
    *out = r;
    return VQE_OK;
}

// Per-column lists of the column moves for the beta strings of `cs`,
// entry-major and padded to the longest list.
static int ci_colmoves(const vqe_hamiltonian* H, CiHam* c, const CiSpace& cs, ColMoves** out) {
    std::lock_guard<std::mutex> lk(H->mu);
    const CiSpace* key = &cs;
    auto it = c->cm.find(key);
    if (it != c->cm.end()) {
        *out = it->second;
        return VQE_OK;
    }
    std::vector<std::vector<CiColMove>> per(size_t(cs.NB));
    size_t ncm = 0;
    for (int ib = 0; ib < cs.NB; ++ib) {
        const uint32_t b = cs.sb[size_t(ib)];
        for (const ColMoveGroup& g : c->cmg) {
            if (2 * __builtin_popcount(b & g.xb) != __builtin_popcount(g.xb)) continue;
            uint32_t pat = 0;   // b's bits at the table positions, in ascending order
            int k = 0;
            for (uint32_t m = g.tbb; m; m &= m - 1, ++k)
                pat |= ((b >> __builtin_ctz(m)) & 1u) << k;
            const double sg = (__builtin_popcount(b & g.wb) & 1) ? -1.0 : 1.0;
            CiColMove e{};
            e.coef = sg * g.tab[size_t(pat)];
            e.partner = cs.rank_b[size_t(b ^ g.xb)];
            e.wa = g.wa;
            if (e.partner < 0 || e.coef == 0.0) continue;
            per[size_t(ib)].push_back(e);
        }
        ncm = std::max(ncm, per[size_t(ib)].size());
    }
    std::vector<CiColMove> cm(ncm * size_t(cs.NB));
    for (int ib = 0; ib < cs.NB; ++ib)
        for (size_t e = 0; e < ncm; ++e)
            cm[e * size_t(cs.NB) + size_t(ib)] =
                e < per[size_t(ib)].size() ? per[size_t(ib)][e] : CiColMove{0.0, ib, 0u};
    auto* r = new ColMoves();
    r->ncm = int(ncm);
    if (!cm.empty())
        if (int rc = upload(&r->d_cm, cm.data(), cm.size())) {
            delete r;
            return rc;
        }
    c->cm[key] = r;
    *out = r;
    return VQE_OK;
}

// Per-column lists of the beta hops for the beta strings of `cs`, entry-major
// and padded to the longest list.
static int ci_betahops(const vqe_hamiltonian* H, CiHam* c, const CiSpace& cs, BetaHops** out) {
    std::lock_guard<std::mutex> lk(H->mu);
    const CiSpace* key = &cs;
    auto it = c->bh.find(key);
    if (it != c->bh.end()) {
        *out = it->second;
        return VQE_OK;
    }
    std::vector<std::vector<CiBetaHop>> per(size_t(cs.NB));
    size_t nbh = 0;
    for (int ib = 0; ib < cs.NB; ++ib) {
        const uint32_t b = cs.sb[size_t(ib)];
        for (const BetaHopGroup& g : c->bhg) {
            const uint32_t plo = (b >> g.lo) & 1u, phi_ = (b >> g.hi) & 1u;
            if (plo == phi_) continue;
            const int pat = int(plo | (phi_ << 1));
            const bool neg = __builtin_popcount(b & g.wb0) & 1;
            double v = g.S[pat];
            for (uint32_t m = b & ~g.xb; m; m &= m - 1)
                v += g.Tb[size_t(__builtin_ctz(m)) * 4 + size_t(pat)];
            CiBetaHop e{};
            e.coef = neg ? -v : v;
            const int partner = cs.rank_b[size_t(b ^ g.xb)];
            if (partner < 0) continue;
            e.w = uint32_t(partner) | (uint32_t(g.pair) << 16) | (uint32_t(pat - 1) << 24) |
                  (uint32_t(neg) << 25) | (1u << 26);
            e.wa = g.wa0;
            per[size_t(ib)].push_back(e);
        }
        nbh = std::max(nbh, per[size_t(ib)].size());
    }
    std::vector<CiBetaHop> bh(nbh * size_t(cs.NB));
    for (int ib = 0; ib < cs.NB; ++ib)
        for (size_t e = 0; e < nbh; ++e)
            bh[e * size_t(cs.NB) + size_t(ib)] =
                e < per[size_t(ib)].size() ? per[size_t(ib)][e] : CiBetaHop{0.0, uint32_t(ib), 0u};
    auto* r = new BetaHops();
    r->nbh = int(nbh);
    if (!bh.empty())
        if (int rc = upload(&r->d_bh, bh.data(), bh.size())) {
            delete r;
            return rc;
        }
    c->bh[key] = r;
    *out = r;
    return VQE_OK;
}

// Per-row lists of the alpha hops and their per-column beta parts for the
// strings of `cs`.
static int ci_alphahops(const vqe_hamiltonian* H, CiHam* c, const CiSpace& cs, AlphaHops** out) {
    std::lock_guard<std::mutex> lk(H->mu);
    auto it = c->ah.find(&cs);
    if (it != c->ah.end()) {
        *out = it->second;
        return VQE_OK;
    }
    const int pairs_a = cs.oa * (cs.oa - 1) / 2;
    std::vector<CiAlphaHop> ah;
    std::vector<int32_t> off;
    for (int ia = 0; ia < cs.NA; ++ia) {
        off.push_back(int32_t(ah.size()));
        const uint32_t a = cs.sa[size_t(ia)];
        for (const AlphaHopGroup& g : c->ahg) {
            const uint32_t plo = (a >> g.lo) & 1u, phi_ = (a >> g.hi) & 1u;
            if (plo == phi_) continue;
            const int pat = int(plo | (phi_ << 1));
            const bool neg = __builtin_popcount(a & g.wa0) & 1;
            double v = g.S[pat];
            for (uint32_t m = a & ~g.xa; m; m &= m - 1)
                v += g.Ta[size_t(__builtin_ctz(m)) * 4 + size_t(pat)];
            const int partner = cs.rank_a[size_t(a ^ g.xa)];
            if (partner < 0) continue;
            CiAlphaHop e{};
            e.coef = neg ? -v : v;
            e.w = uint32_t(partner) | (uint32_t(g.pair) << 16) | (uint32_t(pat - 1) << 24) |
                  (uint32_t(neg) << 25);
            e.wb = g.wb0;
            ah.push_back(e);
        }
    }
    off.push_back(int32_t(ah.size()));
    std::vector<double> bpart(size_t(std::max(pairs_a, 1)) * 2 * size_t(cs.NB), 0.0);
    for (const AlphaHopGroup& g : c->ahg)
        for (int pi = 0; pi < 2; ++pi)
            for (int ib = 0; ib < cs.NB; ++ib) {
                double v = 0.0;
                for (uint32_t m = cs.sb[size_t(ib)]; m; m &= m - 1)
                    v += g.Tb[size_t(__builtin_ctz(m)) * 4 + size_t(pi + 1)];
                bpart[(size_t(g.pair) * 2 + pi) * cs.NB + ib] = v;
            }
    auto* r = new AlphaHops();
    int rc = upload(&r->d_off, off.data(), off.size());
    if (!rc && !ah.empty()) rc = upload(&r->d_ah, ah.data(), ah.size());
    if (!rc) rc = upload(&r->d_b, bpart.data(), bpart.size());
    if (rc) {
        (void)hipFree(r->d_off);
        (void)hipFree(r->d_ah);
        (void)hipFree(r->d_b);
        delete r;
        return rc;
    }
    c->ah[&cs] = r;
    *out = r;
    return VQE_OK;
}

// Row and column parts of the diagonal for the strings of `cs`.
static int ci_diag(const vqe_hamiltonian* H, CiHam* c, const CiSpace& cs, DiagParts** out) {
    std::lock_guard<std::mutex> lk(H->mu);
    auto it = c->dg.find(&cs);
    if (it != c->dg.end()) {
        *out = it->second;
        return VQE_OK;
    }
    const int n = H->n;
    const DiagForm& d = c->diag;
    auto part = [&](uint32_t s, int spin) {   // s: compact string of one spin
        double v = 0.0;
        for (uint32_t m = s; m; m &= m - 1) {
            const int q = 2 * __builtin_ctz(m) + spin;
            v += d.L[size_t(q)];
            for (uint32_t m2 = m & (m - 1); m2; m2 &= m2 - 1) {
                const int q2 = 2 * __builtin_ctz(m2) + spin;
                v += d.Q[size_t(q) * n + q2];
            }
        }
        return v;
    };
    std::vector<double> row(size_t(cs.NA)), col(size_t(cs.NB));
    for (int ia = 0; ia < cs.NA; ++ia) row[size_t(ia)] = part(cs.sa[size_t(ia)], 0);
    for (int ib = 0; ib < cs.NB; ++ib) col[size_t(ib)] = d.K + part(cs.sb[size_t(ib)], 1);
    auto* r = new DiagParts();
    int rc = upload(&r->d_row, row.data(), row.size());
    if (!rc) rc = upload(&r->d_col, col.data(), col.size());
    if (rc) {
        (void)hipFree(r->d_row);
        (void)hipFree(r->d_col);
        delete r;
        return rc;
    }
    c->dg[&cs] = r;
    *out = r;
    return VQE_OK;
}

// 0: full 2^n vectors; 1: packed layout with the block-order H-apply;
// 2: packed layout with the string-product H-apply where it applies.
static std::atomic<int> g_packed_enabled{2};
// Real amplitudes on the packed string-product path (see k_packed.hip): on by
// default; off keeps complex amplitudes there (tests compare the two).
static std::atomic<int> g_real_enabled{1};

// ------------------------------------------------------------- workspaces

// Reusable device memory of the single-state path, one per (device, stream).
struct Workspace {
    size_t state_bytes = 0;
    double2* phi = nullptr;
    double2* lam = nullptr;
    double2* aux = nullptr;      // lambda in string-product order (packed path), per split
    size_t aux_bytes = 0;
    int64_t lam_zero_key = -1;   // sector for which lambda is zero outside it
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

static int workspace(void* stream, size_t state_bytes, size_t aux_bytes, size_t scratch_bytes,
                     Workspace** out) {
    int dev;
    if (int rc = current_device(&dev)) return rc;
    std::lock_guard<std::mutex> lk(g_ws_mu);
    Workspace*& ws = g_ws[{dev, stream}];
    if (!ws) ws = new Workspace();
    if (ws->state_bytes < state_bytes) {
        HIPCHK(hipStreamSynchronize((hipStream_t)stream));
        (void)hipFree(ws->phi);
        (void)hipFree(ws->lam);
        ws->phi = ws->lam = nullptr;
        ws->state_bytes = 0;
        ws->lam_zero_key = -1;
        if (int rc = fits_device(state_bytes * 2)) return rc;
        HIPCHK(hipMalloc(&ws->phi, state_bytes));
        HIPCHK(hipMalloc(&ws->lam, state_bytes));
        ws->state_bytes = state_bytes;
    }
    if (ws->aux_bytes < aux_bytes) {
        HIPCHK(hipStreamSynchronize((hipStream_t)stream));
        (void)hipFree(ws->aux);
        ws->aux = nullptr;
        ws->aux_bytes = 0;
        if (int rc = fits_device(aux_bytes)) return rc;
        HIPCHK(hipMalloc(&ws->aux, aux_bytes));
        ws->aux_bytes = aux_bytes;
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
        off += std::max<size_t>(count, 1) * sizeof(T);
        return p;
    }
};

struct ScratchSize {
    size_t s = 256;
    template <class T>
    void add(size_t count) {
        s = ((s + 255) & ~size_t(255)) + std::max<size_t>(count, 1) * sizeof(T);
    }
};

// -------------------------------------------------------------- evaluation

// What one evaluation of a group of identical-program states needs.
struct EvalPlan {
    int n = 0, ne = 0, M = 0;
    const vqe_ansatz* A = nullptr;
    AnsatzPlan* ap = nullptr;
    bool sector = false;
    bool packed = false;     // the whole evaluation on the packed sector layout
    PackedLayout* lay = nullptr;
    PackedPlan* pp = nullptr;
    HxPlan hx{};
    HxTables* hxt = nullptr;
    int nblk_e = 1;          // energy partials per state
    int32_t gstride = 1;     // gradient partials per gate (stride)
    const int32_t* d_gcnt = nullptr;
    int64_t elems = 0;       // amplitudes per state vector
    double fwd_bytes = 0.0, adj_bytes = 0.0;
    size_t fwd_steps = 0, adj_steps = 0;
    bool ci = false;         // packed path with the string-product H-apply
    const CiSpace* cspace = nullptr;
    CiArgs ciargs{};
    const int32_t* perm = nullptr;
    bool real = false;       // packed path with real amplitudes (double, not double2)
    double pairs = 0.0;      // packed path: pair updates of one pass over the gates
    bool small = false;      // whole-state kernels on a small number-conserving sector
    SmallSpace sspace{};
};

// The strings of k set qubits among n (increasing) and their rank table, per
// (device, n, k).
struct SmallTables {
    uint32_t* str = nullptr;
    int16_t* rank = nullptr;
    int nsec = 0;
    std::vector<int16_t> rank_h;
};
static std::mutex g_small_mu;
static std::map<std::tuple<int, int, int>, SmallTables*> g_small;

static int small_tables(int n, int k, SmallTables** out) {
    int dev;
    if (int rc = current_device(&dev)) return rc;
    std::lock_guard<std::mutex> lk(g_small_mu);
    SmallTables*& t = g_small[std::make_tuple(dev, n, k)];
    if (t) {
        *out = t;
        return VQE_OK;
    }
    auto* x = new SmallTables();
    std::vector<uint32_t> str;
    x->rank_h.assign(size_t(1) << n, int16_t(-1));
    for (uint32_t b = 0; b < (1u << n); ++b)
        if (__builtin_popcount(b) == k) {
            x->rank_h[b] = int16_t(str.size());
            str.push_back(b);
        }
    x->nsec = int(str.size());
    int rc = upload(&x->str, str.data(), str.size());
    if (!rc) rc = upload(&x->rank, x->rank_h.data(), x->rank_h.size());
    if (rc) {
        (void)hipFree(x->str);
        (void)hipFree(x->rank);
        delete x;
        return rc;
    }
    t = x;
    *out = t;
    return VQE_OK;
}

// Every gate an excitation whose created qubits are as many as its
// annihilated ones: the number of set qubits is conserved.
static bool number_conserving(const vqe_ansatz* A) {
    for (const GateDesc& g : A->gates)
        if (g.type != kExcitation || __builtin_popcount(g.pd) != __builtin_popcount(g.x & ~g.pd))
            return false;
    return true;
}

// Let the small-sector H-apply stage Hamiltonian H in LDS when it fits (the
// launch then reserves room for the largest of its states' Hamiltonians).
static void small_fit_ham(EvalPlan* ep, const vqe_hamiltonian* H) {
    if (!ep->small) return;
    const size_t bytes = small_ham_bytes(int(H->groups.size()), int(H->subs.size()), int(H->tabs.size()));
    if (bytes > size_t(kSmallHamLds) || bytes <= size_t(ep->sspace.ham_lds)) return;
    SmallSpace t = ep->sspace;
    t.ham_lds = int32_t((bytes + 7) & ~size_t(7));
    if (small_prepare(t) == 0) ep->sspace = t;
}

static bool sector_path(const vqe_ansatz* A, int ne) {
    return A->sector_conserving && A->n_electrons == ne;
}

// force_L > 0: block bits of the packed layout (and sector H-apply tile)
// regardless of the tuning (the persistent batch passes use one common value).
static int make_eval_plan(const vqe_ansatz* A, int ne, bool batched, EvalPlan* ep, int force_L = 0) {
    const int n = A->n;
    ep->n = n;
    ep->ne = ne;
    ep->M = int(A->gates.size());
    ep->A = A;
    Tuning tn = tuning_for(n, batched);
    if (force_L > 0) tn.L = force_L;
    DevAnsatz* da;
    if (int rc = dev_ansatz(A, &da)) return rc;
    if (int rc = get_plan(A, da, tn, &ep->ap)) return rc;
    ep->sector = sector_path(A, ne);
    ep->gstride = ep->ap->gstride;
    ep->d_gcnt = ep->ap->d_gcnt;
    ep->elems = int64_t(1) << n;
    ep->fwd_bytes = ep->ap->fwd_bytes;
    ep->adj_bytes = ep->ap->adj_bytes;
    ep->fwd_steps = ep->ap->fwd_steps.size();
    ep->adj_steps = ep->ap->adj_steps.size();
    if (ep->sector) {
        ep->hx.L = std::min(n, tn.L);
        const int need = g_packed_enabled.load() ? packed_min_L(A, ne) : -1;
        if (need > 0 && need <= std::min(n, kHxMaxL)) {
            ep->packed = true;
            ep->hx.L = std::max(ep->hx.L, need);
        }
        ep->hx.ntiles = 1 << (n - ep->hx.L);
        ep->hx.na = (ne + 1) / 2;
        ep->hx.nb = ne / 2;
        if (int rc = hx_tables(ep->hx.L, &ep->hxt)) return rc;
        ep->nblk_e = ep->hx.ntiles;
        if (ep->packed) {
            if (int rc = packed_layout(n, ne, ep->hx.L, &ep->lay)) return rc;
            if (int rc = packed_plan(A, da, *ep->lay, tn, &ep->pp)) return rc;
            ep->gstride = ep->pp->gstride;
            ep->d_gcnt = ep->pp->d_gcnt_live;
            ep->elems = ep->lay->size;
            ep->fwd_bytes = ep->pp->fwd_bytes;
            ep->adj_bytes = ep->pp->adj_bytes;
            ep->pairs = ep->pp->pairs;
            ep->fwd_steps = ep->adj_steps = ep->pp->runs.size();
            if (g_packed_enabled.load() >= 2 && (n + 1) / 2 <= kCiMaxBits) {
                CiSpace* cs;
                if (int rc = ci_space(n, ne, &cs)) return rc;
                if (cs->NB <= kCiMaxCols) {
                    if (int rc = layout_perm(ep->lay, *cs, *host_tables(ep->hx.L))) return rc;
                    ep->ci = true;
                    // excitations are real rotations and H is a real matrix:
                    // phi and lambda stay real on this path
                    ep->real = g_real_enabled.load() != 0;
                    if (ep->real) {   // the plan's bytes count complex amplitudes
                        ep->fwd_bytes *= 0.5;
                        ep->adj_bytes *= 0.5;
                    }
                    ep->cspace = cs;
                    ep->ciargs = cs->args();
                    ep->ciargs.nsplit = batched ? 1 : ci_choose_splits(ep->ciargs);
                    ep->perm = ep->lay->d_perm;
                    ep->nblk_e = cs->NA * ep->ciargs.nsplit;
                    if (ci_prepare(ep->ciargs) != 0)
                        return fail(VQE_EDEVICE, "could not enable the string-product LDS size");
                }
            }
        }
    } else {
        ep->nblk_e = blocks_for(uint64_t(1) << n);
        // number-conserving programs on a small sector: whole-state kernels
        const uint32_t ref = A->ref_bits >= 0 ? uint32_t(A->ref_bits) : uint32_t((uint64_t(1) << ne) - 1);
        if (g_packed_enabled.load() >= 1 && n <= kSmallMaxN && number_conserving(A) &&
            binom(n, __builtin_popcount(ref)) <= kSmallMaxSector && A->gates.size() <= size_t(kSmallMaxGates)) {
            SmallTables* st;
            if (int rc = small_tables(n, __builtin_popcount(ref), &st)) return rc;
            ep->small = true;
            ep->sspace.str = st->str;
            ep->sspace.rank = st->rank;
            ep->sspace.n = n;
            ep->sspace.nsec = st->nsec;
            ep->sspace.ref_rank = st->rank_h[ref];
            ep->sspace.M = int32_t(A->gates.size());
            ep->sspace.ham_lds = 0;
            // pair moves are real rotations and H is a real matrix (as on the
            // string-product path): real amplitudes unless switched off
            ep->real = g_real_enabled.load() != 0;
            ep->sspace.vbytes = ep->real ? 8 : 16;
            ep->elems = st->nsec;
            ep->nblk_e = 1;
            ep->gstride = 1;
            ep->d_gcnt = nullptr;
            ep->fwd_bytes = double(ep->sspace.vbytes) * double(st->nsec);        // phi written
            ep->adj_bytes = 2.0 * double(ep->sspace.vbytes) * double(st->nsec);  // phi, lambda read
            ep->fwd_steps = ep->adj_steps = 1;
            if (small_prepare(ep->sspace) != 0)
                return fail(VQE_EDEVICE, "could not enable the small-sector kernels' LDS size");
        }
    }
    return VQE_OK;
}

enum Phase { kPhaseFwd = 0, kPhaseHx = 1, kPhaseAdj = 2, kPhaseReduce = 3 };

// Enqueue one phase of an evaluation for `count` states at sd.
static void enqueue_packed(const EvalPlan& ep, const StateDesc* sd, int count, int phase,
                           bool grad, hipStream_t st) {
    const PackedPlan& pp = *ep.pp;
    if (phase == kPhaseFwd) {
        launch_angles(sd, count, ep.M, st);
        launch_packed_hf(sd, count, ep.lay->size, ep.real, st);
        for (size_t r = 0; r < pp.runs.size(); ++r)
            launch_packed_run(sd, count, pp.runs[r], pp.d_gates + pp.off[r], false, ep.real, st);
    } else if (phase == kPhaseHx) {
        if (ep.ci) {
            launch_ci_scatter(sd, count, ep.perm, ep.lay->size, ep.real, st);
            launch_hx_ci(sd, count, ep.ciargs, ep.real, st);
            launch_ci_gather(sd, count, ep.perm, ep.lay->size, ep.ciargs.nsplit, ep.real, st);
        } else {
            launch_hx_packed(sd, count, ep.hx, ep.hxt, ep.lay->d_base, st);
        }
    } else if (phase == kPhaseAdj) {
        if (!grad) return;
        for (size_t r = pp.runs.size(); r-- > 0;)
            launch_packed_run(sd, count, pp.runs[r], pp.d_gates + pp.off[r], true, ep.real, st);
    } else {
        launch_reduce_e(sd, count, ep.nblk_e, st);
        if (grad) launch_reduce_g(sd, count, ep.M, pp.d_gcnt_live, 0, st);
    }
}

static void enqueue_phase(const EvalPlan& ep, const StateDesc* sd, int count, int phase, bool grad,
                          hipStream_t st) {
    if (ep.small) {
        if (phase == kPhaseFwd) {
            launch_small(0, sd, count, ep.sspace, st);
        } else if (phase == kPhaseHx) {
            launch_small(1, sd, count, ep.sspace, st);
        } else if (phase == kPhaseAdj) {
            if (grad) launch_small(2, sd, count, ep.sspace, st);
        }
        // the H-apply writes the energy, the reverse sweep the per-gate sums
        return;
    }
    if (ep.packed) {
        enqueue_packed(ep, sd, count, phase, grad, st);
        return;
    }
    const uint64_t N = uint64_t(1) << ep.n;
    const AnsatzPlan& ap = *ep.ap;
    if (phase == kPhaseFwd) {
        launch_angles(sd, count, ep.M, st);
        launch_hf(sd, count, N, st);
        for (auto& s : ap.fwd_steps) {
            if (s.first == 0)
                launch_run_fwd(sd, count, ap.fwd_runs[s.second], ap.d_fwd_tg + ap.fwd_off[s.second],
                               st);
            else
                launch_pauli(sd, count, s.second, N, st);
        }
    } else if (phase == kPhaseHx) {
        if (ep.sector)
            launch_hx_sector(sd, count, ep.hx, ep.hxt, st);
        else
            launch_hx_dense(sd, count, N, ep.nblk_e, grad ? 1 : 0, st);
    } else if (phase == kPhaseAdj) {
        if (!grad) return;
        for (auto it = ap.adj_steps.rbegin(); it != ap.adj_steps.rend(); ++it) {
            if (it->first == 0)
                launch_run_adj(sd, count, ap.adj_runs[it->second],
                               ap.d_adj_tg + ap.adj_off[it->second], st);
            else
                launch_adj_pauli(sd, count, it->second, N, ap.gcnt[it->second], st);
        }
    } else {
        launch_reduce_e(sd, count, ep.nblk_e, st);
        if (grad) launch_reduce_g(sd, count, ep.M, ap.d_gcnt, 0, st);
    }
}

static int enqueue_eval(const EvalPlan& ep, const StateDesc* sd, int count, bool grad,
                        hipStream_t st) {
    for (int ph = kPhaseFwd; ph <= kPhaseReduce; ++ph) enqueue_phase(ep, sd, count, ph, grad, st);
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

// Basis index of the reference state: the ansatz's own (a mapping other than
// Jordan-Wigner moves it), else the lowest ne qubits.
static uint32_t reference_index(const vqe_ansatz* A, int ne) {
    return A->ref_bits >= 0 ? uint32_t(A->ref_bits) : uint32_t((uint64_t(1) << ne) - 1);
}

static int check_pair(const vqe_hamiltonian* H, const vqe_ansatz* A, int ne) {
    if (!H || !A) return fail(VQE_EINVAL, "null Hamiltonian or ansatz");
    if (H->n != A->n) return fail(VQE_EINVAL, "Hamiltonian and ansatz qubit counts differ");
    if (ne < 0 || ne > H->n) return fail(VQE_ERANGE, "n_electrons must be in [0, n_qubits]");
    if (A->n_electrons >= 0 && A->n_electrons != ne)
        return fail(VQE_EINVAL, "n_electrons differs from the ansatz reference");
    return VQE_OK;
}

static int64_t sector_key(int n, int ne) { return (int64_t(n) << 16) | ne; }

// A UCCSD program under a linear encoding other than Jordan-Wigner is the
// Jordan-Wigner program conjugated by the basis relabelling b = beta n, and
// so is its Hamiltonian when both come from the same integrals: energy and
// gradient are those of (H in the occupation basis, the occupation-basis
// program) from the decoded reference, which the packed sector path
// evaluates (the decoded occupations define the sector).  With the packed
// layout off, the encoded rotations run on full vectors as given.
static int resolve_encoded(const vqe_hamiltonian*& H, const vqe_ansatz*& A) {
    if (!A->occ || g_packed_enabled.load() == 0) return VQE_OK;
    const std::vector<uint32_t> key(A->enc_r, A->enc_r + A->n);
    vqe_hamiltonian* ho = nullptr;
    {
        std::lock_guard<std::mutex> lk(H->mu);
        auto it = H->occ.find(key);
        if (it != H->occ.end()) ho = it->second;
    }
    if (!ho) {
        vqe_hamiltonian* made = nullptr;
        if (int rc = hamiltonian_to_occupation(H, A->enc_c, A->enc_r, &made)) return rc;
        std::lock_guard<std::mutex> lk(H->mu);
        auto ins = H->occ.emplace(key, made);
        if (!ins.second) delete made;   // another thread made it first
        ho = ins.first->second;
    }
    H = ho;
    A = A->occ;
    return VQE_OK;
}

}  // namespace vqe

namespace vqe {

// ------------------------------------------------ allocation-free evaluation
//
// vqe_energy_grad_noalloc keeps its device workspace (phi, lambda, the
// string-product lambda planes, angles, partials, outputs and the state
// descriptor) in this array of the code object's static device memory (each
// device holds its own copy from module load to process end) and its plans
// in the records vqe_energy_grad leaves; it allocates nothing.
constexpr size_t kNoAllocBytes = size_t(64) << 20;
__device__ __align__(256) char scratch[kNoAllocBytes];

// Host-side device address of `scratch` per device ordinal, looked up once
// per device with that device current (the array's name in host code is a
// stand-in, not a device address).
constexpr int kNoAllocDevices = 64;
static char* g_scratch_ptr[kNoAllocDevices] = {};
static std::mutex g_scratch_mu;

static int scratch_address(int dev, char** out) {
    if (dev < 0 || dev >= kNoAllocDevices) return fail(VQE_ERANGE, "device ordinal beyond the scratch table");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(VQE_EDEVICE, std::string("scratch address: ") + hipGetErrorString(e));
        g_scratch_ptr[dev] = static_cast<char*>(p);
    }
    *out = g_scratch_ptr[dev];
    return VQE_OK;
}

// What the allocation-free call reuses from the last vqe_energy_grad of the
// same (device, Hamiltonian, ansatz, n_electrons): the evaluation plan and
// the state descriptor's plan pointers.
struct NoAllocRec {
    EvalPlan ep;
    StateDesc sd;
    const vqe_ansatz* prog = nullptr;   // the program the plan runs (an encoded one's occupation form)
};
static std::mutex g_noalloc_mu;
static std::map<std::tuple<int, const void*, const void*, int>, NoAllocRec> g_noalloc;

static void noalloc_forget(const void* handle) {
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    for (auto it = g_noalloc.begin(); it != g_noalloc.end();)
        if (std::get<1>(it->first) == handle || std::get<2>(it->first) == handle)
            it = g_noalloc.erase(it);
        else
            ++it;
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
    noalloc_forget(this);
    for (auto& kv : occ) delete kv.second;
    int cur = 0;
    (void)hipGetDevice(&cur);
    for (auto& kv : dev) {
        (void)hipSetDevice(kv.first);
        (void)hipFree(kv.second->groups);
        (void)hipFree(kv.second->subs);
        (void)hipFree(kv.second->tabs);
        for (auto& w : kv.second->work) {
            (void)hipFree(w.second->chunks);
            (void)hipFree(w.second->cgroups);
            (void)hipFree(w.second->csubs);
            delete w.second;
        }
        if (CiHam* c = kv.second->ci) {
            (void)hipFree(c->chunks);
            (void)hipFree(c->groups);
            (void)hipFree(c->subs);
            (void)hipFree(c->tabs);
            (void)hipFree(c->pcls);
            (void)hipFree(c->precs);
            (void)hipFree(c->rgroups);
            (void)hipFree(c->rsubs);
            (void)hipFree(c->ptabs);
            (void)hipFree(c->pcoef);
            for (auto& r : c->rm) {
                (void)hipFree(r.second->d_rm);
                (void)hipFree(r.second->d_off);
                delete r.second;
            }
            for (auto& r : c->cm) {
                (void)hipFree(r.second->d_cm);
                delete r.second;
            }
            for (auto& r : c->bh) {
                (void)hipFree(r.second->d_bh);
                delete r.second;
            }
            (void)hipFree(c->d_hopa);
            (void)hipFree(c->d_dgx);
            for (auto& r : c->dg) {
                (void)hipFree(r.second->d_row);
                (void)hipFree(r.second->d_col);
                delete r.second;
            }
            for (auto& r : c->ah) {
                (void)hipFree(r.second->d_ah);
                (void)hipFree(r.second->d_off);
                (void)hipFree(r.second->d_b);
                delete r.second;
            }
            delete c;
        }
        delete kv.second;
    }
    (void)hipSetDevice(cur);
}

vqe_ansatz::~vqe_ansatz() {
    noalloc_forget(this);
    int cur = 0;
    (void)hipGetDevice(&cur);
    for (auto& kv : dev) {
        (void)hipSetDevice(kv.first);
        (void)hipFree(kv.second->gates);
        for (auto& pl : kv.second->plans) {
            (void)hipFree(pl.second->d_fwd_tg);
            (void)hipFree(pl.second->d_adj_tg);
            (void)hipFree(pl.second->d_gcnt);
            delete pl.second;
        }
        for (auto& pl : kv.second->packed) {
            (void)hipFree(pl.second->d_gates);
            (void)hipFree(pl.second->d_gcnt);
            (void)hipFree(pl.second->d_info);
            (void)hipFree(pl.second->d_ent);
            (void)hipFree(pl.second->d_live);
            (void)hipFree(pl.second->d_tdesc);
            (void)hipFree(pl.second->d_gcnt_live);
            (void)hipFree(pl.second->d_runs);
            (void)hipFree(pl.second->d_blk);
            delete pl.second;
        }
        delete kv.second;
    }
    (void)hipSetDevice(cur);
    delete occ;
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

namespace {
// Scratch of a state-level call: descriptor plus small buffers.
struct StateCall {
    Workspace* ws = nullptr;
    Carver cv{nullptr};
    StateDesc sd{};
    StateDesc* sd_dev = nullptr;
};

int begin_state_call(const vqe_state* s, int64_t M, int64_t P, int nblk_e, StateCall* c) {
    ScratchSize sz;
    sz.add<double>(P);
    sz.add<double2>(M);
    sz.add<GateDesc>(M);
    sz.add<double>(nblk_e);
    sz.add<double>(1);
    sz.add<StateDesc>(1);
    if (int rc = workspace(s->st, 0, 0, sz.s, &c->ws)) return rc;
    c->cv = Carver{c->ws->scratch};
    std::memset(&c->sd, 0, sizeof(StateDesc));
    c->sd.phi = s->ptr;
    c->sd.n = s->n;
    c->sd.gstride = 1;
    c->sd.theta = c->cv.take<double>(P);
    c->sd.cs = c->cv.take<double2>(M);
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
    c.sd.ref = uint32_t((uint64_t(1) << ne) - 1);
    HIPCHK(hipMemcpyAsync(c.sd_dev, &c.sd, sizeof(StateDesc), hipMemcpyHostToDevice, s->st));
    launch_hf(c.sd_dev, 1, uint64_t(1) << s->n, s->st);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(s->st));
    return VQE_OK;
}

extern "C" int vqe_prepare_basis(vqe_state* s, uint64_t index) {
    if (!s) return fail(VQE_EINVAL, "null state");
    if (index >> s->n) return fail(VQE_ERANGE, "basis index beyond 2^n_qubits");
    StateCall c;
    if (int rc = begin_state_call(s, 0, 0, 1, &c)) return rc;
    c.sd.ref = uint32_t(index);
    HIPCHK(hipMemcpyAsync(c.sd_dev, &c.sd, sizeof(StateDesc), hipMemcpyHostToDevice, s->st));
    launch_hf(c.sd_dev, 1, uint64_t(1) << s->n, s->st);
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
    launch_angles(c.sd_dev, 1, 1, s->st);
    launch_pauli(c.sd_dev, 1, 0, uint64_t(1) << s->n, s->st);
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
    AnsatzPlan* ap;
    if (int rc = get_plan(A, da, tuning_for(A->n, false), &ap)) return rc;
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
    launch_angles(c.sd_dev, 1, int(M), s->st);
    for (auto& st : ap->fwd_steps) {
        if (st.first == 0)
            launch_run_fwd(c.sd_dev, 1, ap->fwd_runs[st.second], ap->d_fwd_tg + ap->fwd_off[st.second],
                           s->st);
        else
            launch_pauli(c.sd_dev, 1, st.second, N, s->st);
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
    const uint64_t N = uint64_t(1) << s->n;
    const int nblk = blocks_for(N);
    StateCall c;
    if (int rc = begin_state_call(s, 0, 0, nblk, &c)) return rc;
    c.sd.groups = dh->groups;
    c.sd.subs = dh->subs;
    c.sd.tabs = dh->tabs;
    c.sd.G = int32_t(H->groups.size());
    c.sd.nsub = int32_t(H->subs.size());
    c.sd.ntab = int32_t(H->tabs.size());
    HIPCHK(hipMemcpyAsync(c.sd_dev, &c.sd, sizeof(StateDesc), hipMemcpyHostToDevice, s->st));
    launch_hx_dense(c.sd_dev, 1, N, nblk, 0, s->st);
    launch_reduce_e(c.sd_dev, 1, nblk, s->st);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(energy, c.sd.out_e, sizeof(double), hipMemcpyDeviceToHost, s->st));
    HIPCHK(hipStreamSynchronize(s->st));
    if (!std::isfinite(*energy)) return fail(VQE_ENUMERIC, "non-finite expectation value");
    return VQE_OK;
}

namespace {
// Set-up of a single-state evaluation: plan, workspace, descriptor (uploaded
// with theta); `extra` reserves more scratch for the caller.
struct SingleEval {
    EvalPlan ep;
    DevHam* dh = nullptr;
    DevAnsatz* da = nullptr;
    Workspace* ws = nullptr;
    Carver cv{nullptr};
    StateDesc sd{};
    StateDesc* sd_dev = nullptr;
};

int setup_single(const vqe_hamiltonian* H, const vqe_ansatz* A, int ne, const double* theta,
                 hipStream_t st, const ScratchSize& extra, SingleEval* e) {
    const int n = H->n;
    const int64_t M = int64_t(A->gates.size()), P = A->n_params;
    if (int rc = dev_ham(H, &e->dh)) return rc;
    if (int rc = make_eval_plan(A, ne, false, &e->ep)) return rc;
    small_fit_ham(&e->ep, H);
    if (int rc = dev_ansatz(A, &e->da)) return rc;
    const EvalPlan& ep = e->ep;
    HxWork* hw = nullptr;
    if (ep.sector)
        if (int rc = ham_chunks(H, e->dh, ep.hx.L, &hw)) return rc;
    ScratchSize sz = extra;
    sz.add<double>(P);
    sz.add<double2>(M);
    sz.add<double>(ep.nblk_e);
    sz.add<double>(size_t(std::max<int64_t>(M, 1)) * ep.gstride);
    sz.add<double>(1);
    sz.add<double>(M);
    sz.add<StateDesc>(1);
    const size_t sbytes = sizeof(double2) * size_t(ep.elems);
    if (int rc = workspace(st, sbytes, ep.ci ? sbytes * size_t(ep.ciargs.nsplit) : sbytes, sz.s,
                           &e->ws)) return rc;
    Workspace* ws = e->ws;
    // the full-layout sector H-apply writes only in-sector entries: lambda
    // must be zero elsewhere (the packed layout holds nothing else)
    if (ep.packed) {
        ws->lam_zero_key = -1;
    } else if (ep.sector && ws->lam_zero_key != sector_key(n, ne)) {
        launch_fill_zero(ws->lam, ws->state_bytes / sizeof(double2), st);
        ws->lam_zero_key = sector_key(n, ne);
    } else if (!ep.sector) {
        ws->lam_zero_key = -1;
    }
    e->cv = Carver{ws->scratch};
    StateDesc& sd = e->sd;
    sd = StateDesc{};
    sd.phi = ws->phi;
    sd.lam = ws->lam;
    sd.aux = ws->aux;
    if (ep.ci) {
        CiHam* ch;
        if (int rc = ci_ham(H, e->dh, &ch)) return rc;
        sd.ci_chunks = ch->chunks;
        sd.ci_groups = ch->groups;
        sd.ci_subs = ch->subs;
        sd.ci_tabs = ch->tabs;
        sd.ci_nchunks = ch->nchunks;
        sd.ci_pcls = ch->pcls;
        sd.ci_precs = ch->precs;
        sd.ci_rgroups = ch->rgroups;
        sd.ci_rsubs = ch->rsubs;
        sd.ci_ptabs = ch->ptabs;
        sd.ci_pcoef = ch->pcoef;
        sd.ci_npcls = ch->npcls;
        sd.ci_psplit = ch->psplit ? 1 : 0;
        RowMoves* rm;
        if (int rc = ci_rowmoves(H, ch, *ep.cspace, &rm)) return rc;
        sd.ci_rm = rm->d_rm;
        sd.ci_rm_off = rm->d_off;
        ColMoves* cm;
        if (int rc = ci_colmoves(H, ch, *ep.cspace, &cm)) return rc;
        sd.ci_cm = cm->d_cm;
        sd.ci_ncm = cm->ncm;
        BetaHops* bh;
        if (int rc = ci_betahops(H, ch, *ep.cspace, &bh)) return rc;
        sd.ci_bh = bh->d_bh;
        sd.ci_nbh = bh->nbh;
        sd.ci_hopa = ch->d_hopa;
        AlphaHops* ahp;
        if (int rc = ci_alphahops(H, ch, *ep.cspace, &ahp)) return rc;
        sd.ci_ah = ahp->d_ah;
        sd.ci_ah_off = ahp->d_off;
        sd.ci_ahb = ahp->d_b;
        if (ch->diag.on) {
            DiagParts* dp;
            if (int rc = ci_diag(H, ch, *ep.cspace, &dp)) return rc;
            sd.ci_dgr = dp->d_row;
            sd.ci_dgc = dp->d_col;
            sd.ci_dgx = ch->d_dgx;
        }
    }
    Carver& cv = e->cv;
    sd.gates = e->da->gates;
    sd.theta = cv.take<double>(P);
    sd.cs = cv.take<double2>(M);
    sd.groups = e->dh->groups;
    sd.subs = e->dh->subs;
    sd.tabs = e->dh->tabs;
    if (hw) {
        sd.chunks = hw->chunks;
        sd.cgroups = hw->cgroups;
        sd.csubs = hw->csubs;
        sd.nb = hw->count;
    }
    sd.part_e = cv.take<double>(ep.nblk_e);
    sd.part_g = cv.take<double>(size_t(std::max<int64_t>(M, 1)) * ep.gstride);
    sd.out_e = cv.take<double>(1);
    sd.out_g = cv.take<double>(M);
    sd.n = n;
    sd.G = int32_t(H->groups.size());
    sd.nsub = int32_t(H->subs.size());
    sd.ntab = int32_t(H->tabs.size());
    sd.M = int32_t(M);
    sd.ne = ne;
    sd.ref = reference_index(A, ne);
    sd.gstride = ep.gstride;
    e->sd_dev = cv.take<StateDesc>(1);
    if (P > 0)
        HIPCHK(hipMemcpyAsync(const_cast<double*>(sd.theta), theta, sizeof(double) * P,
                              hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(e->sd_dev, &sd, sizeof(StateDesc), hipMemcpyHostToDevice, st));
    return VQE_OK;
}
}  // namespace

extern "C" int vqe_energy_grad(const vqe_hamiltonian* H, const vqe_ansatz* A, int ne,
                               const double* theta, double* energy, double* grad, void* stream) {
    if (int rc = check_pair(H, A, ne)) return rc;
    if (!energy) return fail(VQE_EINVAL, "null energy pointer");
    if (A->n_params > 0 && !theta) return fail(VQE_EINVAL, "null theta");
    if (!finite_all(theta, A->n_params)) return fail(VQE_EINVAL, "theta has a non-finite entry");
    const void* const key_h = H;   // the allocation-free call is keyed by the caller's handles
    const void* const key_a = A;
    if (int rc = resolve_encoded(H, A)) return rc;
    hipStream_t st = (hipStream_t)stream;
    const int64_t M = int64_t(A->gates.size()), P = A->n_params;
    SingleEval e;
    if (int rc = setup_single(H, A, ne, theta, st, ScratchSize{}, &e)) return rc;
    {   // the plans the allocation-free call reuses
        int dev = 0;
        HIPCHK(hipGetDevice(&dev));
        std::lock_guard<std::mutex> lk(g_noalloc_mu);
        g_noalloc[std::make_tuple(dev, key_h, key_a, ne)] = NoAllocRec{e.ep, e.sd, A};
    }
    if (int rc = enqueue_eval(e.ep, e.sd_dev, 1, grad != nullptr, st)) return rc;
    std::vector<double> raw(std::max<int64_t>(M, 1));
    HIPCHK(hipMemcpyAsync(energy, e.sd.out_e, sizeof(double), hipMemcpyDeviceToHost, st));
    if (grad && M > 0)
        HIPCHK(hipMemcpyAsync(raw.data(), e.sd.out_g, sizeof(double) * M, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    bool ok = std::isfinite(*energy);
    if (grad) {
        accumulate_grad(A, raw.data(), grad);
        ok = ok && finite_all(grad, P);
    }
    if (!ok) return fail(VQE_ENUMERIC, "non-finite energy or gradient");
    return VQE_OK;
}

extern "C" int vqe_energy_grad_noalloc(const vqe_hamiltonian* H, const vqe_ansatz* A, int ne,
                                       const double* theta, double* energy, double* grad, void* stream) {
    if (int rc = check_pair(H, A, ne)) return rc;
    if (!energy) return fail(VQE_EINVAL, "null energy pointer");
    if (A->n_params > 0 && !theta) return fail(VQE_EINVAL, "null theta");
    if (!finite_all(theta, A->n_params)) return fail(VQE_EINVAL, "theta has a non-finite entry");
    const void* const key_h = H;
    const void* const key_a = A;
    hipStream_t st = (hipStream_t)stream;
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    NoAllocRec rec;
    {
        std::lock_guard<std::mutex> lk(g_noalloc_mu);
        auto it = g_noalloc.find(std::make_tuple(dev, key_h, key_a, ne));
        if (it == g_noalloc.end())
            return fail(VQE_EINVAL, "no plan for this Hamiltonian, ansatz and n_electrons on this device: "
                                    "call vqe_energy_grad with them once first");
        rec = it->second;
    }
    A = rec.prog;   // the program the recorded plan runs
    const int64_t M = int64_t(A->gates.size()), P = A->n_params;
    const EvalPlan& ep = rec.ep;
    // the workspace the regular call carves, in the scratch array
    const size_t elems = size_t(ep.elems);
    const size_t planes = ep.ci ? size_t(ep.ciargs.nsplit) : 1;
    ScratchSize sz;
    sz.add<double2>(elems);
    sz.add<double2>(elems);
    sz.add<double2>(elems * planes);
    sz.add<double>(size_t(P));
    sz.add<double2>(size_t(M));
    sz.add<double>(size_t(ep.nblk_e));
    sz.add<double>(size_t(std::max<int64_t>(M, 1)) * size_t(ep.gstride));
    sz.add<double>(1);
    sz.add<double>(size_t(M));
    sz.add<StateDesc>(1);
    if (sz.s > kNoAllocBytes)
        return fail(VQE_ERANGE, "the allocation-free evaluation needs " + std::to_string(sz.s) +
                                    " bytes of scratch; it has " + std::to_string(kNoAllocBytes));
    char* base = nullptr;
    if (int rc = scratch_address(dev, &base)) return rc;
    Carver cv{base};
    StateDesc sd = rec.sd;
    sd.phi = cv.take<double2>(elems);
    sd.lam = cv.take<double2>(elems);
    sd.aux = cv.take<double2>(elems * planes);
    sd.theta = cv.take<double>(size_t(P));
    sd.cs = cv.take<double2>(size_t(M));
    sd.part_e = cv.take<double>(size_t(ep.nblk_e));
    sd.part_g = cv.take<double>(size_t(std::max<int64_t>(M, 1)) * size_t(ep.gstride));
    sd.out_e = cv.take<double>(1);
    sd.out_g = cv.take<double>(size_t(M));
    StateDesc* sd_dev = cv.take<StateDesc>(1);
    // the array keeps the last call's contents: the full-layout sector
    // H-apply writes only in-sector entries, so lambda starts at zero
    if (ep.sector && !ep.packed) launch_fill_zero(sd.lam, elems, st);
    if (P > 0)
        HIPCHK(hipMemcpyAsync(const_cast<double*>(sd.theta), theta, sizeof(double) * P,
                              hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(sd_dev, &sd, sizeof(StateDesc), hipMemcpyHostToDevice, st));
    if (int rc = enqueue_eval(ep, sd_dev, 1, grad != nullptr, st)) return rc;
    HIPCHK(hipMemcpyAsync(energy, sd.out_e, sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    bool ok = std::isfinite(*energy);
    if (grad) {   // per-gate sums in fixed-size pieces, added in gate order
        std::fill(grad, grad + P, 0.0);
        constexpr int64_t kPiece = 2048;
        double raw[kPiece];
        for (int64_t j0 = 0; j0 < M; j0 += kPiece) {
            const int64_t cnt = std::min(kPiece, M - j0);
            HIPCHK(hipMemcpyAsync(raw, sd.out_g + j0, sizeof(double) * cnt, hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
            for (int64_t k = 0; k < cnt; ++k) {
                const GateDesc& g = A->gates[size_t(j0 + k)];
                grad[g.param] += (g.type == kExcitation ? 2.0 : 1.0) * g.scale * raw[k];
            }
        }
        ok = ok && finite_all(grad, P);
    }
    if (!ok) return fail(VQE_ENUMERIC, "non-finite energy or gradient");
    return VQE_OK;
}

// The single-launch zero-angle sweep of a packed plan (pool gradients).
static int pool_sweep(const vqe_ansatz* pool, PackedPlan* p, const PoolSweep** out) {
    std::lock_guard<std::mutex> lk(pool->mu);
    if (p->d_runs) {
        *out = &p->sweep;
        return VQE_OK;
    }
    std::vector<int32_t> blk, first;
    int maxe = 1;
    for (size_t r = 0; r < p->runs.size(); ++r) {
        first.push_back(int32_t(blk.size()));
        blk.insert(blk.end(), size_t(p->runs[r].ntiles), int32_t(r));
        maxe = std::max(maxe, p->runs[r].max_entries);
    }
    if (blk.size() > size_t(1) << 30) return fail(VQE_ERANGE, "pool sweep: too many tiles");
    const int nblk = int(blk.size());
    blk.insert(blk.end(), first.begin(), first.end());
    PoolSweep ps{};
    ps.shape = packed_shape((maxe + 1) / 2, 256);
    if (ps.shape < 0) return fail(VQE_EINVAL, "pool sweep: block too large for the run kernels");
    PackedRun* d_runs = nullptr;
    int32_t* d_blk = nullptr;
    int rc = upload(&d_runs, p->runs.data(), p->runs.size());
    if (!rc) rc = upload(&d_blk, blk.data(), blk.size());
    if (rc) {
        (void)hipFree(d_runs);
        (void)hipFree(d_blk);
        return rc;
    }
    ps.runs = d_runs;
    ps.blk_run = d_blk;
    ps.blk0 = d_blk + nblk;
    ps.gates = p->d_gates;
    ps.nblk = nblk;
    ps.lds = size_t(maxe) * sizeof(double2) * 2;
    p->d_runs = d_runs;
    p->d_blk = d_blk;
    p->sweep = ps;
    *out = &p->sweep;
    return VQE_OK;
}

namespace {
// The pool gradient, optionally timed: with reps > 0 the whole sequence runs
// reps times with HIP events between its phases (forward, H-apply, pool
// sweep, reductions); ms receives their means and work the forward and
// pool-sweep algorithmic bytes and the sweep's launch count.
int pool_gradient_impl(const vqe_hamiltonian* H, const vqe_ansatz* A, const vqe_ansatz* pool,
                       int ne, const double* theta, double* energy, double* pool_grad,
                       void* stream, int reps, double* ms, double* work) {
    if (int rc = check_pair(H, A, ne)) return rc;
    if (!pool || !energy || !pool_grad) return fail(VQE_EINVAL, "null pointer argument");
    if (pool->n != H->n) return fail(VQE_EINVAL, "pool and Hamiltonian qubit counts differ");
    if (pool->n_electrons >= 0 && pool->n_electrons != ne)
        return fail(VQE_EINVAL, "n_electrons differs from the pool's reference");
    if (pool->n_params < 1) return fail(VQE_ERANGE, "pool has no parameters");
    if (A->n_params > 0 && !theta) return fail(VQE_EINVAL, "null theta");
    if (!finite_all(theta, A->n_params)) return fail(VQE_EINVAL, "theta has a non-finite entry");
    hipStream_t st = (hipStream_t)stream;
    const int n = H->n;
    const int64_t Mp = int64_t(pool->gates.size()), Pp = pool->n_params;
    // the pool's reverse-sweep plan in the evaluation's layout
    EvalPlan probe;
    if (int rc = make_eval_plan(A, ne, false, &probe)) return rc;
    DevAnsatz* dp;
    if (int rc = dev_ansatz(pool, &dp)) return rc;
    const Tuning tn = tuning_for(n, false);
    PackedPlan* ppool = nullptr;
    const PoolSweep* psw = nullptr;
    AnsatzPlan* apool = nullptr;
    if (probe.packed) {
        const int need = packed_min_L(pool, ne);
        if (need < 0 || need > probe.hx.L || !pool->sector_conserving)
            return fail(VQE_EINVAL, "pool does not fit the packed sector evaluation of this ansatz");
        if (int rc = packed_plan(pool, dp, *probe.lay, tn, &ppool)) return rc;
        if (int rc = pool_sweep(pool, ppool, &psw)) return rc;
    } else {
        if (int rc = get_plan(pool, dp, tn, &apool)) return rc;
    }
    const int32_t gstride_p = probe.packed ? ppool->gstride : apool->gstride;
    ScratchSize extra;
    extra.add<double>(Pp);                                       // zero angles
    extra.add<double2>(Mp);                                      // their (cos, sin)
    extra.add<double>(size_t(Mp) * size_t(gstride_p));           // pool partials
    extra.add<double>(Mp);                                       // pool raw sums
    extra.add<StateDesc>(1);
    SingleEval e;
    if (int rc = setup_single(H, A, ne, theta, st, extra, &e)) return rc;
    StateDesc sp = e.sd;   // the same phi, lambda; the pool's gates, angles and partials
    sp.gates = dp->gates;
    sp.theta = e.cv.take<double>(Pp);
    sp.cs = e.cv.take<double2>(Mp);
    sp.part_g = e.cv.take<double>(size_t(Mp) * size_t(gstride_p));
    sp.out_g = e.cv.take<double>(Mp);
    sp.M = int32_t(Mp);
    sp.gstride = gstride_p;
    StateDesc* sp_dev = e.cv.take<StateDesc>(1);
    const std::vector<double> zeros(size_t(Pp), 0.0);
    HIPCHK(hipMemcpyAsync(const_cast<double*>(sp.theta), zeros.data(), sizeof(double) * Pp,
                          hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(sp_dev, &sp, sizeof(StateDesc), hipMemcpyHostToDevice, st));
    const EvalPlan& ep = e.ep;
    // phi = U(theta)|HF>, lambda = H phi, then the pool's gates at angle 0
    // swept on (phi, lambda): each leaves both unchanged and yields
    // Re <lambda|A_k phi>, the derivative of appending A_k after U(theta).
    // Packed layout: one read-only launch over every run and tile; full
    // layout: the reverse-sweep kernels at zero angles.
    auto phase = [&](int ph) {
        if (ph == 0) {
            enqueue_phase(ep, e.sd_dev, 1, kPhaseFwd, false, st);
        } else if (ph == 1) {
            enqueue_phase(ep, e.sd_dev, 1, kPhaseHx, true, st);
        } else if (ph == 2) {
            if (probe.packed) {
                launch_pool_sweep(sp_dev, 1, *psw, ep.hxt, ep.lay->d_base, ep.real, st);
            } else {
                launch_angles(sp_dev, 1, int(Mp), st);
                const uint64_t N = uint64_t(1) << n;
                for (auto it = apool->adj_steps.rbegin(); it != apool->adj_steps.rend(); ++it) {
                    if (it->first == 0)
                        launch_run_adj(sp_dev, 1, apool->adj_runs[it->second],
                                       apool->d_adj_tg + apool->adj_off[it->second], st);
                    else
                        launch_adj_pauli(sp_dev, 1, it->second, N, apool->gcnt[it->second], st);
                }
            }
        } else {
            launch_reduce_e(e.sd_dev, 1, ep.nblk_e, st);
            launch_reduce_g(sp_dev, 1, int(Mp), probe.packed ? ppool->d_gcnt : apool->d_gcnt, 0,
                            st);
        }
    };
    if (reps <= 0) {
        for (int ph = 0; ph < 4; ++ph) phase(ph);
        HIPCHK(hipGetLastError());
    } else {
        hipEvent_t ev[5];
        for (auto& x : ev) HIPCHK(hipEventCreate(&x));
        double acc[4] = {0, 0, 0, 0};
        int rc = VQE_OK;
        for (int r = 0; r < reps && rc == VQE_OK; ++r) {
            (void)hipEventRecord(ev[0], st);
            for (int ph = 0; ph < 4; ++ph) {
                phase(ph);
                (void)hipEventRecord(ev[ph + 1], st);
            }
            hipError_t err = hipEventSynchronize(ev[4]);
            if (err == hipSuccess) err = hipGetLastError();
            if (err != hipSuccess) {
                rc = fail(VQE_EDEVICE, std::string("profile: ") + hipGetErrorString(err));
                break;
            }
            for (int ph = 0; ph < 4; ++ph) {
                float t = 0.f;
                (void)hipEventElapsedTime(&t, ev[ph], ev[ph + 1]);
                acc[ph] += t;
            }
        }
        for (auto& x : ev) (void)hipEventDestroy(x);
        if (rc) return rc;
        for (int ph = 0; ph < 4; ++ph) ms[ph] = acc[ph] / reps;
        work[0] = ep.fwd_bytes;
        work[1] = 0.0;
        work[2] = probe.packed ? ppool->sweep_bytes * (ep.real ? 0.5 : 1.0) : apool->adj_bytes;
        work[3] = double(probe.packed ? 1 : apool->adj_steps.size());
    }
    std::vector<double> raw(static_cast<size_t>(Mp));
    HIPCHK(hipMemcpyAsync(energy, e.sd.out_e, sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(raw.data(), sp.out_g, sizeof(double) * Mp, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    accumulate_grad(pool, raw.data(), pool_grad);
    if (!std::isfinite(*energy) || !finite_all(pool_grad, Pp))
        return fail(VQE_ENUMERIC, "non-finite energy or pool gradient");
    return VQE_OK;
}

}  // namespace

extern "C" int vqe_pool_gradient(const vqe_hamiltonian* H, const vqe_ansatz* A,
                                 const vqe_ansatz* pool, int ne, const double* theta,
                                 double* energy, double* pool_grad, void* stream) {
    return pool_gradient_impl(H, A, pool, ne, theta, energy, pool_grad, stream, 0, nullptr,
                              nullptr);
}

extern "C" int vqe_pool_gradient_profile(const vqe_hamiltonian* H, const vqe_ansatz* A,
                                         const vqe_ansatz* pool, int ne, const double* theta,
                                         int reps, double* ms, double* work, void* stream) {
    if (!ms || !work) return fail(VQE_EINVAL, "null pointer argument");
    if (reps < 1) return fail(VQE_ERANGE, "reps must be >= 1");
    if (!pool) return fail(VQE_EINVAL, "null pool");
    double e = 0.0;
    std::vector<double> g(static_cast<size_t>(std::max(pool->n_params, 1)));
    return pool_gradient_impl(H, A, pool, ne, theta, &e, g.data(), stream, reps, ms, work);
}

// ===================================================================== batch

namespace vqe {

// Persistent batch passes (k_persist.hip): mode 1 = on where the device
// reports its XCDs, 0 = one launch per run and size class (default: measured
// faster on the 512-state batch).
static std::atomic<int> g_persist_mode{0};
static std::atomic<int> g_persist_L{12};
static std::atomic<int> g_persist_spin{1 << 20};

// Queue of each raw XCC id on a device: a probe launch of many one-wave
// workgroups records the id each ran on; ids are numbered in ascending order.
// The persistent passes are used only when the probe finds as many distinct
// ids as the device has XCDs of 32 CUs (every workgroup of one queue then
// shares one L2).
struct XccMap {
    int nq = 0;
    std::vector<int32_t> map;   // [kPqMaxXcc]
    int32_t* d_map = nullptr;
};
static std::mutex g_xcc_mu;
static std::map<int, XccMap*> g_xcc;

static int xcc_map(XccMap** out) {
    int dev;
    if (int rc = current_device(&dev)) return rc;
    std::lock_guard<std::mutex> lk(g_xcc_mu);
    XccMap*& m = g_xcc[dev];
    if (m) {
        *out = m;
        return VQE_OK;
    }
    int cus = 0;
    HIPCHK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    const int blocks = 4096;
    int32_t* d = nullptr;
    HIPCHK(hipMalloc(&d, sizeof(int32_t) * blocks));
    launch_xcc_probe(d, blocks, nullptr);
    std::vector<int32_t> ids(blocks, -1);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpy(ids.data(), d, sizeof(int32_t) * blocks, hipMemcpyDeviceToHost);
    (void)hipFree(d);
    HIPCHK(e);
    auto* x = new XccMap();
    x->map.assign(kPqMaxXcc, -1);
    std::vector<int32_t> seen;
    bool ok = true;
    for (int32_t v : ids) {
        if (v < 0 || v >= kPqMaxXcc) ok = false;
        else if (std::find(seen.begin(), seen.end(), v) == seen.end()) seen.push_back(v);
    }
    std::sort(seen.begin(), seen.end());
    if (ok && cus % 32 == 0 && int(seen.size()) == cus / 32) {
        for (size_t i = 0; i < seen.size(); ++i) x->map[size_t(seen[i])] = int32_t(i);
        x->nq = int(seen.size());
        if (int rc = upload(&x->d_map, x->map.data(), x->map.size())) {
            delete x;
            return rc;
        }
    }
    m = x;
    *out = m;
    return VQE_OK;
}

}  // namespace vqe

struct vqe_batch {
    int S = 0;
    int dev = 0;
    hipStream_t user = nullptr;     // caller's stream: evaluations are ordered after its work
    hipStream_t st = nullptr;       // the batch's own stream (graph capture and launches)
    hipEvent_t user_ev = nullptr;
    hipEvent_t done_ev = nullptr;   // end of a device-resident evaluation (the caller's stream waits)
    std::vector<const vqe_ansatz*> A;
    std::vector<int64_t> poff;      // parameter offsets [S+1]
    std::vector<int64_t> goff;      // gate offsets [S+1]
    std::vector<char*> allocs;      // every device allocation of the batch
    std::vector<hipStream_t> side;  // fork streams of the graph capture
    std::vector<hipEvent_t> events;
    struct Class {
        EvalPlan ep;
        int k0 = 0, count = 0;      // slice of the ordered descriptor table
    };
    std::vector<Class> classes;
    StateDesc* sd_dev = nullptr;
    double* theta_dev = nullptr;
    double* e_dev = nullptr;
    double* g_dev = nullptr;        // raw per-gate sums, concatenated
    // parameter -> (gate, coefficient) lists of the whole batch, gate order
    // within a parameter (device-resident gradients; built at first use)
    int64_t* pg_start = nullptr;
    int64_t* pg_gate = nullptr;
    double* pg_coef = nullptr;
    double* theta_h = nullptr;      // pinned staging
    double* e_h = nullptr;
    double* g_h = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    double work[8] = {0, 0, 0, 0, 0, 0, 0, 0};  // algorithmic work of one evaluation
    // persistent gate passes (every class's runs in one launch per direction)
    struct Persist {
        bool on = false;
        int nq = 0, pmax = 1;
        size_t lds[2] = {0, 0};      // forward, reverse
        int grid[2] = {0, 0};
        PqArgs args[2]{};
        int32_t* cnt = nullptr;      // [head nq | done S] x 2 passes, then err [2 nq]
        int ncnt = 0;
        int32_t* err_h = nullptr;    // pinned copy of the error flags
        std::vector<PqItem> items[2];   // host copies (tests may alter one need)
        std::vector<int32_t> qoff[2];
    } pq;
    ~vqe_batch() {
        int cur = 0;
        (void)hipGetDevice(&cur);
        (void)hipSetDevice(dev);
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        for (hipEvent_t e : events) (void)hipEventDestroy(e);
        for (hipStream_t s : side) (void)hipStreamDestroy(s);
        if (user_ev) (void)hipEventDestroy(user_ev);
        if (done_ev) (void)hipEventDestroy(done_ev);
        if (st) (void)hipStreamDestroy(st);
        for (char* p : allocs) (void)hipFree(p);
        (void)hipHostFree(theta_h);
        (void)hipHostFree(e_h);
        (void)hipHostFree(g_h);
        (void)hipHostFree(pq.err_h);
        (void)hipSetDevice(cur);
    }
};

namespace {
bool same_program(const vqe_ansatz* a, const vqe_ansatz* b) {
    return a->n == b->n && a->n_params == b->n_params && a->n_electrons == b->n_electrons &&
           a->sector_conserving == b->sector_conserving && a->gates.size() == b->gates.size() &&
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

// Work queues of the persistent passes: every state goes to one queue (one
// XCD), heaviest first to the queue with the least work so far (work: the
// class's live-tile entries times gates over its runs); a queue lists, run
// step by run step, the live tiles of each of its states (forward: run r at
// step r; reverse: run R - 1 - step), each with the count of the state's
// tiles that must be done before it starts (all tiles of the runs before it
// in that pass).
int build_persist(vqe_batch* b, const XccMap& xm) {
    auto& P = b->pq;
    const int S = b->S, nq = xm.nq;
    const size_t C = b->classes.size();
    std::vector<PqRun> runs;
    std::vector<size_t> run0(C);
    size_t cap = 1;
    int max_stride = 1, max_ng = 1;
    std::vector<double> cw(C, 0.0);
    std::vector<std::vector<int32_t>> pre(C), suf(C);   // tiles before / after each run
    for (size_t c = 0; c < C; ++c) {
        const EvalPlan& ep = b->classes[c].ep;
        const PackedPlan& pp = *ep.pp;
        run0[c] = runs.size();
        const size_t R = pp.runs.size();
        pre[c].assign(R + 1, 0);
        suf[c].assign(R + 1, 0);
        for (size_t r = 0; r < R; ++r) {
            PqRun q{};
            q.r = pp.runs[r];
            q.pg = pp.d_gates + pp.off[r];
            q.base = ep.lay->d_base;
            runs.push_back(q);
            pre[c][r + 1] = pre[c][r] + pp.runs[r].nlive;
            cw[c] += pp.run_work[r];
        }
        for (size_t r = R; r-- > 0;) suf[c][r] = suf[c][r + 1] + pp.runs[r].nlive;
        cap = std::max(cap, size_t(pp.max_entries));
        max_stride = std::max(max_stride, pp.max_stride);
        max_ng = std::max(max_ng, pp.max_gates);
    }
    std::vector<int> cls_of(S, -1);
    for (size_t c = 0; c < C; ++c)
        for (int k = b->classes[c].k0; k < b->classes[c].k0 + b->classes[c].count; ++k) cls_of[k] = int(c);
    std::vector<int> ord(S);
    for (int k = 0; k < S; ++k) ord[k] = k;
    std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return cw[cls_of[x]] > cw[cls_of[y]]; });
    std::vector<double> load(nq, 0.0);
    std::vector<std::vector<int>> qs(nq);
    for (int k : ord) {
        const int q = int(std::min_element(load.begin(), load.end()) - load.begin());
        load[q] += cw[cls_of[k]];
        qs[q].push_back(k);
    }
    for (auto& v : qs) std::sort(v.begin(), v.end());
    for (int pass = 0; pass < 2; ++pass) {
        auto& items = P.items[pass];
        auto& qoff = P.qoff[pass];
        items.clear();
        qoff.assign(1, 0);
        for (int q = 0; q < nq; ++q) {
            size_t maxR = 0;
            for (int k : qs[q]) maxR = std::max(maxR, b->classes[cls_of[k]].ep.pp->runs.size());
            for (size_t step = 0; step < maxR; ++step)
                for (int k : qs[q]) {
                    const int c = cls_of[k];
                    const PackedPlan& pp = *b->classes[c].ep.pp;
                    const size_t R = pp.runs.size();
                    if (step >= R) continue;
                    const size_t r = pass == 0 ? step : R - 1 - step;
                    const int32_t need = pass == 0 ? pre[c][r] : suf[c][r + 1];
                    for (int32_t t = 0; t < pp.runs[r].nlive; ++t)
                        items.push_back(PqItem{int32_t(k), int32_t(run0[c] + r), t, need});
                }
            if (items.size() > size_t(INT32_MAX)) return fail(VQE_ERANGE, "persistent pass: too many items");
            qoff.push_back(int32_t(items.size()));
        }
    }
    PqRun* d_runs = nullptr;
    PqItem* d_items[2] = {nullptr, nullptr};
    int32_t* d_qoff[2] = {nullptr, nullptr};
    if (int rc = dalloc(b, &d_runs, runs.size())) return rc;
    HIPCHK(hipMemcpy(d_runs, runs.data(), sizeof(PqRun) * runs.size(), hipMemcpyHostToDevice));
    for (int pass = 0; pass < 2; ++pass) {
        if (int rc = dalloc(b, &d_items[pass], P.items[pass].size())) return rc;
        if (int rc = dalloc(b, &d_qoff[pass], P.qoff[pass].size())) return rc;
        HIPCHK(hipMemcpy(d_items[pass], P.items[pass].data(), sizeof(PqItem) * P.items[pass].size(),
                         hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(d_qoff[pass], P.qoff[pass].data(), sizeof(int32_t) * P.qoff[pass].size(),
                         hipMemcpyHostToDevice));
    }
    // counters: ctl[1] | per pass: head[nq], done[S] | err[2 nq]
    P.ncnt = 1 + 2 * (nq + S) + 2 * nq;
    if (int rc = dalloc(b, &P.cnt, size_t(P.ncnt))) return rc;
    HIPCHK(hipMemset(P.cnt, 0, sizeof(int32_t) * size_t(P.ncnt)));
    const int32_t spin = g_persist_spin.load();
    HIPCHK(hipMemcpy(P.cnt, &spin, sizeof(int32_t), hipMemcpyHostToDevice));
    HIPCHK(hipHostMalloc(&P.err_h, sizeof(int32_t) * 2 * nq));
    P.nq = nq;
    P.pmax = pq_pmax_for(max_stride);
    int cus = 0;
    HIPCHK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, b->dev));
    for (int pass = 0; pass < 2; ++pass) {
        PqArgs& a = P.args[pass];
        a.sd = b->sd_dev;
        a.runs = d_runs;
        a.items = d_items[pass];
        a.qoff = d_qoff[pass];
        a.qmap = xm.d_map;
        a.head = P.cnt + 1 + pass * (nq + S);
        a.done = a.head + nq;
        a.err = P.cnt + 1 + 2 * (nq + S) + pass * nq;
        a.tabs = b->classes[0].ep.hxt;
        a.ctl = P.cnt;
        a.cap = int32_t(cap);
        a.max_ng = int32_t(max_ng);
        P.lds[pass] = (size_t(pass + 1) * cap + 2 * size_t(max_ng)) * sizeof(double2) +
                      (pass == 1 ? size_t(max_ng) * sizeof(double) : 0);
        int bpc = 0;
        if (pq_prepare(pass + 1, P.pmax, P.lds[pass], &bpc) != 0)
            return fail(VQE_EDEVICE, "persistent pass: kernel does not fit " + std::to_string(P.lds[pass]) +
                                         " bytes of LDS");
        P.grid[pass] = bpc * cus;
    }
    P.on = true;
    return VQE_OK;
}

// Enqueue fn(class, stream) for every class: with fork, on the side streams
// (heaviest class first, each on the stream with the least work so far)
// between a fork from b->st and a join back into it; else in order on st.
template <class F>
int for_classes(vqe_batch* b, bool fork, hipStream_t st, int fork_id, F fn) {
    if (!fork) {
        for (auto& c : b->classes) fn(c, st);
        return VQE_OK;
    }
    const size_t C = b->classes.size();
    const size_t ns = b->side.size();
    hipEvent_t* ev = b->events.data() + size_t(fork_id) * (ns + 1);
    HIPCHK(hipEventRecord(ev[0], st));
    for (size_t i = 0; i < ns; ++i) HIPCHK(hipStreamWaitEvent(b->side[i], ev[0], 0));
    std::vector<size_t> ord(C);
    std::vector<double> w(C), load(ns, 0.0);
    for (size_t i = 0; i < C; ++i) {
        ord[i] = i;
        w[i] = double(b->classes[i].count) * (b->classes[i].ep.fwd_bytes + b->classes[i].ep.adj_bytes);
    }
    std::stable_sort(ord.begin(), ord.end(), [&](size_t a, size_t c) { return w[a] > w[c]; });
    for (size_t i : ord) {
        const size_t k = size_t(std::min_element(load.begin(), load.end()) - load.begin());
        load[k] += w[i];
        fn(b->classes[i], b->side[k]);
    }
    for (size_t i = 0; i < ns; ++i) {
        HIPCHK(hipEventRecord(ev[1 + i], b->side[i]));
        HIPCHK(hipStreamWaitEvent(st, ev[1 + i], 0));
    }
    return VQE_OK;
}

// One phase of an evaluation with the persistent gate passes.  Forward: the
// angles and |HF> of every class, then one launch of all forward runs;
// H-apply per class; reverse: one launch of all reverse runs; reduction per
// class.  The counters of both passes are cleared at the start (a fill
// kernel, not a memset node).
int enqueue_pq_phase(vqe_batch* b, int ph, bool fork, hipStream_t st) {
    auto& P = b->pq;
    if (ph == kPhaseFwd) {
        launch_pq_reset(P.cnt + 1, P.ncnt - 1, st);
        if (int rc = for_classes(b, fork, st, 0, [&](vqe_batch::Class& c, hipStream_t s) {
                launch_angles(b->sd_dev + c.k0, c.count, c.ep.M, s);
                launch_packed_hf(b->sd_dev + c.k0, c.count, c.ep.lay->size, c.ep.real, s);
            }))
            return rc;
        launch_pq(1, P.pmax, P.args[0], P.grid[0], P.lds[0], st);
    } else if (ph == kPhaseHx) {
        if (int rc = for_classes(b, fork, st, 1, [&](vqe_batch::Class& c, hipStream_t s) {
                enqueue_phase(c.ep, b->sd_dev + c.k0, c.count, kPhaseHx, true, s);
            }))
            return rc;
    } else if (ph == kPhaseAdj) {
        launch_pq(2, P.pmax, P.args[1], P.grid[1], P.lds[1], st);
    } else {
        if (int rc = for_classes(b, fork, st, 2, [&](vqe_batch::Class& c, hipStream_t s) {
                enqueue_phase(c.ep, b->sd_dev + c.k0, c.count, kPhaseReduce, true, s);
            }))
            return rc;
    }
    HIPCHK(hipGetLastError());
    return VQE_OK;
}

// After a synchronised evaluation: did a dependency wait of a persistent
// pass give up?
int check_persist(vqe_batch* b) {
    if (!b->pq.on) return VQE_OK;
    for (int i = 0; i < 2 * b->pq.nq; ++i)
        if (b->pq.err_h[i] != 0)
            return fail(VQE_EDEVICE, std::string("persistent ") + (i < b->pq.nq ? "forward" : "reverse") +
                                         " pass: a dependency wait gave up (queue " +
                                         std::to_string(i % b->pq.nq) + ")");
    return VQE_OK;
}

int enqueue_err_copy(vqe_batch* b) {
    if (b->pq.on)
        HIPCHK(hipMemcpyAsync(b->pq.err_h, b->pq.args[0].err, sizeof(int32_t) * 2 * b->pq.nq,
                              hipMemcpyDeviceToHost, b->st));
    return VQE_OK;
}

// One full evaluation of every class; classes run on forked streams, the
// heaviest first, each on the stream with the least work so far (work: the
// class's run traffic, which scales with its state size, gate count and
// states), so that the largest class does not queue behind others.
int enqueue_batch(vqe_batch* b) {
    if (b->pq.on) {
        for (int ph = kPhaseFwd; ph <= kPhaseReduce; ++ph)
            if (int rc = enqueue_pq_phase(b, ph, true, b->st)) return rc;
        return VQE_OK;
    }
    const size_t C = b->classes.size();
    const size_t ns = b->side.size();
    HIPCHK(hipEventRecord(b->events[0], b->st));
    for (size_t i = 0; i < ns; ++i) HIPCHK(hipStreamWaitEvent(b->side[i], b->events[0], 0));
    std::vector<size_t> ord(C);
    std::vector<double> w(C), load(ns, 0.0);
    for (size_t i = 0; i < C; ++i) {
        ord[i] = i;
        w[i] = double(b->classes[i].count) * (b->classes[i].ep.fwd_bytes + b->classes[i].ep.adj_bytes);
    }
    std::stable_sort(ord.begin(), ord.end(), [&](size_t a, size_t c) { return w[a] > w[c]; });
    for (size_t i : ord) {
        auto& c = b->classes[i];
        const size_t k = size_t(std::min_element(load.begin(), load.end()) - load.begin());
        load[k] += w[i];
        if (int rc = enqueue_eval(c.ep, b->sd_dev + c.k0, c.count, true, b->side[k])) return rc;
    }
    for (size_t i = 0; i < ns; ++i) {
        HIPCHK(hipEventRecord(b->events[1 + i], b->side[i]));
        HIPCHK(hipStreamWaitEvent(b->st, b->events[1 + i], 0));
    }
    return VQE_OK;
}
}  // namespace

extern "C" int vqe_batch_create(int S, const vqe_hamiltonian* const* H, const vqe_ansatz* const* A,
                                const int* ne, void* stream, vqe_batch** out) {
    if (!out || !H || !A || !ne) return fail(VQE_EINVAL, "null pointer argument");
    *out = nullptr;
    if (S < 1) return fail(VQE_ERANGE, "n_states must be >= 1");
    for (int i = 0; i < S; ++i)
        if (int rc = check_pair(H[i], A[i], ne[i]))
            return fail(rc, "state " + std::to_string(i) + ": " + vqe_last_error());
    // encoded programs evaluate in the occupation basis (resolve_encoded)
    std::vector<const vqe_hamiltonian*> Hr(H, H + S);
    std::vector<const vqe_ansatz*> Ar(A, A + S);
    for (int i = 0; i < S; ++i)
        if (int rc = resolve_encoded(Hr[i], Ar[i])) return rc;
    H = Hr.data();
    A = Ar.data();
    auto* b = new vqe_batch();
    std::unique_ptr<vqe_batch> guard(b);
    b->S = S;
    b->user = (hipStream_t)stream;
    HIPCHK(hipGetDevice(&b->dev));
    HIPCHK(hipStreamCreateWithFlags(&b->st, hipStreamNonBlocking));
    HIPCHK(hipEventCreateWithFlags(&b->user_ev, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&b->done_ev, hipEventDisableTiming));
    HIPCHK(hipStreamSynchronize(b->user));
    b->A.assign(A, A + S);
    b->poff.assign(S + 1, 0);
    b->goff.assign(S + 1, 0);
    for (int i = 0; i < S; ++i) {
        b->poff[i + 1] = b->poff[i] + A[i]->n_params;
        b->goff[i + 1] = b->goff[i] + int64_t(A[i]->gates.size());
    }
    // classes: states with identical gate programs and references
    std::vector<int> cls(S, -1), rep;
    for (int i = 0; i < S; ++i) {
        for (size_t c = 0; c < rep.size(); ++c)
            if (same_program(A[rep[c]], A[i]) && ne[rep[c]] == ne[i]) {
                cls[i] = int(c);
                break;
            }
        if (cls[i] < 0) {
            cls[i] = int(rep.size());
            rep.push_back(i);
        }
    }
    std::vector<int> order(S);
    for (int i = 0; i < S; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int c) { return cls[a] < cls[c]; });
    b->classes.resize(rep.size());
    for (size_t c = 0; c < rep.size(); ++c)
        if (int rc = make_eval_plan(A[rep[c]], ne[rep[c]], true, &b->classes[c].ep)) return rc;
    // persistent gate passes: every class on the packed layout with one common
    // block-bit count (planned again with it), on a device whose XCDs the
    // probe identified
    XccMap* xm = nullptr;
    bool persist = g_persist_mode.load() == 1;
    const int Lp = g_persist_L.load();
    for (size_t c = 0; c < rep.size() && persist; ++c) {
        const EvalPlan& ep = b->classes[c].ep;
        persist = ep.packed && ep.n >= Lp && packed_min_L(A[rep[c]], ne[rep[c]]) <= Lp;
    }
    if (persist) {
        if (int rc = xcc_map(&xm)) return rc;
        persist = xm->nq > 0;
    }
    if (persist)
        for (size_t c = 0; c < rep.size(); ++c) {
            b->classes[c].ep = EvalPlan{};
            if (int rc = make_eval_plan(A[rep[c]], ne[rep[c]], true, &b->classes[c].ep, Lp)) return rc;
            if (b->classes[c].ep.real) {   // the persistent passes move complex amplitudes
                b->classes[c].ep.real = false;
                b->classes[c].ep.fwd_bytes *= 2.0;
                b->classes[c].ep.adj_bytes *= 2.0;
            }
            persist = persist && b->classes[c].ep.packed && b->classes[c].ep.hx.L == Lp;
        }
    size_t need = 0;
    for (int i = 0; i < S; ++i)
        need += (b->classes[cls[i]].ep.ci ? 3 : 2) * sizeof(double2) * size_t(b->classes[cls[i]].ep.elems);
    if (int rc = fits_device(need)) return rc;
    if (int rc = dalloc(b, &b->theta_dev, b->poff[S])) return rc;
    if (int rc = dalloc(b, &b->e_dev, S)) return rc;
    if (int rc = dalloc(b, &b->g_dev, b->goff[S])) return rc;
    HIPCHK(hipHostMalloc(&b->theta_h, sizeof(double) * std::max<int64_t>(b->poff[S], 1)));
    HIPCHK(hipHostMalloc(&b->e_h, sizeof(double) * S));
    HIPCHK(hipHostMalloc(&b->g_h, sizeof(double) * std::max<int64_t>(b->goff[S], 1)));
    std::vector<StateDesc> sds(S);
    for (int k = 0; k < S; ++k) {
        const int i = order[k];
        auto& cl = b->classes[cls[i]];
        if (cl.count == 0) cl.k0 = k;
        ++cl.count;
        small_fit_ham(&cl.ep, H[i]);
        const EvalPlan& ep = cl.ep;
        const int n = H[i]->n;
        const int64_t M = int64_t(A[i]->gates.size());
        DevHam* dh;
        DevAnsatz* da;
        if (int rc = dev_ham(H[i], &dh)) return rc;
        if (int rc = dev_ansatz(A[i], &da)) return rc;
        StateDesc& sd = sds[k];
        std::memset(&sd, 0, sizeof(sd));
        if (ep.sector) {
            HxWork* hw = nullptr;
            if (int rc = ham_chunks(H[i], dh, ep.hx.L, &hw)) return rc;
            sd.chunks = hw->chunks;
            sd.cgroups = hw->cgroups;
            sd.csubs = hw->csubs;
            sd.nb = hw->count;
        }
        if (int rc = dalloc(b, &sd.phi, size_t(ep.elems))) return rc;
        if (int rc = dalloc(b, &sd.lam, size_t(ep.elems))) return rc;
        if (ep.ci) {
            if (int rc = dalloc(b, &sd.aux, size_t(ep.elems))) return rc;
            CiHam* ch;
            if (int rc = ci_ham(H[i], dh, &ch)) return rc;
            sd.ci_chunks = ch->chunks;
            sd.ci_groups = ch->groups;
            sd.ci_subs = ch->subs;
            sd.ci_tabs = ch->tabs;
            sd.ci_nchunks = ch->nchunks;
            sd.ci_pcls = ch->pcls;
            sd.ci_precs = ch->precs;
            sd.ci_rgroups = ch->rgroups;
            sd.ci_rsubs = ch->rsubs;
            sd.ci_ptabs = ch->ptabs;
            sd.ci_pcoef = ch->pcoef;
            sd.ci_npcls = ch->npcls;
            sd.ci_psplit = ch->psplit ? 1 : 0;
            RowMoves* rm;
            if (int rc = ci_rowmoves(H[i], ch, *ep.cspace, &rm)) return rc;
            sd.ci_rm = rm->d_rm;
            sd.ci_rm_off = rm->d_off;
            ColMoves* cm;
            if (int rc = ci_colmoves(H[i], ch, *ep.cspace, &cm)) return rc;
            sd.ci_cm = cm->d_cm;
            sd.ci_ncm = cm->ncm;
            BetaHops* bh;
            if (int rc = ci_betahops(H[i], ch, *ep.cspace, &bh)) return rc;
            sd.ci_bh = bh->d_bh;
            sd.ci_nbh = bh->nbh;
            sd.ci_hopa = ch->d_hopa;
            AlphaHops* ahp;
            if (int rc = ci_alphahops(H[i], ch, *ep.cspace, &ahp)) return rc;
            sd.ci_ah = ahp->d_ah;
            sd.ci_ah_off = ahp->d_off;
            sd.ci_ahb = ahp->d_b;
            if (ch->diag.on) {
                DiagParts* dp;
                if (int rc = ci_diag(H[i], ch, *ep.cspace, &dp)) return rc;
                sd.ci_dgr = dp->d_row;
                sd.ci_dgc = dp->d_col;
                sd.ci_dgx = ch->d_dgx;
            }
        }
        launch_fill_zero(sd.lam, uint64_t(ep.elems), b->st);
        if (int rc = dalloc(b, &sd.cs, M)) return rc;
        if (int rc = dalloc(b, &sd.part_e, ep.nblk_e)) return rc;
        if (int rc = dalloc(b, &sd.part_g, size_t(std::max<int64_t>(M, 1)) * ep.gstride))
            return rc;
        sd.gates = da->gates;
        sd.theta = b->theta_dev + b->poff[i];
        sd.groups = dh->groups;
        sd.subs = dh->subs;
        sd.tabs = dh->tabs;
        sd.out_e = b->e_dev + i;
        sd.out_g = b->g_dev + b->goff[i];
        sd.n = n;
        sd.G = int32_t(H[i]->groups.size());
        sd.nsub = int32_t(H[i]->subs.size());
        sd.ntab = int32_t(H[i]->tabs.size());
        sd.M = int32_t(M);
        sd.ne = ne[i];
        sd.ref = reference_index(A[i], ne[i]);
        sd.gstride = ep.gstride;
        b->work[0] += ep.fwd_bytes;
        b->work[2] += ep.adj_bytes;
        if (ep.real) b->work[7] += 1.0;
        b->work[1] += ep.pairs;
        b->work[3] += 2.0 * double(ep.real ? sizeof(double) : sizeof(double2)) * double(ep.elems);
    }
    HIPCHK(hipGetLastError());
    for (auto& c : b->classes) {   // launches per evaluation (one per class and step)
        b->work[4] += double(c.ep.fwd_steps);
        b->work[5] += 1.0;
        b->work[6] += double(c.ep.adj_steps);
    }
    if (int rc = dalloc(b, &b->sd_dev, S)) return rc;
    HIPCHK(hipMemcpy(b->sd_dev, sds.data(), sizeof(StateDesc) * S, hipMemcpyHostToDevice));
    HIPCHK(hipStreamSynchronize(b->st));
    if (persist) {
        if (int rc = build_persist(b, *xm)) return rc;
        b->work[4] = b->work[6] = 1.0;   // one launch per pass
    }
    // side streams of the graph: on the 512-state batch (nine classes) six
    // measured 4.39 ms per evaluation against 4.68 with four, 4.41 with eight
    // and 4.52 with one per class
    constexpr size_t kBatchStreams = 6;
    const int nside = int(std::min<size_t>(b->classes.size(), kBatchStreams));
    for (int i = 0; i < nside; ++i) {
        hipStream_t s;
        HIPCHK(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
        b->side.push_back(s);
    }
    for (int i = 0; i < 3 * (nside + 1); ++i) {   // up to three fork/join points
        hipEvent_t e;
        HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        b->events.push_back(e);
    }
    HIPCHK(hipStreamBeginCapture(b->st, hipStreamCaptureModeThreadLocal));
    const int cap_rc = enqueue_batch(b);
    hipGraph_t graph = nullptr;
    const hipError_t ce = hipStreamEndCapture(b->st, &graph);
    b->graph = graph;
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

static int batch_upload_theta(vqe_batch* b, const double* theta_all) {
    const int64_t P = b->poff[b->S];
    if (P > 0 && !theta_all) return fail(VQE_EINVAL, "null theta_all");
    if (!finite_all(theta_all, P)) return fail(VQE_EINVAL, "theta_all has a non-finite entry");
    int cur = 0;
    HIPCHK(hipGetDevice(&cur));
    if (cur != b->dev) return fail(VQE_EINVAL, "batch belongs to another device");
    // order after the caller's pending work, and do not overwrite the pinned
    // staging buffer while a previous upload could still read it
    HIPCHK(hipEventRecord(b->user_ev, b->user));
    HIPCHK(hipStreamWaitEvent(b->st, b->user_ev, 0));
    HIPCHK(hipStreamSynchronize(b->st));
    std::memcpy(b->theta_h, theta_all, sizeof(double) * P);
    HIPCHK(hipMemcpyAsync(b->theta_dev, b->theta_h, sizeof(double) * P, hipMemcpyHostToDevice,
                          b->st));
    return VQE_OK;
}

extern "C" int vqe_batch_energy_grad(vqe_batch* b, const double* theta_all, double* e_all,
                                     double* g_all) {
    if (!b || !e_all) return fail(VQE_EINVAL, "null pointer argument");
    if (int rc = batch_upload_theta(b, theta_all)) return rc;
    HIPCHK(hipGraphLaunch(b->exec, b->st));
    HIPCHK(hipMemcpyAsync(b->e_h, b->e_dev, sizeof(double) * b->S, hipMemcpyDeviceToHost, b->st));
    if (g_all)
        HIPCHK(hipMemcpyAsync(b->g_h, b->g_dev, sizeof(double) * b->goff[b->S],
                              hipMemcpyDeviceToHost, b->st));
    if (int rc = enqueue_err_copy(b)) return rc;
    HIPCHK(hipStreamSynchronize(b->st));
    if (int rc = check_persist(b)) return rc;
    std::memcpy(e_all, b->e_h, sizeof(double) * b->S);
    bool ok = finite_all(e_all, b->S);
    if (g_all) {
        for (int i = 0; i < b->S; ++i)
            accumulate_grad(b->A[i], b->g_h + b->goff[i], g_all + b->poff[i]);
        ok = ok && finite_all(g_all, b->poff[b->S]);
    }
    if (!ok) return fail(VQE_ENUMERIC, "non-finite energy or gradient");
    return VQE_OK;
}

// The parameter -> gate lists of the batch (accumulate_grad's sums, in its
// order), uploaded once.
static int batch_param_map(vqe_batch* b) {
    if (b->pg_start) return VQE_OK;
    const int64_t P = b->poff[b->S];
    std::vector<int64_t> start(size_t(P) + 1, 0), gate(size_t(std::max<int64_t>(b->goff[b->S], 1)));
    std::vector<double> coef(gate.size());
    for (int i = 0; i < b->S; ++i)
        for (const GateDesc& g : b->A[i]->gates) ++start[size_t(b->poff[i] + g.param) + 1];
    for (int64_t q = 0; q < P; ++q) start[size_t(q) + 1] += start[size_t(q)];
    std::vector<int64_t> fill(start.begin(), start.end() - 1);
    for (int i = 0; i < b->S; ++i) {
        const auto& gates = b->A[i]->gates;
        for (size_t j = 0; j < gates.size(); ++j) {
            const GateDesc& g = gates[j];
            const int64_t k = fill[size_t(b->poff[i] + g.param)]++;
            gate[size_t(k)] = b->goff[i] + int64_t(j);
            coef[size_t(k)] = (g.type == kExcitation ? 2.0 : 1.0) * g.scale;
        }
    }
    int64_t *ds, *dg;
    double* dc;
    if (int rc = dalloc(b, &ds, start.size())) return rc;
    if (int rc = dalloc(b, &dg, gate.size())) return rc;
    if (int rc = dalloc(b, &dc, coef.size())) return rc;
    HIPCHK(hipMemcpy(ds, start.data(), sizeof(int64_t) * start.size(), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(dg, gate.data(), sizeof(int64_t) * gate.size(), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(dc, coef.data(), sizeof(double) * coef.size(), hipMemcpyHostToDevice));
    b->pg_start = ds;
    b->pg_gate = dg;
    b->pg_coef = dc;
    return VQE_OK;
}

extern "C" int vqe_batch_energy_grad_device(vqe_batch* b, const double* theta_all, double* e_all,
                                            double* g_all) {
    if (!b || !e_all) return fail(VQE_EINVAL, "null pointer argument");
    const int64_t P = b->poff[b->S];
    if (P > 0 && !theta_all) return fail(VQE_EINVAL, "null theta_all");
    int cur = 0;
    HIPCHK(hipGetDevice(&cur));
    if (cur != b->dev) return fail(VQE_EINVAL, "batch belongs to another device");
    if (b->pq.on)
        return fail(VQE_EINVAL, "the device-resident evaluation is not available with persistent passes "
                                "(their wait checks need the host)");
    if (g_all)
        if (int rc = batch_param_map(b)) return rc;
    HIPCHK(hipEventRecord(b->user_ev, b->user));
    HIPCHK(hipStreamWaitEvent(b->st, b->user_ev, 0));
    if (P > 0)
        HIPCHK(hipMemcpyAsync(b->theta_dev, theta_all, sizeof(double) * P, hipMemcpyDeviceToDevice, b->st));
    HIPCHK(hipGraphLaunch(b->exec, b->st));
    HIPCHK(hipMemcpyAsync(e_all, b->e_dev, sizeof(double) * b->S, hipMemcpyDeviceToDevice, b->st));
    if (g_all) launch_param_grad(b->pg_start, b->pg_gate, b->pg_coef, b->g_dev, g_all, P, b->st);
    HIPCHK(hipGetLastError());
    HIPCHK(hipEventRecord(b->done_ev, b->st));
    HIPCHK(hipStreamWaitEvent(b->user, b->done_ev, 0));
    return VQE_OK;
}

extern "C" int vqe_batch_profile(vqe_batch* b, const double* theta_all, int reps, double* ms) {
    if (!b || !ms) return fail(VQE_EINVAL, "null pointer argument");
    if (reps < 1) return fail(VQE_ERANGE, "reps must be >= 1");
    if (int rc = batch_upload_theta(b, theta_all)) return rc;
    hipEvent_t ev[5];
    for (auto& e : ev) HIPCHK(hipEventCreate(&e));
    double acc[4] = {0, 0, 0, 0};
    int rc = VQE_OK;
    for (int r = 0; r < reps && rc == VQE_OK; ++r) {
        (void)hipEventRecord(ev[0], b->st);
        for (int ph = kPhaseFwd; ph <= kPhaseReduce; ++ph) {
            if (b->pq.on) {
                if ((rc = enqueue_pq_phase(b, ph, false, b->st)) != VQE_OK) break;
            } else {
                for (auto& c : b->classes) enqueue_phase(c.ep, b->sd_dev + c.k0, c.count, ph, true, b->st);
            }
            (void)hipEventRecord(ev[ph + 1], b->st);
        }
        if (rc == VQE_OK) rc = enqueue_err_copy(b);
        if (rc != VQE_OK) break;
        hipError_t e = hipEventSynchronize(ev[4]);
        if (e == hipSuccess) e = hipGetLastError();
        if (e != hipSuccess) {
            rc = fail(VQE_EDEVICE, std::string("profile: ") + hipGetErrorString(e));
            break;
        }
        (void)hipStreamSynchronize(b->st);
        if ((rc = check_persist(b)) != VQE_OK) break;
        for (int ph = 0; ph < 4; ++ph) {
            float t = 0.f;
            (void)hipEventElapsedTime(&t, ev[ph], ev[ph + 1]);
            acc[ph] += t;
        }
    }
    for (auto& e : ev) (void)hipEventDestroy(e);
    if (rc) return rc;
    for (int ph = 0; ph < 4; ++ph) ms[ph] = acc[ph] / reps;
    return VQE_OK;
}

extern "C" int vqe_batch_work(const vqe_batch* b, double* work) {
    if (!b || !work) return fail(VQE_EINVAL, "null pointer argument");
    std::copy(b->work, b->work + 8, work);
    return VQE_OK;
}

extern "C" int vqe_set_tuning(int n_qubits, int batched, int64_t fwd_lds_bytes,
                              int64_t adj_lds_bytes, int hx_tile_bits) {
    if (n_qubits < 1 || n_qubits > 32) return fail(VQE_ERANGE, "n_qubits must be in [1, 32]");
    std::lock_guard<std::mutex> lk(g_tune_mu);
    const auto key = std::make_pair(n_qubits, batched ? 1 : 0);
    if (fwd_lds_bytes <= 0 && adj_lds_bytes <= 0 && hx_tile_bits <= 0) {
        g_tune.erase(key);   // back to the built-in heuristic
        return VQE_OK;
    }
    if (fwd_lds_bytes < 4096 || fwd_lds_bytes > (160 << 10) || adj_lds_bytes < 4096 ||
        adj_lds_bytes > (160 << 10))
        return fail(VQE_ERANGE, "LDS budgets must be in [4 KiB, 160 KiB]");
    if (hx_tile_bits < 2 || hx_tile_bits > kHxMaxL)
        return fail(VQE_ERANGE, "hx_tile_bits must be in [2, 14]");
    g_tune[key] = Tuning{fwd_lds_bytes, adj_lds_bytes, hx_tile_bits};
    return VQE_OK;
}

extern "C" void vqe_batch_free(vqe_batch* b) { delete b; }

extern "C" int vqe_set_run_threads(int n_qubits, int batched, int fwd_threads, int adj_threads) {
    if (n_qubits < 1 || n_qubits > 32) return fail(VQE_ERANGE, "n_qubits must be in [1, 32]");
    std::lock_guard<std::mutex> lk(g_tune_mu);
    const auto key = std::make_pair(n_qubits, batched ? 1 : 0);
    if (fwd_threads <= 0 && adj_threads <= 0) {
        g_threads.erase(key);
        return VQE_OK;
    }
    auto ok = [](int t) { return t == 64 || t == 256 || t == 512 || t == 1024; };
    if (!ok(fwd_threads) || !ok(adj_threads))
        return fail(VQE_ERANGE, "run threads must be 64, 256, 512 or 1024");
    g_threads[key] = {fwd_threads, adj_threads};
    return VQE_OK;
}

extern "C" int vqe_set_tile_cap(int n_qubits, int batched, int entries) {
    if (n_qubits < 1 || n_qubits > 32) return fail(VQE_ERANGE, "n_qubits must be in [1, 32]");
    if (entries != 0 && (entries < 16 || entries > kMaxTileEntries))
        return fail(VQE_ERANGE, "entries must be 0 or in [16, 8192]");
    std::lock_guard<std::mutex> lk(g_tune_mu);
    if (entries == 0)
        g_tile_cap.erase({n_qubits, batched ? 1 : 0});
    else
        g_tile_cap[{n_qubits, batched ? 1 : 0}] = entries;
    return VQE_OK;
}

extern "C" int vqe_set_persistent(int mode, int block_bits) {
    if (mode < 0 || mode > 1) return fail(VQE_ERANGE, "persistent mode must be 0 or 1");
    if (block_bits != 0 && (block_bits < 8 || block_bits > kHxMaxL))
        return fail(VQE_ERANGE, "block_bits must be 0 or in [8, 14]");
    g_persist_mode.store(mode);
    g_persist_L.store(block_bits == 0 ? 12 : block_bits);
    return VQE_OK;
}

extern "C" int vqe_batch_persistent(const vqe_batch* b, int* info) {
    if (!b || !info) return fail(VQE_EINVAL, "null pointer argument");
    const auto& P = b->pq;
    info[0] = P.on ? 1 : 0;
    info[1] = P.nq;
    info[2] = P.grid[0];
    info[3] = P.grid[1];
    info[4] = int(std::min<size_t>(P.items[0].size(), size_t(INT32_MAX)));
    info[5] = P.pmax;
    info[6] = int(P.lds[0]);
    info[7] = int(P.lds[1]);
    return VQE_OK;
}

extern "C" int vqe_batch_test_wait(vqe_batch* b, int spin_limit, int poison) {
    if (!b) return fail(VQE_EINVAL, "null batch");
    if (spin_limit < 0) return fail(VQE_ERANGE, "spin_limit must be >= 0");
    auto& P = b->pq;
    if (!P.on) return fail(VQE_EINVAL, "the batch does not use the persistent passes");
    int cur = 0;
    HIPCHK(hipGetDevice(&cur));
    if (cur != b->dev) return fail(VQE_EINVAL, "batch belongs to another device");
    HIPCHK(hipStreamSynchronize(b->st));
    const int32_t spin = spin_limit == 0 ? g_persist_spin.load() : spin_limit;
    HIPCHK(hipMemcpy(P.cnt, &spin, sizeof(int32_t), hipMemcpyHostToDevice));
    // the first forward item with a dependency: its count out of reach, or restored
    for (size_t i = 0; i < P.items[0].size(); ++i) {
        if (P.items[0][i].need <= 0) continue;
        PqItem it = P.items[0][i];
        if (poison) it.need = INT32_MAX;
        HIPCHK(hipMemcpy(const_cast<PqItem*>(P.args[0].items) + i, &it, sizeof(PqItem),
                         hipMemcpyHostToDevice));
        break;
    }
    return VQE_OK;
}

extern "C" int vqe_set_real(int on) {
    g_real_enabled.store(on ? 1 : 0);
    return VQE_OK;
}

extern "C" int vqe_set_packed(int mode) {
    if (mode < 0 || mode > 2) return fail(VQE_ERANGE, "packed mode must be 0, 1 or 2");
    g_packed_enabled.store(mode);
    return VQE_OK;
}
