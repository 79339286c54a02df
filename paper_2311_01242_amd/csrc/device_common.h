// Device-side declarations shared by the kernel translation units and the
// host glue (vqe_device.hip).  Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "internal.h"

namespace vqe {

constexpr int kBlock = 256;          // threads per block (4 wave64)
constexpr int kMaxBlocks = 2048;     // grid-stride cap for the per-gate kernels
constexpr int kHxOuts = 5;           // in-sector outputs per thread in the sector H-apply
constexpr int kHxMaxL = 14;          // largest low-bit tile of the sector H-apply
constexpr int kMaxRunGates = 128;    // gates per fused run (per-gate partials live in LDS)

// Per-state record; kernels take their state from blockIdx.y.
struct StateDesc {
    double2* phi;            // forward state (overwritten by the reverse sweep)
    double2* lam;            // lambda = H phi
    const GateDesc* gates;   // [M]
    double2* cs;             // [M] (cos, sin) of each gate's angle
    const double* theta;     // [P]
    const GroupDesc* groups; // [G]
    const SubDesc* subs;
    const double* tabs;
    const struct HxChunk* chunks;   // sector H-apply work list [nb]
    const GroupDesc* cgroups;       // chunk-local group descriptors
    const SubDesc* csubs;           // chunk-local subgroup descriptors
    double* part_e;          // energy partials
    double* part_g;          // gradient partials [M * gstride]
    double* out_e;           // [1]
    double* out_g;           // [M] raw per-gate gradient sums
    const struct CiChunk* ci_chunks;    // string-product H-apply plan (packed path)
    const struct CiGroup* ci_groups;
    const struct CiSub* ci_subs;
    const double* ci_tabs;
    const struct CiPairClass* ci_pcls;   // beta-pair classes
    const struct CiPairRec* ci_precs;
    const struct CiGroup* ci_rgroups;    // their other groups
    const struct CiSub* ci_rsubs;
    const double* ci_ptabs;              // tables of the pair classes (global offsets)
    const double2* ci_pcoef;             // per class, alpha pattern and pair: the two coefficients
    const struct CiRowMove* ci_rm;       // row moves of each alpha string
    const int32_t* ci_rm_off;            // [na_str + 1] offsets into ci_rm
    const struct CiColMove* ci_cm;       // column moves, entry-major [ci_ncm][nb_str]
    const struct CiBetaHop* ci_bh;       // beta hops, entry-major [ci_nbh][nb_str]
    const double* ci_hopa;               // their alpha tables [pair][16][2]
    const struct CiAlphaHop* ci_ah;      // alpha hops of each alpha string
    const int32_t* ci_ah_off;            // [na_str + 1] offsets into ci_ah
    const double* ci_ahb;                // their beta parts [alpha pair][2][nb_str]
    const double* ci_dgr;                // diagonal in occupation form: row part [na_str]
    const double* ci_dgc;                // column part (with the constant) [nb_str]
    const double* ci_dgx;                // alpha-beta pair coefficients [alpha][16]; null: none
    double2* aux;            // packed path: lambda in string-product order
    int32_t n, G, M, ne;
    uint32_t ref;            // basis index of the reference (full-vector layout)
    int32_t nb;              // number of H-apply chunks
    int32_t gstride;         // stride of part_g between gates
    int32_t ci_nchunks;
    int32_t ci_npcls;
    int32_t ci_ncm;          // column moves per column
    int32_t ci_nbh;          // beta hops per column
    // 1: every pair record's beta sign mask is (beta orbitals strictly between
    // the pair) ^ (its class's wbc without the pair's two orbitals); the list
    // entry carries the first part's parity for its column (bit 31)
    int32_t ci_psplit;
    int32_t nsub, ntab;      // subgroup descriptors and table entries of the Hamiltonian
};

// String-product ("CI") order of the sector: the amplitude of alpha string a
// and beta string b sits at rank(a) * NB + rank(b), ranks counted among the
// strings with the reference's alpha / beta electron counts (ascending).
// Strings are compact: bit i of an alpha string is qubit 2i, of a beta
// string qubit 2i + 1.  The H-apply in this order takes one alpha string
// (a row) per wave and the beta strings across the lanes; the groups are
// sorted into classes by the alpha part of their flip mask, so whether a
// group can pair the row with an in-sector partner row is the same for all
// lanes.
//
// A linear group (meta bit 17) has subgroups whose sign masks differ from a
// common w0 by at most one orbital t (a hop with its n_t-weighted two-body
// parts): its coefficient is sign(w0) [S(p) - 2 sum over occupied t of
// T_t(p)], S the sum of all its tables.  Then wa, wb hold w0; s0, s1 the
// compact alpha and beta orbitals t that have a table; tab the start of
// S, followed by the tables -2 T_t of alpha orbital i at tab + (1 + i) nt and
// of beta orbital i at tab + (1 + oa + i) nt (nt = pad[0] & 255 entries,
// oa = pad[0] >> 8).
struct CiGroup {
    uint32_t xa;             // compact alpha flip mask (the group's class)
    uint32_t xb;             // compact beta flip mask
    uint32_t tbb;            // compact beta table positions, 4 x 5 bits (31 = none)
    uint32_t tba;            // compact alpha table positions (mask)
    int32_t meta;            // |xa| / 2 | ka << 8 | col_only << 16 | linear << 17
    int32_t s0, s1;          // subgroup range, local to the chunk (linear: orbital masks)
    uint32_t wa, wb;         // the first subgroup (s0), repeated here (linear: w0)
    int32_t tab;
    int32_t pad[2];          // linear: pad[0] = nt | oa << 8
};

// A row move: a group that flips alpha orbitals only, with one subgroup whose
// table bits are its flip bits, pairs row a with row a ^ xa in every column
// with a coefficient fixed by the row (table entry of a's pattern, sign of a's
// chain bits) times (-1)^{|b & wb|}.  The moves valid for row a (half of xa
// occupied) are listed per row.
struct CiRowMove {
    double coef;
    int32_t partner;         // rank of the partner alpha string
    uint32_t wb;
};

// A column move: a group that flips beta orbitals only, with one subgroup
// whose table bits are its flip bits, pairs column b with column b ^ xb in
// every row with the coefficient (table entry of b's pattern, sign of b's
// chain bits) times (-1)^{|a & wa|}.  Each column lists its valid moves,
// padded to one count with zero coefficients (partner: the column itself).
struct CiColMove {
    double coef;
    int32_t partner;         // rank of the partner beta string
    uint32_t wa;
};

// A beta hop: a linear group (see CiGroup) flipping two beta orbitals p < q
// only.  Its coefficient in row a, column b is
//   (-1)^{|a & wa0|} [coef + sb A_j(a, pi)],
// coef = (-1)^{|b & wb0|} [S(pat) - 2 sum_{occupied beta t} T_t(pat)] (the
// column's part), sb = (-1)^{|b & wb0|}, and A_j(a, pi) = -2 sum_{occupied
// alpha t} T_t(pat), the row's part, from ci_hopa (pat = pi + 1: which of p,
// q is occupied in b).  w = partner | j << 16 | pi << 24 | (sb < 0) << 25 |
// live << 26 (padding entries have live = 0 and coef = 0).
struct CiBetaHop {
    double coef;
    uint32_t w;
    uint32_t wa;
};

// An alpha hop: a linear group flipping two alpha orbitals p < q only.  Row
// a lists its valid hops (one of p, q occupied); the coefficient in column b
// is (-1)^{|b & wb0|} [coef + sa B_j(b, pi)], coef = (-1)^{|a & wa0|}
// [S(pat) - 2 sum_{occupied alpha t} T_t(pat)] (the row's part), sa =
// (-1)^{|a & wa0|}, and B_j(b, pi) = -2 sum_{occupied beta u} T_u(pat) from
// ci_ahb (pat = pi + 1).  w = partner | j << 16 | pi << 24 | (sa < 0) << 25.
struct CiAlphaHop {
    double coef;
    uint32_t w;
    uint32_t wb;
};

// Table index: (alpha pattern) | (beta pattern << ka), patterns in ascending
// position order; sign (-1)^{|a & wa| + |b & wb|}.
struct CiSub {
    uint32_t wa, wb;
    int32_t tab;             // local to the chunk
    int32_t pad;
};

// The groups, sorted by (xa, xb), cut into chunks that fit the kernel's LDS
// buffers; a group with many subgroups may continue in the next chunk.
constexpr int kCiChunkGroups = 128;
constexpr int kCiChunkSubs = 256;
constexpr int kCiChunkTabs = 1024;

struct CiChunk {
    int32_t g0, g1, s0, s1, t0, t1;
    int32_t pad[2];
};

// Beta-pair classes.  The groups of a class (xa) that flip exactly two beta
// orbitals and have one subgroup are applied by walking, per column, the
// beta pairs that column can flip (one orbital occupied, one empty; the
// same count for every column) from a precomputed list, instead of testing
// every group in every lane.  Pair p of the class has record rec0 + p.
struct CiPairClass {
    uint32_t xa;
    int32_t half;
    int32_t rec0;
    int32_t rest0, rest1;    // the class's other groups (CiGroup with global subgroups)
    uint32_t wbc;            // with ci_psplit: the beta chain mask shared by the class's records
    int32_t coef0;           // its block of ci_pcoef: [alpha pattern][pair] (c1, c2)
    int32_t pad;
};

struct CiPairRec {
    int32_t tab;             // table offset (-1: the class has no group for this pair)
    uint32_t wa, wb;
    int32_t ka;              // bits 0..7: alpha table bits, entry (alpha pattern) | (beta pattern << ka);
                             // bits 8..15 and 16..23: the pair's beta orbitals p < q
};

struct CiArgs {
    const uint32_t* sa;      // alpha strings [na_str]
    const uint32_t* sb;      // beta strings [nb_str]
    const int32_t* rank_a;   // [2^oa], -1 for other popcounts
    const int16_t* rank_b;   // [2^ob], -1 for other popcounts
    // beta-pair lists, entry-major [e1][nb_str]: 8 x the partner column (bits
    // 0-15), 8 x (2 pair index + 1 if the pair's higher orbital is the
    // occupied one) (bits 16-30), the parity of the occupied orbitals between
    // the pair's two (bit 31)
    const uint32_t* plist;
    int32_t na_str, nb_str, ob;
    int32_t npairs, e1;      // beta pairs C(ob, 2); list entries per column
    // the groups are split over nsplit workgroups per row (grid z); split z
    // writes its partial lambda to aux plane z (na_str * nb_str entries each)
    int32_t nsplit;
    int32_t pad[2];
};

// A fused tile pass over consecutive excitation gates [g0, g1) that share
// their created orbitals `key` (so each pair (D, E) has key bits 0 in D and
// all 1 in E).  A tile holds, for one value of the `outer` bits, every
// amplitude with key pattern 0 or `key` and any value of the `inner` bits:
// element e < 2^m has key pattern 0 and inner bits pdep(e, inner); element
// 2^m + e has key pattern `key`.
struct RunDesc {
    int32_t g0, g1;
    uint32_t inner, key, outer;
    int32_t m;               // popcount(inner)
    int32_t contiguous;      // inner == 2^m - 1 (pdep is the identity)
    int32_t ntiles;          // 2^popcount(outer)
    int32_t kind;            // 0: excitations (tile 2^(m+1): key 0 and 1); 1: Pauli rotations (tile 2^m)
};

// One excitation gate of a run, with its masks compressed into the tile's
// inner coordinates (r-space).  Sign of pair D: csign * (-1)^{popcount(D & chain)}
// split into the outer part (uniform per tile) and the r-space part.  For a
// Pauli rotation exp(-i phi/2 P(x, z)): xr = x in r-space, pdr = z in r-space,
// chr = |x & z| mod 4 (the Y count), chain_out = z outside the tile.
struct TileGate {
    uint32_t xr, pdr, chr, chain_out;
    double csign;
};

// Tables of the sector H-apply for a low tile of L bits (alpha = even bits,
// beta = odd bits).  unA[offA[k] + i] is the i-th L_alpha-bit string of
// popcount k (ascending) spread onto the even bits; rankA[s] is the rank of
// compact string s among strings of its popcount.  Same for beta.
struct HxTables {
    int32_t L, La, Lb;
    int32_t offA[9], offB[9];        // popcount offsets (L_alpha, L_beta <= 7)
    uint16_t unA[128], unB[128];     // spread strings (L <= 14 bits)
    uint8_t rankA[128], rankB[128];
};

static_assert(sizeof(HxTables) % 4 == 0, "HxTables is copied as 32-bit words");

// Rank of a compact 7-bit string within a popcount class, or -4096 when the
// string's popcount differs: a[k][s] for alpha strings with k electrons,
// b[k][s] for beta.  Stored right after HxTables (kRankKOffset bytes in).
struct RankK {
    int16_t a[8][128];
    int16_t b[8][128];
};
constexpr size_t kRankKOffset = (sizeof(HxTables) + 255) & ~size_t(255);
constexpr int kRankMiss = -4096;

// The sector H-apply walks the groups in chunks small enough to stage in
// LDS: chunk c covers chunk-local groups [cg0, cg1) (their sub ranges are
// relative to cs0), subgroups [cs0, cs1) (table offsets relative to t0) and
// table entries [t0, t1) of the state's tables.  All groups of a chunk share
// x >> L; a group with many subgroups may continue in the next chunk.
constexpr int kChunkGroups = 128;
constexpr int kChunkSubs = 256;
constexpr int kChunkTabs = 1024;

struct HxChunk {
    int32_t cg0, cg1, cs0, cs1, t0, t1;
    uint32_t xhi;
    int32_t pad;
};

// A run on the packed sector layout: gates [g0, g1) whose created orbitals
// have the same high part khi (bits of the block index h = b >> L).  Tile o
// is the block pair (h, h | khi) with h = pdep(o, free_hi), or the single
// block h when khi = 0.  shape selects the launch shape; max_entries bounds
// the entries of one tile (LDS per vector).
// Gate j of a run pairs, in a tile whose first block has electron class
// cls = kA * (Lb + 1) + kB, the entries listed in ent[off, off + cnt) with
// {off, cnt} = info[(j - g0) * ncls + cls]: D index (bits 0-10), E index in
// the tile (bits 11-22), parity of the D string's low chain bits (bit 23).
// Padding of a gate's pair list up to its class's stride.
constexpr uint32_t kPairNone = 0xffffffffu;

constexpr int kMaxTileBlocks = 16;   // blocks of one packed tile (window of at most 4 high bits)

// A launched tile of a packed run, computed on the host: its entries, pair
// list class and high part, and where each of its blocks starts in the tile
// (off) and in the state vector (entry k of block b, off[b] <= k, is at
// k + delta[b]).  Blocks absent from the sector have the size 0.
struct TileDesc {
    int32_t nE;                       // entries (0: an empty tile)
    int32_t cls;                      // the pair lists' class
    uint32_t hbase;                   // high part of the tile's base (no window bits)
    int32_t pad;
    int32_t off[kMaxTileBlocks];      // tile offset of each block (prefix sums)
    int32_t delta[kMaxTileBlocks];    // state offset minus tile offset of each block
};
static_assert(sizeof(TileDesc) == 144, "TileDesc is read as whole words");

// State-vector index of entry k (0 <= k < nE) of a tile.
__device__ __forceinline__ int tile_index(const TileDesc& d, int nblk, int k) {
    int g = k + d.delta[0];
#pragma unroll
    for (int b = 1; b < kMaxTileBlocks; ++b)
        if (b < nblk && k >= d.off[b]) g = k + d.delta[b];
    return g;
}

// A run of consecutive gates on the packed layout.  Its window W (high-part
// bits, i.e. qubits L + bit) holds every high orbital its gates annihilate or
// create; a tile is the set of blocks whose high parts agree outside W: tile
// o has base high part pdep(o, free_hi) (free_hi = the high bits outside W),
// and its blocks are base | blk[b] for the nblk patterns blk[b] within W that
// some gate of the run pairs (blocks of other patterns stay unchanged).  A
// tile's blocks are staged one after the other (empty blocks take no
// entries); a gate's pairs come from the run's precomputed list for the
// tile's class (the alpha and beta electron counts of the base).
struct PackedRun {
    int32_t g0, g1;
    uint32_t W;                   // window (high-part bits)
    uint32_t free_hi;             // high-part bits outside the window
    int32_t ntiles, L, na, nb;
    int32_t shape, shape_adj;     // launch shapes of the forward and reverse passes
    int32_t max_entries;          // largest tile (entries per vector)
    int32_t ncls, cls_b;          // classes: a * cls_b + b, a/b the base's alpha/beta electrons
    int32_t nblk;                 // blocks per tile
    uint32_t blk[kMaxTileBlocks]; // their patterns within W
    const int2* info;        // per class: {offset, stride} of the padded lists
    const uint32_t* ent;     // gate g of class c: ent[info[c].x + g * info[c].y + i]
    // the tiles that can hold a nonzero amplitude (starting from the
    // reference, a tile stays zero until a run pairs one of its blocks with a
    // nonzero block); null when that is every tile.  Both passes launch these
    // only.  The reverse sweep may skip a tile that is not live: its blocks
    // are zero in phi before the run, so they are zero whenever an earlier
    // gate is reached, and lambda on them is never paired with a nonzero phi
    // (a tile that pairs a zero block with a nonzero one is live, and all its
    // blocks count as nonzero afterwards); its gradient partials are zero.
    // Partials are stored by position in this list (by tile without a list).
    const int32_t* live;
    int32_t nlive;
    // the launched tiles in launch order (the live list's, else every tile)
    const TileDesc* tdesc;
};

// Pair-list entry: D's index in the tile (bits 0-12), E's (bits 13-25), the
// parity of D's chain bits in the low part and in the window (bit 26).
constexpr int kEntBits = 13;
constexpr uint32_t kEntMask = (1u << kEntBits) - 1u;
constexpr int kEntParity = 2 * kEntBits;
constexpr int kMaxTileEntries = 1 << kEntBits;

// The blocks of packed tile o of a run: base high part, the global offset and
// tile offset of each block, total entries and class.  Uniform over a
// workgroup; T is the layout's block tables (in LDS), base the block offsets.
struct TileBlocks {
    uint32_t hbase;               // high part of the tile's base (no window bits)
    int nE;                       // entries of the tile
    int cls;                      // the pair lists' class
    int off[kMaxTileBlocks];      // tile offset of each block (prefix sums)
    int64_t gb[kMaxTileBlocks];   // global offset of each block
};

__device__ __forceinline__ void tile_blocks(const HxTables& T, const PackedRun& run, int o,
                                            const int32_t* __restrict__ base, TileBlocks& tb) {
    uint32_t hb = 0, bits = run.free_hi, v = uint32_t(o);
    while (bits) {   // pdep(o, free_hi)
        const uint32_t low = bits & (~bits + 1u);
        if (v & 1u) hb |= low;
        v >>= 1;
        bits &= bits - 1;
    }
    tb.hbase = hb;
    const uint32_t hbg = hb << run.L;
    const int ca = __popc(hbg & 0x55555555u), cb = __popc(hbg & 0xAAAAAAAAu);
    tb.cls = ca * run.cls_b + cb;
    int acc = 0;
#pragma unroll
    for (int b = 0; b < kMaxTileBlocks; ++b) {
        tb.off[b] = acc;
        tb.gb[b] = 0;
        if (b < run.nblk) {
            const uint32_t sg = run.blk[b] << run.L;
            const int kA = run.na - ca - __popc(sg & 0x55555555u);
            const int kB = run.nb - cb - __popc(sg & 0xAAAAAAAAu);
            if (kA >= 0 && kA <= T.La && kB >= 0 && kB <= T.Lb) {
                acc += (T.offA[kA + 1] - T.offA[kA]) * (T.offB[kB + 1] - T.offB[kB]);
                tb.gb[b] = base[hb | run.blk[b]];
            }
        }
    }
    // a tile larger than the run's planned largest cannot occur; should it,
    // it is treated as empty rather than overrun the LDS tile
    tb.nE = acc <= run.max_entries ? acc : 0;
}

// Global offset of tile entry k (0 <= k < nE).
__device__ __forceinline__ int64_t tile_global(const TileBlocks& tb, int nblk, int k) {
    int64_t g = tb.gb[0] + k;
#pragma unroll
    for (int b = 1; b < kMaxTileBlocks; ++b)
        if (b < nblk && k >= tb.off[b]) g = tb.gb[b] + (k - tb.off[b]);
    return g;
}

// One excitation of a packed run: annihilated orbitals pd and created
// orbitals klo in the low bits, chain parity split into low (chlo) and high
// (chhi, global bit positions) parts; pair sign csign (-1)^{|D & chain|}.
struct PackedGate {
    uint32_t pd, klo, chlo, chhi;
    double csign;
};

struct HxPlan {
    int32_t L;
    int32_t ntiles;          // 2^(n - L)
    int32_t na, nb;          // electrons per spin
};

// ---------------------------------------------------------------- helpers

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Wave total of v in a fixed order, returned to every lane: inclusive scans
// within each 16-lane row by DPP row shifts (VALU only, no LDS round trips),
// then the four row totals read from lanes 15, 31, 47, 63.
template <int CTRL>
__device__ __forceinline__ double dpp_from(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xf, 0xf, true);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double wave_total(double v) {
    v += dpp_from<0x111>(v);   // row_shr:1
    v += dpp_from<0x112>(v);   // row_shr:2
    v += dpp_from<0x114>(v);   // row_shr:4
    v += dpp_from<0x118>(v);   // row_shr:8
    auto lane = [&](int l) {
        return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), l),
                                __builtin_amdgcn_readlane(__double2loint(v), l));
    };
    return (lane(15) + lane(31)) + (lane(47) + lane(63));
}

// Swaps of whole 16-lane rows between two doubles (gfx950 v_permlane16_swap /
// v_permlane32_swap on both halves): swap32 exchanges lanes 32-63 of d with
// lanes 0-31 of s, swap16 rows 1 and 3 of d with rows 0 and 2 of s.
__device__ __forceinline__ void swap_rows32(double& d, double& s) {
    const auto lo = __builtin_amdgcn_permlane32_swap(uint32_t(__double2loint(d)), uint32_t(__double2loint(s)), false, false);
    const auto hi = __builtin_amdgcn_permlane32_swap(uint32_t(__double2hiint(d)), uint32_t(__double2hiint(s)), false, false);
    d = __hiloint2double(int(hi[0]), int(lo[0]));
    s = __hiloint2double(int(hi[1]), int(lo[1]));
}
__device__ __forceinline__ void swap_rows16(double& d, double& s) {
    const auto lo = __builtin_amdgcn_permlane16_swap(uint32_t(__double2loint(d)), uint32_t(__double2loint(s)), false, false);
    const auto hi = __builtin_amdgcn_permlane16_swap(uint32_t(__double2hiint(d)), uint32_t(__double2hiint(s)), false, false);
    d = __hiloint2double(int(hi[0]), int(lo[0]));
    s = __hiloint2double(int(hi[1]), int(lo[1]));
}

// Wave totals of eight values per lane at once: lane l returns the total over
// the 64 lanes of v[(l >> 3) & 7].  Three halving steps pair lane l with
// l ^ 32, l ^ 16 and l ^ 8 (row swaps, then a DPP row rotation): each lane
// keeps the sum for one half of its values.  Then the eight lanes of a group
// add by DPP mirror and quad permutations.  Every partial sum is formed once
// in a fixed order, and the last three steps give equal bits on all lanes of a
// group (a + b == b + a), so the totals are deterministic.  VALU only: no LDS
// traffic and no wait counters.
__device__ __forceinline__ double wave_totals8(const double (&v)[8], int lane) {
    double a[4], b[2];
#pragma unroll
    for (int i = 0; i < 4; ++i) {   // lanes < 32 keep v[i], lanes >= 32 v[i + 4]
        double d = v[i], s = v[i + 4];
        swap_rows32(d, s);
        a[i] = d + s;
    }
#pragma unroll
    for (int i = 0; i < 2; ++i) {   // even rows keep a[i], odd rows a[i + 2]
        double d = a[i], s = a[i + 2];
        swap_rows16(d, s);
        b[i] = d + s;
    }
    const bool h8 = lane & 8;   // lanes 8-15 of a row keep b[1]
    double c = (h8 ? b[1] : b[0]) + dpp_from<0x128>(h8 ? b[0] : b[1]);   // row_ror:8
    c += dpp_from<0x141>(c);   // row_half_mirror
    c += dpp_from<0x4e>(c);    // quad_perm [2, 3, 0, 1]
    c += dpp_from<0xb1>(c);    // quad_perm [1, 0, 3, 2]
    return c;
}

// Fixed-order block sum over kBlock threads; result valid in thread 0.
// Contains __syncthreads(): every thread of the block must call it.
__device__ __forceinline__ double block_sum(double v, double* sh4) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sh4[w] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0) {
#pragma unroll
        for (int i = 0; i < kBlock / 64; ++i) r += sh4[i];
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

// Scatter the low bits of v onto the set bits of mask (ascending).
__device__ __forceinline__ uint32_t pdep32(uint32_t v, uint32_t mask) {
    uint32_t out = 0;
    while (mask) {
        const uint32_t low = mask & (~mask + 1u);
        if (v & 1u) out |= low;
        v >>= 1;
        mask &= mask - 1;
    }
    return out;
}

// Read-only load of a descriptor that is the same for every lane, through
// the scalar data cache (constant address space: the compiler emits scalar
// loads when the address is uniform).
template <class T>
__device__ __forceinline__ T ldc(const T* p) {
    static_assert(sizeof(T) % 4 == 0, "descriptor of whole words");
    using W = const __attribute__((address_space(4))) uint32_t;
    W* w = reinterpret_cast<W*>(reinterpret_cast<uintptr_t>(p));
    T out;
    uint32_t* o = reinterpret_cast<uint32_t*>(&out);
#pragma unroll
    for (int i = 0; i < int(sizeof(T) / 4); ++i) o[i] = w[i];
    return out;
}

// Loads and stores through the global address space.  Through a generic
// pointer the compiler emits flat accesses, which also count as LDS traffic:
// a later LDS access then waits for the global access to complete.
__device__ __forceinline__ double2 ldg2(const double2* p) {
    const __attribute__((address_space(1))) double* q =
        reinterpret_cast<const __attribute__((address_space(1))) double*>(reinterpret_cast<uintptr_t>(p));
    return make_double2(q[0], q[1]);
}

__device__ __forceinline__ void stg2(double2* p, double2 v) {
    __attribute__((address_space(1))) double* q =
        reinterpret_cast<__attribute__((address_space(1))) double*>(reinterpret_cast<uintptr_t>(p));
    q[0] = v.x;
    q[1] = v.y;
}

__device__ __forceinline__ double ldg64(const double* p) {
    return *reinterpret_cast<const __attribute__((address_space(1))) double*>(reinterpret_cast<uintptr_t>(p));
}

__device__ __forceinline__ uint32_t ldg32(const uint32_t* p) {
    return *reinterpret_cast<const __attribute__((address_space(1))) uint32_t*>(reinterpret_cast<uintptr_t>(p));
}

// Streaming (non-temporal) accesses for data with no reuse in L2.
__device__ __forceinline__ double2 nt_load(const double2* p) {
    return make_double2(__builtin_nontemporal_load(&p->x), __builtin_nontemporal_load(&p->y));
}

__device__ __forceinline__ void nt_store(double2* p, double2 v) {
    __builtin_nontemporal_store(v.x, &p->x);
    __builtin_nontemporal_store(v.y, &p->y);
}

// Pair update of an excitation: D' = c D - ss E, E' = c E + ss D (ss = s * sin).
__device__ __forceinline__ void givens(double2& d, double2& e, double c, double ss) {
    const double2 pd = d, pe = e;
    d = make_double2(c * pd.x - ss * pe.x, c * pd.y - ss * pe.y);
    e = make_double2(c * pe.x + ss * pd.x, c * pe.y + ss * pd.y);
}

// Amplitudes of the packed path come in two value types: double2 (complex)
// and double.  Excitation gates are real rotations and the Hamiltonian's
// matrix is real in this library's representation (the i^#Y phase of every
// Pauli term is folded into a real coefficient), so a state prepared from a
// basis state by excitations, and H applied to it, are real: the packed path
// then stores and moves real parts only.  These overloads let one kernel
// source serve both types.
__device__ __forceinline__ double ldgv(const double* p) { return ldg64(p); }
__device__ __forceinline__ double2 ldgv(const double2* p) { return ldg2(p); }
__device__ __forceinline__ void stgv(double* p, double v) {
    *reinterpret_cast<__attribute__((address_space(1))) double*>(reinterpret_cast<uintptr_t>(p)) = v;
}
__device__ __forceinline__ void stgv(double2* p, double2 v) { stg2(p, v); }
__device__ __forceinline__ void nt_store(double* p, double v) { __builtin_nontemporal_store(v, p); }
__device__ __forceinline__ void givens(double& d, double& e, double c, double ss) {
    const double pd = d, pe = e;
    d = c * pd - ss * pe;
    e = c * pe + ss * pd;
}
// Re(conj(a) b)
__device__ __forceinline__ double redot(double a, double b) { return a * b; }
__device__ __forceinline__ double redot(double2 a, double2 b) { return a.x * b.x + a.y * b.y; }
// acc += c p (c real)
__device__ __forceinline__ void axpy(double& acc, double c, double p) { acc += c * p; }
__device__ __forceinline__ void axpy(double2& acc, double c, double2 p) {
    acc.x += c * p.x;
    acc.y += c * p.y;
}
template <typename V>
__device__ __forceinline__ V vzero();
template <>
__device__ __forceinline__ double vzero<double>() { return 0.0; }
template <>
__device__ __forceinline__ double2 vzero<double2>() { return make_double2(0.0, 0.0); }
__device__ __forceinline__ double vunit(double) { return 1.0; }
__device__ __forceinline__ double2 vunit(double2) { return make_double2(1.0, 0.0); }
__device__ __forceinline__ void vadd(double& a, double b) { a += b; }
__device__ __forceinline__ void vadd(double2& a, double2 b) {
    a.x += b.x;
    a.y += b.y;
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

// D_g(b) = sum over the group's subgroups of (-1)^{|b & w|} tab[pext(b, x)].
__device__ __forceinline__ double group_coeff(const GroupDesc& gd, const SubDesc* __restrict__ subs,
                                              const double* __restrict__ tabs, uint32_t b) {
    const uint32_t u = pext_pos(b, gd.pos);
    double d = 0.0;
    for (int si = gd.sub_begin; si < gd.sub_end; ++si) {
        const SubDesc sub = subs[si];
        const double t = tabs[sub.tab + u];
        d += (__popc(b & sub.w) & 1) ? -t : t;
    }
    return d;
}

// ---------------------------------------------------------------- launchers
// (defined next to their kernels; all asynchronous on `st`)

void launch_angles(const StateDesc* sd, int count, int M, hipStream_t st);
void launch_hf(const StateDesc* sd, int count, uint64_t N, hipStream_t st);
void launch_exc(const StateDesc* sd, int count, int j, uint64_t npairs, hipStream_t st);
void launch_pauli(const StateDesc* sd, int count, int j, uint64_t N, hipStream_t st);
void launch_adj_exc(const StateDesc* sd, int count, int j, uint64_t npairs, int nblk,
                    hipStream_t st);
void launch_adj_pauli(const StateDesc* sd, int count, int j, uint64_t N, int nblk,
                      hipStream_t st);
void launch_hx_dense(const StateDesc* sd, int count, uint64_t N, int nblk, int write_lam,
                     hipStream_t st);
void launch_reduce_e(const StateDesc* sd, int count, int nblk, hipStream_t st);
void launch_param_grad(const int64_t* start, const int64_t* gate, const double* coef, const double* raw,
                       double* g, int64_t P, hipStream_t st);
void launch_reduce_g(const StateDesc* sd, int count, int M, const int32_t* cnt, int cnt_uniform,
                     hipStream_t st);
void launch_run_fwd(const StateDesc* sd, int count, const RunDesc& run, const TileGate* tg,
                    hipStream_t st);
void launch_run_adj(const StateDesc* sd, int count, const RunDesc& run, const TileGate* tg,
                    hipStream_t st);
void launch_hx_sector(const StateDesc* sd, int count, const HxPlan& plan, const HxTables* tabs,
                      hipStream_t st);
void launch_hx_packed(const StateDesc* sd, int count, const HxPlan& plan, const HxTables* tabs,
                      const int32_t* base, hipStream_t st);
void launch_fill_zero(double2* p, uint64_t n, hipStream_t st);
// Packed block order <-> string-product order: lam[perm[k]] = phi[k], and
// lam[k] = aux[perm[k]].  real: the vectors hold doubles (real states).
void launch_ci_scatter(const StateDesc* sd, int count, const int32_t* perm, int64_t size, bool real,
                       hipStream_t st);
void launch_ci_gather(const StateDesc* sd, int count, const int32_t* perm, int64_t size,
                      int nsplit, bool real, hipStream_t st);
int ci_choose_splits(const CiArgs& ci);
// lambda (aux) = H phi (lam) in string-product order, energy partial per row.
void launch_hx_ci(const StateDesc* sd, int count, const CiArgs& ci, bool real, hipStream_t st);
int ci_prepare(const CiArgs& ci);   // 0 when the kernel can launch for these sizes
void launch_packed_hf(const StateDesc* sd, int count, int64_t size, bool real, hipStream_t st);
void launch_packed_run(const StateDesc* sd, int count, const PackedRun& run, const PackedGate* pg,
                       bool adjoint, bool real, hipStream_t st);
// Launch shape covering blocks of max_block entries with at least min_threads
// threads per tile if there is one (else any), or -1.
// Single-launch zero-angle sweep of a pool's packed runs (pool gradients):
// block b covers tile b - blk0[r] of run r = blk_run[b]; runs[r].g0 indexes
// the pool's gates.
struct PoolSweep {
    const PackedRun* runs;
    const int32_t* blk_run;
    const int32_t* blk0;
    const PackedGate* gates;
    int32_t nblk;
    int32_t shape;
    size_t lds;
};
void launch_pool_sweep(const StateDesc* sd, int count, const PoolSweep& ps, const HxTables* tabs,
                       const int32_t* base, bool real, hipStream_t st);
int packed_shape(int max_block, int min_threads);
int packed_shape_threads(int shape);
int packed_enable_lds(size_t bytes);  // 0 on success

int blocks_for(uint64_t work);

// ------------------------------------------------------ small sectors
//
// Number-conserving programs whose sector (strings of k set qubits among n)
// fits one workgroup: whole-state kernels (k_small.hip).
constexpr int kSmallMaxN = 13;          // rank table of 2^n int16 entries in LDS
constexpr int kSmallMaxSector = 2048;   // amplitudes per state

constexpr int kSmallMaxGates = 1024;
constexpr int kSmallHamLds = 96 << 10;  // largest Hamiltonian staged in LDS (bytes)

struct SmallSpace {
    const uint32_t* str;     // [nsec] the sector's strings, increasing
    const int16_t* rank;     // [2^n] rank of a string in the sector, -1 outside
    int32_t n, nsec, ref_rank, M;
    int32_t ham_lds;         // LDS bytes for the largest Hamiltonian of the launch; 0: read from memory
    int32_t vbytes;          // bytes per amplitude: 8 real, 16 complex
};

// LDS bytes of a Hamiltonian staged for the small-sector H-apply: groups,
// tables, subgroups and the subgroup -> group map, each 16-byte aligned.
__host__ __device__ inline size_t small_ham_bytes(int G, int nsub, int ntab) {
    auto r16 = [](size_t v) { return (v + 15) & ~size_t(15); };
    return 16 * size_t(G) + r16(8 * size_t(ntab)) + r16(8 * size_t(nsub)) + r16(4 * size_t(nsub));
}
size_t small_lds(const SmallSpace& sp, int phase);
int small_prepare(const SmallSpace& sp);   // 0 when the kernels can launch
void launch_small(int phase, const StateDesc* sd, int count, const SmallSpace& sp, hipStream_t st);

// ------------------------------------------------------- persistent passes
//
// One launch applies every run of every packed state of a batch (k_persist.hip).

constexpr int kPqMaxXcc = 256;   // raw XCC ids the queue map covers

// A run of a class with what its tiles need besides the run descriptor.
struct PqRun {
    PackedRun r;
    const PackedGate* pg;    // the run's gates
    const int32_t* base;     // block offsets of the class's layout
};

// Tile `tile` (position in the run's live list) of run `run` (index into the
// PqRun table) of state `state` (index into the StateDesc table); it may start
// once `need` tiles of the state are done in this pass.
struct PqItem {
    int32_t state, run, tile, need;
};

struct PqArgs {
    const StateDesc* sd;
    const PqRun* runs;
    const PqItem* items;     // the queues' items, concatenated
    const int32_t* qoff;     // [nq + 1] item range of each queue
    const int32_t* qmap;     // [kPqMaxXcc] raw XCC id -> queue (-1: none)
    int32_t* head;           // [nq] next item of each queue, 0 at launch
    int32_t* done;           // [states] finished tiles of each state, 0 at launch
    int32_t* err;            // [nq] set when a wait gave up, 0 at launch
    const HxTables* tabs;    // block tables of the common block bits
    const int32_t* ctl;      // ctl[0]: polls before a dependency wait gives up
    int32_t cap;             // tile entries the dynamic LDS holds (per vector)
    int32_t max_ng;          // longest run (gate parameters and partials in LDS)
};

int pq_pmax_for(int max_stride);
int pq_prepare(int vec, int pmax, size_t lds_bytes, int* blocks_per_cu);   // 0 on success
void launch_pq(int vec, int pmax, const PqArgs& a, int grid, size_t lds_bytes, hipStream_t st);
void launch_pq_reset(int32_t* p, int n, hipStream_t st);
void launch_xcc_probe(int32_t* out, int blocks, hipStream_t st);

}  // namespace vqe
