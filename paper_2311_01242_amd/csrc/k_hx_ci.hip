// H-apply in string-product order (Sec. 2.1.1, Eq. 1): lambda = H phi and
// Re <phi|lambda> restricted to the reference's (N, S_z) sector.
//
// With alpha strings along rows and beta strings along columns, a group with
// flip mask x = xa (alpha part) + xb (beta part) maps row a to row a ^ xa and
// column b to column b ^ xb.  A row has an in-sector partner row iff half of
// xa is occupied in it, which is the same for every column of the row, so a
// wave (one row, beta strings across the lanes) skips such a group as a
// whole; only the beta half of the test remains per lane.  Groups come
// sorted by (xa, xb): the partner row changes only between classes of equal
// xa and is staged once per class in the wave's slice of LDS, from which the
// lanes gather column b ^ xb.  Groups of classes whose members all have
// xb = 0 read the partner in the same column straight from memory.  Group,
// subgroup and table data are read through the caches (every row of a state
// reads the same ones).
#include <type_traits>

#include "device_common.h"

namespace vqe {

// Group and subgroup descriptors are the same for every lane: they are read
// through the scalar data cache (ldc) one group ahead; the tables, gathered
// per lane, through the vector caches.
__device__ __forceinline__ uint32_t pext_mask(uint32_t v, uint32_t mask) {
    uint32_t out = 0;
    int k = 0;
    while (mask) {
        const int q = __ffs(mask) - 1;
        mask &= mask - 1;
        out |= ((v >> q) & 1u) << k++;
    }
    return out;
}

// Words of a wave's LDS slice: its staged row (nb amplitudes of vbytes
// each), then the beta-pair coefficient records of the current pair class,
// then 16 doubles for the row's part of the diagonal's alpha-beta terms.
__host__ __device__ inline int ci_row_words(int nb, int vbytes) { return (nb * vbytes + 15) / 16; }
__host__ __device__ inline int ci_wave_words(int nb, int npairs, int vbytes) {
    return ci_row_words(nb, vbytes) + npairs + (npairs * 4 + 15) / 16 + 8;   // in 16-byte units
}

// lambda += D_G(b) phi(partner) for one group over the wave's columns.
// tab: the group's table base (LDS or global); sp: its subgroups.
// V: amplitude type (double2, or double for real states).
template <int COLS, int W, bool GTAB, typename V>
__device__ __forceinline__ void ci_group(const CiGroup& G, const CiSub* sp, const double* tab,
                                         uint32_t sA, const uint32_t (&sB)[COLS],
                                         const int (&ibc)[COLS], bool col_only,
                                         const V* prow, const V* row,
                                         const int16_t* RB, V (&sig)[COLS]) {
    const uint32_t ta = pext_mask(sA, G.tba);
    const int ka = (G.meta >> 8) & 0xff;
    const uint32_t q0 = G.tbb & 31, q1 = (G.tbb >> 5) & 31, q2 = (G.tbb >> 10) & 31,
                   q3 = (G.tbb >> 15) & 31;
    V p[COLS];
    bool ok[COLS];
    if (col_only) {
#pragma unroll
        for (int c = 0; c < COLS; ++c) {
            p[c] = ldgv(prow + ibc[c]);
            ok[c] = true;
        }
    } else {   // all loads first, then the selects
        int rp[COLS];
#pragma unroll
        for (int c = 0; c < COLS; ++c) rp[c] = RB[sB[c] ^ G.xb];
#pragma unroll
        for (int c = 0; c < COLS; ++c) {
            ok[c] = rp[c] >= 0;
            p[c] = row[ok[c] ? rp[c] : 0];
        }
    }
    uint32_t tix[COLS];
#pragma unroll
    for (int c = 0; c < COLS; ++c) {
        // beta table pattern (bit 31 of a beta string is 0)
        const uint32_t tb = __builtin_amdgcn_ubfe(sB[c], q0, 1) |
                            (__builtin_amdgcn_ubfe(sB[c], q1, 1) << 1) |
                            (__builtin_amdgcn_ubfe(sB[c], q2, 1) << 2) |
                            (__builtin_amdgcn_ubfe(sB[c], q3, 1) << 3);
        tix[c] = ta | (tb << ka);
    }
    double d[COLS];
    if ((G.meta >> 17) & 1) {   // linear group: sums over the occupied orbitals with tables
        const int nt = G.pad[0] & 0xff, oa = G.pad[0] >> 8;
        const uint32_t par = uint32_t(__popc(sA & G.wa));
        const uint32_t occa = sA & uint32_t(G.s0);   // the same for every lane
#pragma unroll
        for (int c = 0; c < COLS; ++c) {
            double acc = GTAB ? ldg64(tab + G.tab + tix[c]) : tab[G.tab + tix[c]];
            for (uint32_t m = occa; m; m &= m - 1) {
                const int o = G.tab + (1 + __ffs(m) - 1) * nt + int(tix[c]);
                acc += GTAB ? ldg64(tab + o) : tab[o];
            }
            for (uint32_t m = sB[c] & uint32_t(G.s1); m; m &= m - 1) {
                const int o = G.tab + (oa + __ffs(m)) * nt + int(tix[c]);
                acc += GTAB ? ldg64(tab + o) : tab[o];
            }
            const uint32_t flip = (uint32_t(__popc(sB[c] & G.wb)) + par) << 31;
            d[c] = __hiloint2double(__double2hiint(acc) ^ int(flip), __double2loint(acc));
        }
    } else {   // the first subgroup comes with the group record
        const uint32_t par = uint32_t(__popc(sA & G.wa));
#pragma unroll
        for (int c = 0; c < COLS; ++c) {
            const double t = GTAB ? ldg64(tab + G.tab + tix[c]) : tab[G.tab + tix[c]];
            const uint32_t flip = (uint32_t(__popc(sB[c] & G.wb)) + par) << 31;
            d[c] = __hiloint2double(__double2hiint(t) ^ int(flip), __double2loint(t));
        }
    }
    for (int si = G.s0 + 1; !((G.meta >> 17) & 1) && si < G.s1; ++si) {
        const CiSub S = ldc(sp + si);
        const uint32_t par = uint32_t(__popc(sA & S.wa));
#pragma unroll
        for (int c = 0; c < COLS; ++c) {
            const double t = GTAB ? ldg64(tab + S.tab + tix[c]) : tab[S.tab + tix[c]];
            const uint32_t flip = (uint32_t(__popc(sB[c] & S.wb)) + par) << 31;
            d[c] += __hiloint2double(__double2hiint(t) ^ int(flip), __double2loint(t));
        }
    }
#pragma unroll
    for (int c = 0; c < COLS; ++c) {
        const double dd = ok[c] ? d[c] : 0.0;
        axpy(sig[c], dd, p[c]);
    }
}

// The element of an LDS array at a byte offset.
template <typename T, typename B>
__device__ __forceinline__ T lds_at(const B* base, uint32_t byte_off) {
    return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + byte_off);
}

__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// R rows per workgroup, W waves per row (R = 1 when W > 1), COLS beta
// strings per lane: lane l of the row's wave w holds columns
// (64 w + l) + 64 W c.  The waves of a row share its LDS slice.
//
// xs > 0 (a batch of xs >= 8 states): the grid is one-dimensional and
// workgroup id b (dispatched to XCD b mod 8) takes a row block of state
// 8 q + (b mod 8), q = (b / 8) / nrb: all rows of a state run on one XCD,
// whose L2 then serves the partner rows every pair class and chunk reads
// again.  Workgroups past the last state exit at once.
template <int COLS, int R, int W, typename V>
__global__ void __launch_bounds__(R * W * 64) k_hx_ci(const StateDesc* __restrict__ sd, CiArgs ci,
                                                      int xs, int nrb) {
    static_assert(R == 1 || W == 1, "several rows of one wave each, or one row of several waves");
    constexpr int kT = R * W * 64;
    extern __shared__ double2 lds_ci[];
    __shared__ double ered[W];
    int rblk = blockIdx.x, sidx = blockIdx.y;
    if (xs > 0) {
        const int slot = int(blockIdx.x >> 3), q = slot / nrb;
        rblk = slot - q * nrb;
        sidx = 8 * q + int(blockIdx.x & 7);
        if (sidx >= xs) return;   // the whole workgroup, before any barrier
    }
    const int nrank = 1 << ci.ob;
    int16_t* RB = reinterpret_cast<int16_t*>(lds_ci);
    for (int i = threadIdx.x; i < nrank; i += kT) RB[i] = ci.rank_b[i];
    __syncthreads();   // every wave reads the whole table
    const StateDesc& s = sd[sidx];
    const int split = blockIdx.z, nsplit = ci.nsplit;
    const int wave = __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6)), lane = threadIdx.x & 63;
    const int rslot = wave / W, wr = wave % W;   // row slot in the block, wave within the row
    const int rt = wr * 64 + lane;               // thread within the row
    const int ia = rblk * R + rslot;
    const bool row_live = ia < ci.na_str;   // waves past the last row only help with staging
    const int NB = ci.nb_str;
    double2* slice = lds_ci + ((nrank * 2 + 15) >> 4) + size_t(rslot) * ci_wave_words(NB, ci.npairs, sizeof(V));
    V* row = reinterpret_cast<V*>(slice);
    double2* wc = slice + ci_row_words(NB, sizeof(V));        // pair coefficients (tb = 1, tb = 2)
    uint32_t* ww = reinterpret_cast<uint32_t*>(wc + ci.npairs);   // pair beta sign masks
    const V* __restrict__ phi = reinterpret_cast<const V*>(s.lam);   // phi in string-product order
    const uint32_t sA = ldc(ci.sa + (row_live ? ia : 0));
    uint32_t sB[COLS];
    int ibc[COLS];
    V sig[COLS];   // this lane's part of lambda
#pragma unroll
    for (int c = 0; c < COLS; ++c) {
        const int ib = rt + 64 * W * c;
        ibc[c] = ib < NB ? ib : 0;   // a column past the end repeats column 0, unwritten
        sB[c] = ci.sb[ibc[c]];
        sig[c] = vzero<V>();
    }
    auto row_sync = [&]() {   // the row's LDS slice is shared by its W waves
        if (W == 1)
            wave_lds_sync();
        else
            __syncthreads();
    };
    auto stage_row = [&](const V* prow) {
        V v[COLS];
#pragma unroll
        for (int c = 0; c < COLS; ++c) v[c] = ldgv(prow + ibc[c]);
        if (W == 1) __builtin_amdgcn_wave_barrier();   // reads of the previous row are done
        else __syncthreads();
#pragma unroll
        for (int c = 0; c < COLS; ++c) row[ibc[c]] = v[c];   // a repeated column 0 rewrites its own value
        row_sync();
    };
    // ---- beta-pair classes
    for (int pc = split; row_live && pc < s.ci_npcls; pc += nsplit) {
        const CiPairClass P = ldc(s.ci_pcls + pc);
        if (__popc(sA & P.xa) != P.half) continue;   // no in-sector partner row
        stage_row(phi + size_t(ldc(ci.rank_a + (sA ^ P.xa))) * NB);
        const uint32_t ta = pext_mask(sA, P.xa);
        // this row's coefficients of each pair: the class's precomputed pair for
        // the row's alpha pattern, signed by the row's alpha chain parity
        const double2* pco = s.ci_pcoef + P.coef0 + size_t(ta) * ci.npairs;
        for (int j = rt; j < ci.npairs; j += 64 * W) {
            const double2 cc = ldg2(pco + j);
            const bool neg = __popc(sA & ldg32(&s.ci_precs[P.rec0 + j].wa)) & 1;
            wc[j] = neg ? make_double2(-cc.x, -cc.y) : cc;
            if (!s.ci_psplit) ww[j] = ldg32(&s.ci_precs[P.rec0 + j].wb);
        }
        row_sync();
        // per list entry (partner column | (2 pair + pattern) << 16 | chain
        // parity << 31): the pair's coefficient for the entry's pattern (one
        // double of wc) and the partner amplitude; the beta sign comes, when
        // the records allow it, from the entry and one mask per class instead
        // of a per-pair mask in LDS
        const uint32_t* lst = ci.plist;
        const double* wcd = reinterpret_cast<const double*>(wc);
        if (s.ci_psplit) {
            uint32_t cfl[COLS];
#pragma unroll
            for (int c = 0; c < COLS; ++c) cfl[c] = uint32_t(__popc(sB[c] & P.wbc)) << 31;
            // the list through a buffer resource: the lane's byte offset is fixed
            // and each step adds a scalar offset, so no per-lane address math
            // (the resource also bounds the reads to the list)
            const __amdgpu_buffer_rsrc_t lrs = __builtin_amdgcn_make_buffer_rsrc(
                const_cast<uint32_t*>(ci.plist), 0, int(uint32_t(ci.e1) * uint32_t(NB) * 4u), 0x00020000);
            uint32_t voff[COLS];
#pragma unroll
            for (int c = 0; c < COLS; ++c) voff[c] = uint32_t(ibc[c]) * 4u;
            for (int e = 0; e < ci.e1; ++e) {
#pragma unroll
                for (int c = 0; c < COLS; ++c) {
                    const uint32_t ent = __builtin_amdgcn_raw_buffer_load_b32(lrs, voff[c], e * NB * 4, 0);
                    const double t = lds_at<double>(wcd, (ent >> 16) & 0x7fffu);   // 2 pair + pattern
                    const V p = lds_at<V>(row, (ent & 0xffffu) * uint32_t(sizeof(V) / 8));
                    // chain parity (bit 31) and the class mask over the column; the
                    // class mask's bit at the pair's occupied orbital, which cfl
                    // counted and the record leaves out, is in the coefficient
                    const uint32_t flip = (ent & 0x80000000u) ^ cfl[c];
                    const double coef = __hiloint2double(__double2hiint(t) ^ int(flip), __double2loint(t));
                    axpy(sig[c], coef, p);
                }
            }
        } else {
            for (int e = 0; e < ci.e1; ++e, lst += NB) {
#pragma unroll
                for (int c = 0; c < COLS; ++c) {
                    const uint32_t ent = ldg32(lst + ibc[c]);
                    const int pid = (ent >> 20) & 0x7ff;
                    const double t = lds_at<double>(wcd, (ent >> 16) & 0x7fffu);
                    const V p = lds_at<V>(row, (ent & 0xffffu) * uint32_t(sizeof(V) / 8));
                    const uint32_t flip = uint32_t(__popc(sB[c] & ww[pid])) << 31;
                    const double coef = __hiloint2double(__double2hiint(t) ^ int(flip), __double2loint(t));
                    axpy(sig[c], coef, p);
                }
            }
        }
        for (int g = P.rest0; g < P.rest1; ++g) {   // the class's other groups
            const CiGroup G = ldc(s.ci_rgroups + g);
            ci_group<COLS, W, true, V>(G, s.ci_rsubs, s.ci_ptabs, sA, sB, ibc, false, nullptr, row, RB, sig);
        }
    }
    // ---- row moves: the row's own list, partners read in place
    if (row_live) {
        constexpr int kU = COLS <= 2 ? 4 : 2;   // moves in flight per pass
        const int m1 = ldc(s.ci_rm_off + ia + 1);
        int m = ldc(s.ci_rm_off + ia) + split;
        for (; m + (kU - 1) * nsplit < m1; m += kU * nsplit) {
            CiRowMove e[kU];
#pragma unroll
            for (int u = 0; u < kU; ++u) e[u] = ldc(s.ci_rm + m + u * nsplit);
            V p[kU][COLS];
#pragma unroll
            for (int u = 0; u < kU; ++u)
#pragma unroll
                for (int c = 0; c < COLS; ++c) p[u][c] = ldgv(phi + size_t(e[u].partner) * NB + ibc[c]);
#pragma unroll
            for (int u = 0; u < kU; ++u)
#pragma unroll
                for (int c = 0; c < COLS; ++c) {
                    const uint32_t flip = uint32_t(__popc(sB[c] & e[u].wb)) << 31;
                    const double cf = __hiloint2double(__double2hiint(e[u].coef) ^ int(flip),
                                                       __double2loint(e[u].coef));
                    axpy(sig[c], cf, p[u][c]);
                }
        }
        for (; m < m1; m += nsplit) {
            const CiRowMove e = ldc(s.ci_rm + m);
#pragma unroll
            for (int c = 0; c < COLS; ++c) {
                const V pv = ldgv(phi + size_t(e.partner) * NB + ibc[c]);
                const uint32_t flip = uint32_t(__popc(sB[c] & e.wb)) << 31;
                const double cf = __hiloint2double(__double2hiint(e.coef) ^ int(flip),
                                                   __double2loint(e.coef));
                axpy(sig[c], cf, pv);
            }
        }
    }
    // ---- alpha hops: the row's list, partners read in place, the column part
    // of each hop read per lane
    if (row_live) {
        const int h1 = ldc(s.ci_ah_off + ia + 1);
        // kH hops per pass: their records (scalar loads) and then their
        // partner and column-part loads all in flight together
        constexpr int kH = COLS <= 2 ? 4 : 2;
        int h = ldc(s.ci_ah_off + ia) + split;
        auto hops = [&](auto nh) {
            constexpr int NH = decltype(nh)::value;
            CiAlphaHop e[NH];
#pragma unroll
            for (int u = 0; u < NH; ++u) e[u] = ldc(s.ci_ah + h + u * nsplit);
            V pv[NH][COLS];
            double bv[NH][COLS];
#pragma unroll
            for (int u = 0; u < NH; ++u) {
                const V* prow = phi + size_t(e[u].w & 0xffffu) * NB;
                const double* bp = s.ci_ahb + (size_t((e[u].w >> 16) & 0xffu) * 2 + ((e[u].w >> 24) & 1u)) * NB;
#pragma unroll
                for (int c = 0; c < COLS; ++c) {
                    pv[u][c] = ldgv(prow + ibc[c]);
                    bv[u][c] = ldg64(bp + ibc[c]);
                }
            }
#pragma unroll
            for (int u = 0; u < NH; ++u) {
                const bool neg = (e[u].w >> 25) & 1u;
#pragma unroll
                for (int c = 0; c < COLS; ++c) {
                    const double v = e[u].coef + (neg ? -bv[u][c] : bv[u][c]);
                    const uint32_t flip = uint32_t(__popc(sB[c] & e[u].wb)) << 31;
                    const double cf = __hiloint2double(__double2hiint(v) ^ int(flip), __double2loint(v));
                    axpy(sig[c], cf, pv[u][c]);
                }
            }
        };
        for (; h + (kH - 1) * nsplit < h1; h += kH * nsplit) hops(std::integral_constant<int, kH>{});
        for (; h < h1; h += nsplit) hops(std::integral_constant<int, 1>{});
    }
    // ---- column moves, beta hops and the diagonal: the own row staged, each
    // lane walks its column's lists
    const bool diag = s.ci_dgx != nullptr && split == 0;
    if (row_live && (s.ci_ncm > 0 || s.ci_nbh > 0 || diag)) stage_row(phi + size_t(ia) * NB);
    if (row_live && diag) {
        // E(a, b) = R(a) + C(b) + sum over occupied alpha t, beta u of X[t][u]:
        // the row's sums over t per beta orbital u, then per lane its u
        double* dv = reinterpret_cast<double*>(wc + ci.npairs + (ci.npairs * 4 + 15) / 16);
        for (int u = rt; u < ci.ob; u += 64 * W) {
            double v = 0.0;
            for (uint32_t m = sA; m; m &= m - 1) v += ldg64(s.ci_dgx + (__ffs(m) - 1) * 16 + u);
            dv[u] = v;
        }
        row_sync();
        const double ra = ldg64(s.ci_dgr + ia);
#pragma unroll
        for (int c = 0; c < COLS; ++c) {
            double d = ra + ldg64(s.ci_dgc + ibc[c]);
            for (uint32_t m = sB[c]; m; m &= m - 1) d += dv[__ffs(m) - 1];
            axpy(sig[c], d, row[ibc[c]]);
        }
    }
    if (row_live && s.ci_nbh > 0) {
        // the row's alpha part of every hop, by beta pair: wc[j] = {pat 1, pat 2}
        for (int j = rt; j < ci.npairs; j += 64 * W) {
            double a1 = 0.0, a2 = 0.0;
            const double* ha = s.ci_hopa + size_t(j) * 32;
            for (uint32_t m = sA; m; m &= m - 1) {
                const int t = __ffs(m) - 1;
                a1 += ldg64(ha + 2 * t);
                a2 += ldg64(ha + 2 * t + 1);
            }
            wc[j] = make_double2(a1, a2);
        }
        row_sync();
        const double2* bhv = reinterpret_cast<const double2*>(s.ci_bh);
        const double* wcd = reinterpret_cast<const double*>(wc);
        // branch-free decode (the row part is read for every entry, a padding
        // entry's pair bits are 0, and zeroed by a mask), so that the records
        // of a pass are all in flight before the first is used
        auto hop = [&](const double2 q, int c) {   // q = {coef, w | wa << 32}
            const uint64_t ww2 = uint64_t(__double_as_longlong(q.y));
            const uint32_t w = uint32_t(ww2);
            const double a = wcd[2 * ((w >> 16) & 0xffu) + ((w >> 24) & 1u)];
            const int keep = -int((w >> 26) & 1u);             // all ones when the hop has a row part
            const int hi = (__double2hiint(a) ^ int((w << 6) & 0x80000000u)) & keep;   // bit 25: sign
            const double v = q.x + __hiloint2double(hi, __double2loint(a) & keep);
            const uint32_t flip = uint32_t(__popc(sA & uint32_t(ww2 >> 32))) << 31;
            const double cf = __hiloint2double(__double2hiint(v) ^ int(flip), __double2loint(v));
            axpy(sig[c], cf, row[w & 0xffffu]);
        };
        constexpr int kM = COLS <= 2 ? 4 : 2;
        int e = split;
        for (; e + (kM - 1) * nsplit < s.ci_nbh; e += kM * nsplit) {
            double2 q[kM][COLS];
#pragma unroll
            for (int u = 0; u < kM; ++u)
#pragma unroll
                for (int c = 0; c < COLS; ++c) q[u][c] = ldg2(bhv + size_t(e + u * nsplit) * NB + ibc[c]);
#pragma unroll
            for (int u = 0; u < kM; ++u)
#pragma unroll
                for (int c = 0; c < COLS; ++c) hop(q[u][c], c);
        }
        for (; e < s.ci_nbh; e += nsplit)
#pragma unroll
            for (int c = 0; c < COLS; ++c) hop(ldg2(bhv + size_t(e) * NB + ibc[c]), c);
    }
    if (row_live && s.ci_ncm > 0) {
        const double2* cmv = reinterpret_cast<const double2*>(s.ci_cm);
        auto move = [&](const double2 q, int c) {   // q = {coef, partner | wa << 32}
            const uint64_t pw = uint64_t(__double_as_longlong(q.y));
            const V pv = row[int(uint32_t(pw))];
            const uint32_t flip = uint32_t(__popc(sA & uint32_t(pw >> 32))) << 31;
            const double cf = __hiloint2double(__double2hiint(q.x) ^ int(flip), __double2loint(q.x));
            axpy(sig[c], cf, pv);
        };
        // the moves' records (per column, the same for every row) come from L2:
        // kM of them in flight per pass
        constexpr int kM = COLS <= 2 ? 4 : 2;
        int e = split;
        for (; e + (kM - 1) * nsplit < s.ci_ncm; e += kM * nsplit) {
            double2 q[kM][COLS];
#pragma unroll
            for (int u = 0; u < kM; ++u)
#pragma unroll
                for (int c = 0; c < COLS; ++c) q[u][c] = ldg2(cmv + size_t(e + u * nsplit) * NB + ibc[c]);
#pragma unroll
            for (int u = 0; u < kM; ++u)
#pragma unroll
                for (int c = 0; c < COLS; ++c) move(q[u][c], c);
        }
        for (; e < s.ci_ncm; e += nsplit)
#pragma unroll
            for (int c = 0; c < COLS; ++c) move(ldg2(cmv + size_t(e) * NB + ibc[c]), c);
    }
    // ---- generic groups, chunk by chunk (chunks split, split + nsplit, ...);
    // their tables are read from global memory (every row of the state reads
    // the same ones, so they stay in L2)
    const int nch = s.ci_nchunks;
    uint32_t cur_xa = 0xffffffffu;   // class whose partner row is staged
    bool valid = false, col_only = false;
    const V* prow = phi;
    for (int ch = split; row_live && ch < nch; ch += nsplit) {
        const CiChunk ck = ldc(s.ci_chunks + ch);
        const double* tab = s.ci_tabs + ck.t0;
        const CiGroup* gp = s.ci_groups + ck.g0;
        const CiSub* sp = s.ci_subs + ck.s0;
        const int ng = ck.g1 - ck.g0;
        CiGroup G = ldc(gp);
        for (int g = 0; g < ng; ++g) {
            const CiGroup Gn = ldc(gp + (g + 1 < ng ? g + 1 : g));   // next group, ahead
            if (G.xa != cur_xa) {   // a new class: its partner row
                cur_xa = G.xa;
                valid = __popc(sA & G.xa) == (G.meta & 0xff);
                col_only = (G.meta >> 16) & 1;
                if (valid) {
                    prow = phi + size_t(ldc(ci.rank_a + (sA ^ G.xa))) * NB;
                    if (!col_only) stage_row(prow);
                }
            }
            if (valid) ci_group<COLS, W, true, V>(G, sp, tab, sA, sB, ibc, col_only, prow, row, RB, sig);
            G = Gn;
        }
    }
    if (!row_live) return;
    double acc = 0.0;
    const V* mine = phi + size_t(ia) * NB;
    V* out = reinterpret_cast<V*>(s.aux) + size_t(split) * size_t(ci.na_str) * NB + size_t(ia) * NB;
#pragma unroll
    for (int c = 0; c < COLS; ++c) {
        const int ib = rt + 64 * W * c;
        if (ib < NB) {
            stgv(out + ib, sig[c]);
            acc += redot(ldgv(mine + ib), sig[c]);
        }
    }
    acc = wave_total(acc);
    if (W == 1) {
        if (lane == 0) s.part_e[split * ci.na_str + ia] = acc;
    } else {   // the row's wave totals in fixed order
        if (lane == 0) ered[wr] = acc;
        __syncthreads();
        if (threadIdx.x == 0) {
            double v = 0.0;
#pragma unroll
            for (int w = 0; w < W; ++w) v += ered[w];
            s.part_e[split * ci.na_str + ia] = v;
        }
    }
}

template <typename V>
__global__ void k_ci_scatter(const StateDesc* __restrict__ sd, const int32_t* __restrict__ perm,
                             int64_t size) {
    const StateDesc& s = sd[blockIdx.y];
    const V* phi = reinterpret_cast<const V*>(s.phi);
    V* lam = reinterpret_cast<V*>(s.lam);
    for (int64_t k = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; k < size;
         k += int64_t(gridDim.x) * blockDim.x)
        lam[perm[k]] = phi[k];
}

// lambda in block order: the sum of the split planes, in plane order.
template <typename V>
__global__ void k_ci_gather(const StateDesc* __restrict__ sd, const int32_t* __restrict__ perm,
                            int64_t size, int nsplit) {
    const StateDesc& s = sd[blockIdx.y];
    const V* aux = reinterpret_cast<const V*>(s.aux);
    V* lam = reinterpret_cast<V*>(s.lam);
    for (int64_t k = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; k < size;
         k += int64_t(gridDim.x) * blockDim.x) {
        const int64_t q = perm[k];
        V v = aux[q];
        for (int z = 1; z < nsplit; ++z) vadd(v, aux[size_t(z) * size + q]);
        lam[k] = v;
    }
}

void launch_ci_scatter(const StateDesc* sd, int count, const int32_t* perm, int64_t size, bool real,
                       hipStream_t st) {
    const dim3 grid(blocks_for(uint64_t(size)), count);
    if (real)
        hipLaunchKernelGGL(k_ci_scatter<double>, grid, dim3(kBlock), 0, st, sd, perm, size);
    else
        hipLaunchKernelGGL(k_ci_scatter<double2>, grid, dim3(kBlock), 0, st, sd, perm, size);
}

void launch_ci_gather(const StateDesc* sd, int count, const int32_t* perm, int64_t size,
                      int nsplit, bool real, hipStream_t st) {
    const dim3 grid(blocks_for(uint64_t(size)), count);
    if (real)
        hipLaunchKernelGGL(k_ci_gather<double>, grid, dim3(kBlock), 0, st, sd, perm, size, nsplit);
    else
        hipLaunchKernelGGL(k_ci_gather<double2>, grid, dim3(kBlock), 0, st, sd, perm, size, nsplit);
}

// Launch shape: rows of up to 256 beta strings take one wave each, as many
// rows per workgroup as fit 64 KiB of slices (at most 4: measured on the
// 512-state batch, 8 rows per workgroup were 7% slower, 2 rows 16%); longer
// rows take four waves each, one row per workgroup.  vbytes: bytes per
// amplitude (16 complex, 8 real).
struct CiShape {
    int cols, rows, waves;
};

static CiShape ci_shape(const CiArgs& ci, int vbytes) {
    CiShape sh;
    if (ci.nb_str > 256) {
        sh.waves = 4;
        sh.rows = 1;
        sh.cols = (ci.nb_str + 255) / 256;
        return sh;
    }
    sh.waves = 1;
    sh.cols = (ci.nb_str + 63) / 64;
    const size_t w = size_t(ci_wave_words(ci.nb_str, ci.npairs, vbytes)) * sizeof(double2);
    sh.rows = 4;
    while (sh.rows > 1 && size_t(sh.rows) * w > (64u << 10)) sh.rows >>= 1;
    return sh;
}

// Splits of one state's groups so that a lone state still occupies the
// chip: about 2048 waves (two per SIMD), at most 8 splits.
int ci_choose_splits(const CiArgs& ci) {
    const CiShape sh = ci_shape(ci, 16);
    const int waves = ci.na_str * sh.waves;
    return std::max(1, std::min(8, (2048 + waves - 1) / std::max(waves, 1)));
}

static size_t ci_lds(const CiArgs& ci, int vbytes) {
    const size_t rank_bytes = ((size_t(2) << ci.ob) + 15) & ~size_t(15);
    return rank_bytes +
           size_t(ci_shape(ci, vbytes).rows) * ci_wave_words(ci.nb_str, ci.npairs, vbytes) * sizeof(double2);
}

template <int COLS, int R, int W, typename V>
static void launch_crw(const StateDesc* sd, int count, const CiArgs& ci, hipStream_t st) {
    const int nrb = (ci.na_str + R - 1) / R;
    const size_t lds = ci_lds(ci, int(sizeof(V)));
    if (count >= 8 && ci.nsplit == 1) {   // XCD-grouped batch
        const dim3 grid(unsigned(8 * ((count + 7) / 8) * nrb), 1, 1);
        hipLaunchKernelGGL((k_hx_ci<COLS, R, W, V>), grid, dim3(R * W * 64), lds, st, sd, ci, count, nrb);
        return;
    }
    const dim3 grid(unsigned(nrb), count, ci.nsplit);
    hipLaunchKernelGGL((k_hx_ci<COLS, R, W, V>), grid, dim3(R * W * 64), lds, st, sd, ci, 0, nrb);
}

template <int COLS, typename V>
static void launch_c(const StateDesc* sd, int count, const CiArgs& ci, hipStream_t st) {
    switch (ci_shape(ci, int(sizeof(V))).rows) {
        case 8: launch_crw<COLS, 8, 1, V>(sd, count, ci, st); break;
        case 4: launch_crw<COLS, 4, 1, V>(sd, count, ci, st); break;
        case 2: launch_crw<COLS, 2, 1, V>(sd, count, ci, st); break;
        default: launch_crw<COLS, 1, 1, V>(sd, count, ci, st); break;
    }
}

template <typename V>
static void launch_hx_ci_t(const StateDesc* sd, int count, const CiArgs& ci, hipStream_t st) {
    const CiShape sh = ci_shape(ci, int(sizeof(V)));
    if (sh.waves > 1) {
        if (sh.cols <= 1) launch_crw<1, 1, 4, V>(sd, count, ci, st);
        else if (sh.cols <= 2) launch_crw<2, 1, 4, V>(sd, count, ci, st);
        else if (sh.cols <= 3) launch_crw<3, 1, 4, V>(sd, count, ci, st);
        else launch_crw<4, 1, 4, V>(sd, count, ci, st);
        return;
    }
    if (sh.cols <= 1) launch_c<1, V>(sd, count, ci, st);
    else if (sh.cols <= 2) launch_c<2, V>(sd, count, ci, st);
    else launch_c<4, V>(sd, count, ci, st);
}

void launch_hx_ci(const StateDesc* sd, int count, const CiArgs& ci, bool real, hipStream_t st) {
    if (real)
        launch_hx_ci_t<double>(sd, count, ci, st);
    else
        launch_hx_ci_t<double2>(sd, count, ci, st);
}

// The complex layout needs the most LDS; the real one fits wherever it does.
int ci_prepare(const CiArgs& ci) {
    const size_t lds = ci_lds(ci, 16);
    const size_t fixed = 64;
    if (ci.nb_str > 1024 || lds + fixed > (160u << 10)) return 1;
    if (lds + fixed <= (64u << 10)) return 0;
    hipError_t e = hipSuccess;
    auto set = [&](const void* f) {
        const hipError_t r = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
        if (r != hipSuccess) e = r;
    };
#define VQE_CI_SET(C, V)                                                   \
    set(reinterpret_cast<const void*>(&k_hx_ci<C, 8, 1, V>));              \
    set(reinterpret_cast<const void*>(&k_hx_ci<C, 4, 1, V>));              \
    set(reinterpret_cast<const void*>(&k_hx_ci<C, 2, 1, V>));              \
    set(reinterpret_cast<const void*>(&k_hx_ci<C, 1, 1, V>));
#define VQE_CI_SET_V(V)                                                    \
    VQE_CI_SET(1, V)                                                       \
    VQE_CI_SET(2, V)                                                       \
    VQE_CI_SET(4, V)                                                       \
    set(reinterpret_cast<const void*>(&k_hx_ci<1, 1, 4, V>));              \
    set(reinterpret_cast<const void*>(&k_hx_ci<2, 1, 4, V>));              \
    set(reinterpret_cast<const void*>(&k_hx_ci<3, 1, 4, V>));              \
    set(reinterpret_cast<const void*>(&k_hx_ci<4, 1, 4, V>));
    VQE_CI_SET_V(double2)
    VQE_CI_SET_V(double)
#undef VQE_CI_SET_V
#undef VQE_CI_SET
    return e == hipSuccess ? 0 : 1;
}

}  // namespace vqe
