// Host side of the VQE library: error reporting, the Jordan-Wigner builder
// (Sec. 2.1.1, Eq. 2 and the qubit mapping that follows it), x-mask grouping,
// the UCCSD program (Sec. 2.1.2), the BFGS optimiser (Sec. 3.1) and the
// host-only C-ABI entry points.  Nothing in this file calls HIP, so every
// argument check here runs without a GPU.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <limits>
#include <unordered_map>

#include "internal.h"

namespace vqe {

static thread_local std::string g_last_error;

int fail(int code, const std::string& msg) {
    g_last_error = msg;
    return code;
}

void clear_error() { g_last_error.clear(); }

bool finite_all(const double* v, int64_t n) {
    for (int64_t i = 0; i < n; ++i)
        if (!std::isfinite(v[i])) return false;
    return true;
}

static inline int popc(uint32_t v) { return __builtin_popcount(v); }
static inline uint32_t below(int p) { return (p == 0) ? 0u : ((1u << p) - 1u); }

// ------------------------------------------------------------------ JW algebra
//
// Operators are sums of folded strings c X^x Z^z with real c.  In this form
//   a+_P = 1/2 X_P Z_{<P} (1 + Z_P),   a_P = 1/2 X_P Z_{<P} (1 - Z_P),
// (a+ = |1><0| on qubit P times the Jordan-Wigner parity of the qubits
// below), and products follow X^x1 Z^z1 X^x2 Z^z2 = (-1)^{|z1 & x2|} X^{x1^x2} Z^{z1^z2}.
struct XZ {
    uint32_t x, z;
    double c;
};

// Linear encodings of the occupation vector n into the qubit register
// b = beta n (mod 2): Jordan-Wigner (beta = 1) and Bravyi-Kitaev (qubit j
// holds the parity of orbitals j + 1 - lowbit(j + 1) .. j, the Fenwick-tree
// rows; Sec. 2.1.1 names both mappings).  Then
//   a_P = X^{c_P} Z^{s_P} (1 - Z^{r_P}) / 2,  a+_P = X^{c_P} Z^{s_P} (1 + Z^{r_P}) / 2,
// with c_P = column P of beta (the qubits that flip with n_P), r_P = row P of
// beta^{-1} (n_P as a parity of qubits) and s_P = the XOR of rows P' < P of
// beta^{-1} (the sign parity of the orbitals below P).
struct Encoding {
    uint32_t c[32], r[32], s[32];
};

static bool make_encoding(int n, int mapping, Encoding* e) {
    uint32_t beta[32], inv[32];
    for (int j = 0; j < n; ++j) {
        if (mapping == VQE_MAP_JW) {
            beta[j] = 1u << j;
        } else {
            const int lo = (j + 1) - ((j + 1) & -(j + 1));
            beta[j] = 0;
            for (int k = lo; k <= j; ++k) beta[j] |= 1u << k;
        }
        inv[j] = 1u << j;
    }
    // Gauss-Jordan over GF(2): rows of beta reduced to the identity; the same
    // row operations turn the identity into beta^{-1}
    uint32_t m[32];
    std::copy(beta, beta + n, m);
    for (int col = 0; col < n; ++col) {
        int piv = -1;
        for (int row = col; row < n; ++row)
            if ((m[row] >> col) & 1u) {
                piv = row;
                break;
            }
        if (piv < 0) return false;
        std::swap(m[piv], m[col]);
        std::swap(inv[piv], inv[col]);
        for (int row = 0; row < n; ++row)
            if (row != col && ((m[row] >> col) & 1u)) {
                m[row] ^= m[col];
                inv[row] ^= inv[col];
            }
    }
    uint32_t below = 0;
    for (int P = 0; P < n; ++P) {
        e->c[P] = 0;
        for (int j = 0; j < n; ++j)
            if ((beta[j] >> P) & 1u) e->c[P] |= 1u << j;
        e->r[P] = inv[P];
        e->s[P] = below;
        below ^= inv[P];
    }
    return true;
}

static void ladder_enc(const Encoding& E, int P, bool dagger, XZ out[2]) {
    out[0] = {E.c[P], E.s[P], 0.5};
    out[1] = {E.c[P], E.s[P] ^ E.r[P], dagger ? 0.5 : -0.5};
}

static inline XZ mul(const XZ& a, const XZ& b) {
    double s = (popc(a.z & b.x) & 1) ? -1.0 : 1.0;
    return {a.x ^ b.x, a.z ^ b.z, a.c * b.c * s};
}

struct KeyHash {
    size_t operator()(uint64_t k) const { return std::hash<uint64_t>()(k * 0x9E3779B97F4A7C15ull); }
};
using TermMap = std::unordered_map<uint64_t, double, KeyHash>;

static inline uint64_t key(uint32_t x, uint32_t z) { return (uint64_t(x) << 32) | z; }

// Builds the grouped device description from sorted terms.
static void build_groups(vqe_hamiltonian* H) {
    H->groups.clear();
    H->subs.clear();
    H->tabs.clear();
    H->diag_group = -1;
    const size_t T = H->x.size();
    size_t t0 = 0;
    while (t0 < T) {
        size_t t1 = t0;
        const uint32_t x = H->x[t0];
        while (t1 < T && H->x[t1] == x) ++t1;
        GroupDesc gd{};
        gd.x = x;
        gd.sub_begin = int32_t(H->subs.size());
        const int k = popc(x);
        if (x == 0) H->diag_group = int32_t(H->groups.size());
        if (k <= kMaxTabBits) {
            int posv[kMaxTabBits];
            int kk = 0;
            for (int q = 0; q < 32; ++q)
                if ((x >> q) & 1u) posv[kk++] = q;
            uint32_t pos = uint32_t(k);
            for (int i = 0; i < kMaxTabBits; ++i)   // unused slots name bit 31 (zero when n < 32)
                pos |= uint32_t(i < k ? posv[i] : 31) << (3 + 5 * i);
            gd.pos = pos;
            std::map<uint32_t, int32_t> sub_of;   // w -> subgroup index
            for (size_t t = t0; t < t1; ++t) {
                const uint32_t z = H->z[t];
                const uint32_t w = z & ~x, v = z & x;
                auto it = sub_of.find(w);
                if (it == sub_of.end()) {
                    SubDesc sd{w, int32_t(H->tabs.size())};
                    H->tabs.resize(H->tabs.size() + (size_t(1) << k), 0.0);
                    it = sub_of.emplace(w, int32_t(H->subs.size())).first;
                    H->subs.push_back(sd);
                }
                double* tab = &H->tabs[H->subs[it->second].tab];
                const double sx = (popc(x & z) & 1) ? -1.0 : 1.0;
                for (uint32_t u = 0; u < (1u << k); ++u) {
                    uint32_t bits = 0;  // pattern u deposited on the x positions
                    for (int i = 0; i < k; ++i)
                        if ((u >> i) & 1u) bits |= 1u << posv[i];
                    const double sv = (popc(bits & v) & 1) ? -1.0 : 1.0;
                    tab[u] += H->c[t] * sx * sv;
                }
            }
        } else {
            gd.pos = 0;
            for (int i = 0; i < kMaxTabBits; ++i) gd.pos |= 31u << (3 + 5 * i);
            for (size_t t = t0; t < t1; ++t) {
                const uint32_t z = H->z[t];
                const double sx = (popc(x & z) & 1) ? -1.0 : 1.0;
                H->subs.push_back(SubDesc{z, int32_t(H->tabs.size())});
                H->tabs.push_back(H->c[t] * sx);
            }
        }
        gd.sub_end = int32_t(H->subs.size());
        H->groups.push_back(gd);
        t0 = t1;
    }
}

static void finish_terms(vqe_hamiltonian* H, const TermMap& m, double drop) {
    std::vector<std::pair<uint64_t, double>> v;
    v.reserve(m.size());
    for (auto& kv : m)
        if (std::fabs(kv.second) > drop) v.push_back(kv);
    std::sort(v.begin(), v.end());
    H->x.resize(v.size());
    H->z.resize(v.size());
    H->c.resize(v.size());
    for (size_t i = 0; i < v.size(); ++i) {
        H->x[i] = uint32_t(v[i].first >> 32);
        H->z[i] = uint32_t(v[i].first & 0xffffffffu);
        H->c[i] = v[i].second;
    }
    build_groups(H);
}

// --------------------------------------------------------------- UCCSD program

// Sign of a ladder-operator string applied (right to left) to the bit
// pattern `state`, Jordan-Wigner ordering; ops are (orbital, +1 create / -1 annihilate).
static double string_sign(uint32_t state, const int (*ops)[2], int nops) {
    double s = 1.0;
    for (int k = nops - 1; k >= 0; --k) {
        const int p = ops[k][0];
        if (popc(state & below(p)) & 1) s = -s;
        state ^= 1u << p;
    }
    return s;
}

// Gate of exp(theta (T - T^dag)) for T given as a ladder string over the
// orbitals `occ` (annihilated) and `vir` (created).  Every spectator bit
// contributes to each operator's parity count, so s(D) factors into a
// constant (the string applied to D0 = occupied pattern alone) times
// (-1)^{popcount(D & chain)}, chain = XOR of the below-masks outside x.
static GateDesc excitation_gate(const int (*ops)[2], int nops, uint32_t occ_mask, uint32_t x,
                                int32_t param) {
    GateDesc g{};
    g.type = kExcitation;
    g.x = x;
    g.pd = occ_mask;
    uint32_t chain = 0;
    for (int k = 0; k < nops; ++k) chain ^= below(ops[k][0]);
    g.chain = chain & ~x;
    g.csign = string_sign(occ_mask, ops, nops);
    g.param = param;
    g.scale = 1.0;
    return g;
}

}  // namespace vqe

using namespace vqe;

// ============================================================== C ABI (host)

extern "C" int vqe_abi_version(void) { return VQE_ABI_VERSION; }

extern "C" const char* vqe_last_error(void) { return g_last_error.c_str(); }

// h symmetric and g 8-fold symmetric within 1e-12 (EINVAL otherwise).
static int check_integral_symmetry(int ns, const double* h, const double* g) {
    auto H1 = [&](int p, int q) { return h[p * ns + q]; };
    auto G = [&](int p, int q, int r, int s) { return g[((int64_t(p) * ns + q) * ns + r) * ns + s]; };
    const double tol = 1e-12;
    for (int p = 0; p < ns; ++p)
        for (int q = 0; q < ns; ++q)
            if (std::fabs(H1(p, q) - H1(q, p)) > tol)
                return fail(VQE_EINVAL, "h is not symmetric (h[" + std::to_string(p) + "][" +
                                            std::to_string(q) + "])");
    for (int p = 0; p < ns; ++p)
        for (int q = 0; q < ns; ++q)
            for (int r = 0; r < ns; ++r)
                for (int s = 0; s < ns; ++s) {
                    const double v = G(p, q, r, s);
                    if (std::fabs(v - G(q, p, r, s)) > tol || std::fabs(v - G(p, q, s, r)) > tol ||
                        std::fabs(v - G(r, s, p, q)) > tol)
                        return fail(VQE_EINVAL, "g lacks the 8-fold symmetry of real (pq|rs)");
                }
    return VQE_OK;
}

extern "C" int vqe_hamiltonian_from_integrals(int n, double h0, const double* h, const double* g,
                                              vqe_hamiltonian** out) {
    return vqe_hamiltonian_from_integrals_map(n, VQE_MAP_JW, h0, h, g, out);
}

extern "C" int vqe_hamiltonian_from_integrals_map(int n, int mapping, double h0, const double* h,
                                                  const double* g, vqe_hamiltonian** out) {
    if (!out || !h || !g) return fail(VQE_EINVAL, "null pointer argument");
    *out = nullptr;
    if (n < 1 || n > 32) return fail(VQE_ERANGE, "n_qubits must be in [1, 32]");
    if (mapping != VQE_MAP_JW && mapping != VQE_MAP_BK) return fail(VQE_ERANGE, "unknown mapping");
    Encoding E;
    if (!make_encoding(n, mapping, &E)) return fail(VQE_EINVAL, "singular encoding");
    if (!std::isfinite(h0)) return fail(VQE_EINVAL, "h0 is not finite");
    const int ns = (n + 1) / 2;
    const int64_t n2 = int64_t(ns) * ns, n4 = n2 * n2;
    if (!finite_all(h, n2)) return fail(VQE_EINVAL, "h has a non-finite entry");
    if (!finite_all(g, n4)) return fail(VQE_EINVAL, "g has a non-finite entry");
    auto H1 = [&](int p, int q) { return h[p * ns + q]; };
    auto G = [&](int p, int q, int r, int s) { return g[((int64_t(p) * ns + q) * ns + r) * ns + s]; };
    if (int rc = check_integral_symmetry(ns, h, g)) return rc;

    TermMap m;
    m.reserve(size_t(n) * n * n * n);
    m[key(0, 0)] += h0;
    XZ cr[32][2], an[32][2];
    for (int P = 0; P < n; ++P) {
        ladder_enc(E, P, true, cr[P]);
        ladder_enc(E, P, false, an[P]);
    }
    // one-body: sum_PQ h_pq a+_P a_Q over equal spins
    for (int P = 0; P < n; ++P)
        for (int Q = 0; Q < n; ++Q) {
            if ((P & 1) != (Q & 1)) continue;
            const double v = H1(P / 2, Q / 2);
            if (v == 0.0) continue;
            for (auto& a : cr[P])
                for (auto& b : an[Q]) {
                    XZ t = mul(a, b);
                    m[key(t.x, t.z)] += v * t.c;
                }
        }
    // two-body: 1/2 sum (pq|rs) a+_P a+_R a_S a_Q, P~Q and R~S in spin
    for (int P = 0; P < n; ++P)
        for (int R = 0; R < n; ++R) {
            if (P == R) continue;
            XZ left[4];
            int li = 0;
            for (auto& a : cr[P])
                for (auto& b : cr[R]) left[li++] = mul(a, b);
            for (int S = 0; S < n; ++S) {
                if ((S & 1) != (R & 1)) continue;
                for (int Q = 0; Q < n; ++Q) {
                    if ((Q & 1) != (P & 1) || Q == S) continue;
                    const double v = 0.5 * G(P / 2, Q / 2, R / 2, S / 2);
                    if (v == 0.0) continue;
                    for (auto& a : left)
                        for (auto& b : an[S])
                            for (auto& c : an[Q]) {
                                XZ t = mul(mul(a, b), c);
                                m[key(t.x, t.z)] += v * t.c;
                            }
                }
            }
        }
    auto* H = new (std::nothrow) vqe_hamiltonian();
    if (!H) return fail(VQE_ENOMEM, "host allocation failed");
    H->n = n;
    finish_terms(H, m, 1e-12);
    *out = H;
    return VQE_OK;
}

// Eq. 2 on the seniority-zero space (pUCCD's hard-core-boson form): qubit p
// is spatial orbital p, bit p = 1 when its pair is present.  With N_p the
// pair number and b_p the pair annihilator (Slater-Condon rules for whole
// pairs; moving a pair q -> p is the double excitation with element (pq|pq)
// and sign +1, since the orbitals below each ladder operator hold pairs):
//   H = h0 + sum_p e_p N_p + sum_{p<q} w_pq N_p N_q + sum_{p<q} v_pq (b_p^dag b_q + h.c.),
//   e_p = 2 h_pp + (pp|pp), w_pq = 2 [2 (pp|qq) - (pq|qp)], v_pq = (pq|pq);
// N_p = (1 - Z_p)/2 and b_p^dag b_q + h.c. = (X_p X_q + Y_p Y_q)/2.
extern "C" int vqe_hamiltonian_pairs_from_integrals(int n, double h0, const double* h,
                                                    const double* g, vqe_hamiltonian** out) {
    if (!out || !h || !g) return fail(VQE_EINVAL, "null pointer argument");
    *out = nullptr;
    if (n < 1 || n > 32) return fail(VQE_ERANGE, "n_orbitals must be in [1, 32]");
    if (!std::isfinite(h0)) return fail(VQE_EINVAL, "h0 is not finite");
    const int64_t n2 = int64_t(n) * n, n4 = n2 * n2;
    if (!finite_all(h, n2)) return fail(VQE_EINVAL, "h has a non-finite entry");
    if (!finite_all(g, n4)) return fail(VQE_EINVAL, "g has a non-finite entry");
    if (int rc = check_integral_symmetry(n, h, g)) return rc;
    auto H1 = [&](int p, int q) { return h[p * n + q]; };
    auto G = [&](int p, int q, int r, int s) { return g[((int64_t(p) * n + q) * n + r) * n + s]; };
    TermMap m;
    m[key(0, 0)] += h0;
    for (int p = 0; p < n; ++p) {
        const double e = 2.0 * H1(p, p) + G(p, p, p, p);
        m[key(0, 0)] += 0.5 * e;
        m[key(0, 1u << p)] -= 0.5 * e;
    }
    for (int p = 0; p < n; ++p)
        for (int q = p + 1; q < n; ++q) {
            const uint32_t bp = 1u << p, bq = 1u << q;
            const double w = 2.0 * (2.0 * G(p, p, q, q) - G(p, q, q, p));
            m[key(0, 0)] += 0.25 * w;
            m[key(0, bp)] -= 0.25 * w;
            m[key(0, bq)] -= 0.25 * w;
            m[key(0, bp | bq)] += 0.25 * w;
            const double v = G(p, q, p, q);
            m[key(bp | bq, 0)] += 0.5 * v;            // X_p X_q
            m[key(bp | bq, bp | bq)] -= 0.5 * v;      // Y_p Y_q = -X_p X_q Z_p Z_q
        }
    auto* H = new (std::nothrow) vqe_hamiltonian();
    if (!H) return fail(VQE_ENOMEM, "host allocation failed");
    H->n = n;
    finish_terms(H, m, 1e-12);
    *out = H;
    return VQE_OK;
}

extern "C" int vqe_hamiltonian_from_paulis(int n, int64_t n_terms, const uint32_t* x,
                                           const uint32_t* z, const double* coef,
                                           vqe_hamiltonian** out) {
    if (!out) return fail(VQE_EINVAL, "null output pointer");
    *out = nullptr;
    if (n < 1 || n > 32) return fail(VQE_ERANGE, "n_qubits must be in [1, 32]");
    if (n_terms < 0) return fail(VQE_ERANGE, "n_terms < 0");
    if (n_terms > 0 && (!x || !z || !coef)) return fail(VQE_EINVAL, "null pointer argument");
    const uint32_t lim = (n == 32) ? 0xffffffffu : ((1u << n) - 1u);
    TermMap m;
    for (int64_t k = 0; k < n_terms; ++k) {
        if ((x[k] & ~lim) || (z[k] & ~lim))
            return fail(VQE_ERANGE, "Pauli mask has a bit beyond n_qubits (term " + std::to_string(k) + ")");
        if (!std::isfinite(coef[k])) return fail(VQE_EINVAL, "non-finite coefficient");
        m[key(x[k], z[k])] += coef[k];
    }
    for (auto& kv : m) {
        const uint32_t xx = uint32_t(kv.first >> 32), zz = uint32_t(kv.first);
        if ((popc(xx & zz) & 1) && kv.second != 0.0)
            return fail(VQE_EINVAL, "term with an odd number of Y factors has a nonzero real folded "
                                    "coefficient: H would not be Hermitian");
    }
    auto* H = new (std::nothrow) vqe_hamiltonian();
    if (!H) return fail(VQE_ENOMEM, "host allocation failed");
    H->n = n;
    finish_terms(H, m, 0.0);
    *out = H;
    return VQE_OK;
}

extern "C" int vqe_hamiltonian_info(const vqe_hamiltonian* H, int* n_qubits, int64_t* n_terms,
                                    int64_t* n_groups) {
    if (!H) return fail(VQE_EINVAL, "null Hamiltonian");
    if (n_qubits) *n_qubits = H->n;
    if (n_terms) *n_terms = int64_t(H->x.size());
    if (n_groups) *n_groups = int64_t(H->groups.size());
    return VQE_OK;
}

extern "C" int vqe_hamiltonian_terms(const vqe_hamiltonian* H, int64_t* n_terms, uint32_t* x,
                                     uint32_t* z, double* coef) {
    if (!H || !n_terms) return fail(VQE_EINVAL, "null pointer argument");
    const int64_t cnt = int64_t(H->x.size());
    if (*n_terms < cnt) {
        *n_terms = cnt;
        return fail(VQE_ERANGE, "capacity smaller than the term count");
    }
    if (cnt > 0 && (!x || !z || !coef)) return fail(VQE_EINVAL, "null output array");
    std::memcpy(x, H->x.data(), cnt * sizeof(uint32_t));
    std::memcpy(z, H->z.data(), cnt * sizeof(uint32_t));
    std::memcpy(coef, H->c.data(), cnt * sizeof(double));
    *n_terms = cnt;
    return VQE_OK;
}

extern "C" void vqe_hamiltonian_free(vqe_hamiltonian* H) { delete H; }

extern "C" int vqe_ansatz_uccsd(int n, int ne, vqe_ansatz** out, int32_t* n_params) {
    if (!out) return fail(VQE_EINVAL, "null output pointer");
    *out = nullptr;
    if (n < 1 || n > 32) return fail(VQE_ERANGE, "n_qubits must be in [1, 32]");
    if (ne < 0 || ne > n) return fail(VQE_ERANGE, "n_electrons must be in [0, n_qubits]");
    auto* A = new (std::nothrow) vqe_ansatz();
    if (!A) return fail(VQE_ENOMEM, "host allocation failed");
    A->n = n;
    A->n_electrons = ne;
    A->sector_conserving = true;
    int32_t p = 0;
    // singles: a outer, i inner, equal spin
    for (int a = ne; a < n; ++a)
        for (int i = 0; i < ne; ++i) {
            if ((i & 1) != (a & 1)) continue;
            const int ops[2][2] = {{a, +1}, {i, -1}};
            A->gates.push_back(excitation_gate(ops, 2, 1u << i, (1u << i) | (1u << a), p++));
            A->exc.insert(A->exc.end(), {i, a, -1, -1});
        }
    // doubles: (a, b) outer, (i, j) inner, spin-conserving
    for (int a = ne; a < n; ++a)
        for (int b = a + 1; b < n; ++b)
            for (int i = 0; i < ne; ++i)
                for (int j = i + 1; j < ne; ++j) {
                    if ((i & 1) + (j & 1) != (a & 1) + (b & 1)) continue;
                    const int ops[4][2] = {{a, +1}, {b, +1}, {j, -1}, {i, -1}};
                    const uint32_t occ = (1u << i) | (1u << j);
                    A->gates.push_back(
                        excitation_gate(ops, 4, occ, occ | (1u << a) | (1u << b), p++));
                    A->exc.insert(A->exc.end(), {i, j, a, b});
                }
    A->n_params = p;
    if (n_params) *n_params = p;
    *out = A;
    return VQE_OK;
}

// pUCCD (Sec. 2.1, ansatz list) on the pair space: for occupied pairs i and
// empty orbitals a of the reference (a outer, i inner, ascending),
// exp(theta (b_a^dag b_i - b_i^dag b_a)), a Givens rotation of (D, D ^ x)
// for D with bit i set and bit a clear, T|D> = +|E> (no parity string:
// pairs are bosons).
// UCCSD with `steps` Trotter steps (Sec. 2.1, ansatz list: the depth of
// UCCSD): the UCCSD product with angles theta_j / steps, repeated steps
// times; the parameters are shared by the repetitions.
extern "C" int vqe_ansatz_uccsd_trotter(int n, int ne, int steps, vqe_ansatz** out,
                                        int32_t* n_params) {
    if (!out) return fail(VQE_EINVAL, "null output pointer");
    *out = nullptr;
    if (steps < 1 || steps > 64) return fail(VQE_ERANGE, "steps must be in [1, 64]");
    vqe_ansatz* base = nullptr;
    if (int rc = vqe_ansatz_uccsd(n, ne, &base, n_params)) return rc;
    const std::vector<GateDesc> one = base->gates;
    const std::vector<int32_t> exc = base->exc;
    base->gates.clear();
    base->exc.clear();
    for (int s = 0; s < steps; ++s) {
        for (GateDesc g : one) {
            g.scale = 1.0 / steps;
            base->gates.push_back(g);
        }
        base->exc.insert(base->exc.end(), exc.begin(), exc.end());
    }
    *out = base;
    return VQE_OK;
}

// k-UpCCGSD (Sec. 2.1, ansatz list): each layer holds every generalised
// single T = a+_q a_p (p < q, equal spin; q outer, p inner, ascending) and
// every pair double T = a+_{2q} a+_{2q+1} a_{2p+1} a_{2p} (spatial p < q,
// both spin orbitals present; q outer, p inner), U_j = exp(theta_j (T_j -
// T_j^dag)); k layers with their own angles, applied in order.
extern "C" int vqe_ansatz_kupccgsd(int n, int ne, int k, vqe_ansatz** out, int32_t* n_params) {
    if (!out) return fail(VQE_EINVAL, "null output pointer");
    *out = nullptr;
    if (n < 2 || n > 32) return fail(VQE_ERANGE, "n_qubits must be in [2, 32]");
    if (ne < 0 || ne > n) return fail(VQE_ERANGE, "n_electrons must be in [0, n_qubits]");
    if (k < 1 || k > 64) return fail(VQE_ERANGE, "k must be in [1, 64]");
    auto* A = new (std::nothrow) vqe_ansatz();
    if (!A) return fail(VQE_ENOMEM, "host allocation failed");
    A->n = n;
    A->n_electrons = ne;
    A->sector_conserving = true;
    const int npair = n / 2;   // spatial orbitals with both spin orbitals
    int32_t prm = 0;
    for (int layer = 0; layer < k; ++layer) {
        for (int q = 0; q < n; ++q)
            for (int p = 0; p < q; ++p) {
                if ((p & 1) != (q & 1)) continue;
                const int ops[2][2] = {{q, +1}, {p, -1}};
                A->gates.push_back(excitation_gate(ops, 2, 1u << p, (1u << p) | (1u << q), prm++));
                A->exc.insert(A->exc.end(), {p, q, -1, -1});
            }
        for (int q = 0; q < npair; ++q)
            for (int p = 0; p < q; ++p) {
                const int ops[4][2] = {{2 * q, +1}, {2 * q + 1, +1}, {2 * p + 1, -1}, {2 * p, -1}};
                const uint32_t occ = 3u << (2 * p);
                A->gates.push_back(excitation_gate(ops, 4, occ, occ | (3u << (2 * q)), prm++));
                A->exc.insert(A->exc.end(), {2 * p, 2 * p + 1, 2 * q, 2 * q + 1});
            }
    }
    A->n_params = prm;
    if (n_params) *n_params = prm;
    *out = A;
    return VQE_OK;
}

extern "C" int vqe_ansatz_puccd(int n, int n_pairs, vqe_ansatz** out, int32_t* n_params) {
    if (!out) return fail(VQE_EINVAL, "null output pointer");
    *out = nullptr;
    if (n < 1 || n > 32) return fail(VQE_ERANGE, "n_orbitals must be in [1, 32]");
    if (n_pairs < 0 || n_pairs > n) return fail(VQE_ERANGE, "n_pairs must be in [0, n_orbitals]");
    auto* A = new (std::nothrow) vqe_ansatz();
    if (!A) return fail(VQE_ENOMEM, "host allocation failed");
    A->n = n;
    A->n_electrons = n_pairs;
    A->sector_conserving = false;   // conserves the pair count, not alpha and beta separately
    int32_t p = 0;
    for (int a = n_pairs; a < n; ++a)
        for (int i = 0; i < n_pairs; ++i) {
            GateDesc gd{};
            gd.type = kExcitation;
            gd.x = (1u << i) | (1u << a);
            gd.pd = 1u << i;
            gd.chain = 0;
            gd.csign = 1.0;
            gd.param = p++;
            gd.scale = 1.0;
            A->gates.push_back(gd);
            A->exc.insert(A->exc.end(), {i, a, -1, -1});
        }
    A->n_params = p;
    if (n_params) *n_params = p;
    *out = A;
    return VQE_OK;
}

extern "C" int vqe_ansatz_select(const vqe_ansatz* pool, int64_t count, const int32_t* param_index,
                                 vqe_ansatz** out) {
    if (!out) return fail(VQE_EINVAL, "null output pointer");
    *out = nullptr;
    if (!pool) return fail(VQE_EINVAL, "null pool");
    if (count < 0 || count > (int64_t(1) << 30)) return fail(VQE_ERANGE, "count out of range");
    if (count > 0 && !param_index) return fail(VQE_EINVAL, "null param_index");
    for (int64_t k = 0; k < count; ++k)
        if (param_index[k] < 0 || param_index[k] >= pool->n_params)
            return fail(VQE_ERANGE, "param_index out of range of the pool");
    // gates of each pool parameter, in the pool's order
    std::vector<std::vector<size_t>> of(size_t(pool->n_params));
    for (size_t j = 0; j < pool->gates.size(); ++j) of[size_t(pool->gates[j].param)].push_back(j);
    const bool has_exc = pool->exc.size() == 4 * pool->gates.size();
    auto* A = new (std::nothrow) vqe_ansatz();
    if (!A) return fail(VQE_ENOMEM, "host allocation failed");
    A->n = pool->n;
    A->n_electrons = pool->n_electrons;
    A->sector_conserving = pool->sector_conserving;
    A->ref_bits = pool->ref_bits;
    A->n_params = int32_t(count);
    for (int64_t k = 0; k < count; ++k)
        for (size_t j : of[size_t(param_index[k])]) {
            GateDesc g = pool->gates[j];
            g.param = int32_t(k);
            A->gates.push_back(g);
            if (has_exc) A->exc.insert(A->exc.end(), pool->exc.begin() + 4 * j, pool->exc.begin() + 4 * j + 4);
        }
    *out = A;
    return VQE_OK;
}

// UCCSD under an encoding other than Jordan-Wigner: each generator
// T - T^dag, written with the encoded ladder operators, is a sum of
// commuting anti-Hermitian folded strings c X^x Z^z (odd |x & z|), i.e.
// i d P with P the Hermitian string of the same masks and
// d = c (-1)^((|x & z| + 1) / 2); exp(theta (T - T^dag)) is then the product
// of the rotations exp(-i (-2 d theta) / 2 P).  The reference is beta times
// the lowest n_electrons occupations.
extern "C" int vqe_ansatz_uccsd_map(int n, int ne, int mapping, vqe_ansatz** out,
                                    int32_t* n_params) {
    if (!out) return fail(VQE_EINVAL, "null output pointer");
    *out = nullptr;
    if (mapping == VQE_MAP_JW) return vqe_ansatz_uccsd(n, ne, out, n_params);
    if (mapping != VQE_MAP_BK) return fail(VQE_ERANGE, "unknown mapping");
    vqe_ansatz* base = nullptr;
    if (int rc = vqe_ansatz_uccsd(n, ne, &base, n_params)) return rc;
    Encoding E;
    if (!make_encoding(n, mapping, &E)) {
        vqe_ansatz_free(base);
        return fail(VQE_EINVAL, "singular encoding");
    }
    auto* A = new (std::nothrow) vqe_ansatz();
    if (!A) {
        vqe_ansatz_free(base);
        return fail(VQE_ENOMEM, "host allocation failed");
    }
    A->n = n;
    A->n_electrons = ne;
    A->n_params = base->n_params;
    A->sector_conserving = false;   // encoded basis states do not split into alpha/beta bits
    A->exc = base->exc;
    uint32_t ref = 0;
    for (int P = 0; P < ne; ++P) ref ^= E.c[P];
    A->ref_bits = int64_t(ref);
    for (int P = 0; P < n; ++P) {
        A->enc_c[P] = E.c[P];
        A->enc_r[P] = E.r[P];
    }
    const size_t M = base->exc.size() / 4;
    for (size_t k = 0; k < M; ++k) {
        const int32_t* o = &base->exc[4 * k];
        // T as a product of encoded ladder sums, rightmost operator first
        std::vector<std::pair<int, bool>> ops;   // (orbital, dagger), left to right
        if (o[2] < 0)
            ops = {{o[1], true}, {o[0], false}};
        else
            ops = {{o[2], true}, {o[3], true}, {o[1], false}, {o[0], false}};
        std::vector<XZ> t = {{0u, 0u, 1.0}};
        for (auto& op : ops) {
            XZ l[2];
            ladder_enc(E, op.first, op.second, l);
            std::vector<XZ> nt;
            for (auto& a : t)
                for (auto& b : l) nt.push_back(mul(a, b));
            t.swap(nt);
        }
        TermMap m;
        for (auto& a : t) m[key(a.x, a.z)] += a.c;
        std::vector<std::pair<uint64_t, double>> terms(m.begin(), m.end());
        std::sort(terms.begin(), terms.end());
        for (auto& kv : terms) {
            const uint32_t x = uint32_t(kv.first >> 32), z = uint32_t(kv.first);
            const int y = popc(x & z);
            if (!(y & 1)) continue;   // Hermitian part: cancels in T - T^dag
            const double g = 2.0 * kv.second;   // T - T^dag doubles the anti-Hermitian part
            if (std::fabs(g) <= 1e-14) continue;
            const double d = (((y + 1) / 2) & 1) ? -g : g;
            GateDesc gd{};
            gd.type = kPauli;
            gd.x = x;
            gd.chain = z;
            gd.param = int32_t(k);
            gd.scale = -2.0 * d;
            gd.csign = 1.0;
            A->gates.push_back(gd);
        }
    }
    A->occ = base;   // the same excitations in the occupation basis
    *out = A;
    return VQE_OK;
}

namespace vqe {

int hamiltonian_to_occupation(const vqe_hamiltonian* H, const uint32_t* enc_c, const uint32_t* enc_r,
                              vqe_hamiltonian** out) {
    const size_t T = H->x.size();
    std::vector<uint32_t> x(T), z(T);
    for (size_t t = 0; t < T; ++t) {
        uint32_t xo = 0, zo = 0;
        for (int P = 0; P < H->n; ++P) {
            xo |= uint32_t(popc(H->x[t] & enc_r[P]) & 1) << P;   // beta^-1 x
            zo |= uint32_t(popc(H->z[t] & enc_c[P]) & 1) << P;   // beta^T z
        }
        x[t] = xo;
        z[t] = zo;
    }
    return vqe_hamiltonian_from_paulis(H->n, int64_t(T), x.data(), z.data(), H->c.data(), out);
}

}  // namespace vqe

extern "C" int vqe_ansatz_reference(const vqe_ansatz* A, uint64_t* index) {
    if (!A || !index) return fail(VQE_EINVAL, "null pointer argument");
    if (A->n_electrons < 0) return fail(VQE_EINVAL, "ansatz has no reference");
    *index = A->ref_bits >= 0 ? uint64_t(A->ref_bits) : ((uint64_t(1) << A->n_electrons) - 1);
    return VQE_OK;
}

extern "C" int vqe_ansatz_from_rotations(int n, int32_t n_params, int64_t n_rot, const uint32_t* x,
                                         const uint32_t* z, const int32_t* param_index,
                                         const double* scale, vqe_ansatz** out) {
    if (!out) return fail(VQE_EINVAL, "null output pointer");
    *out = nullptr;
    if (n < 1 || n > 32) return fail(VQE_ERANGE, "n_qubits must be in [1, 32]");
    if (n_params < 0 || n_rot < 0) return fail(VQE_ERANGE, "negative size");
    if (n_rot > 0 && (!x || !z || !param_index || !scale))
        return fail(VQE_EINVAL, "null pointer argument");
    const uint32_t lim = (n == 32) ? 0xffffffffu : ((1u << n) - 1u);
    auto* A = new (std::nothrow) vqe_ansatz();
    if (!A) return fail(VQE_ENOMEM, "host allocation failed");
    A->n = n;
    A->n_params = n_params;
    for (int64_t k = 0; k < n_rot; ++k) {
        if ((x[k] & ~lim) || (z[k] & ~lim)) {
            delete A;
            return fail(VQE_ERANGE, "rotation mask has a bit beyond n_qubits");
        }
        if (param_index[k] < 0 || param_index[k] >= n_params) {
            delete A;
            return fail(VQE_ERANGE, "param_index out of range");
        }
        if (!std::isfinite(scale[k])) {
            delete A;
            return fail(VQE_EINVAL, "non-finite scale");
        }
        GateDesc g{};
        g.type = kPauli;
        g.x = x[k];
        g.chain = z[k];
        g.param = param_index[k];
        g.scale = scale[k];
        g.csign = 1.0;
        A->gates.push_back(g);
    }
    *out = A;
    return VQE_OK;
}

extern "C" int vqe_ansatz_info(const vqe_ansatz* A, int* n_qubits, int32_t* n_params,
                               int64_t* n_gates, int* n_electrons) {
    if (!A) return fail(VQE_EINVAL, "null ansatz");
    if (n_qubits) *n_qubits = A->n;
    if (n_params) *n_params = A->n_params;
    if (n_gates) *n_gates = int64_t(A->gates.size());
    if (n_electrons) *n_electrons = A->n_electrons;
    return VQE_OK;
}

extern "C" int vqe_ansatz_excitations(const vqe_ansatz* A, int64_t* n, int32_t* orbitals) {
    if (!A || !n) return fail(VQE_EINVAL, "null pointer argument");
    if (A->n_electrons < 0) return fail(VQE_EINVAL, "not an excitation ansatz");
    const int64_t cnt = int64_t(A->exc.size() / 4);
    if (*n < cnt) {
        *n = cnt;
        return fail(VQE_ERANGE, "capacity smaller than the excitation count");
    }
    if (cnt > 0 && !orbitals) return fail(VQE_EINVAL, "null output array");
    std::memcpy(orbitals, A->exc.data(), A->exc.size() * sizeof(int32_t));
    *n = cnt;
    return VQE_OK;
}

extern "C" void vqe_ansatz_free(vqe_ansatz* A) { delete A; }

// ================================================================== BFGS
namespace {

struct Objective {
    vqe_objective_fn fn;
    void* ctx;
    int n;
    int evals = 0;
    int status = VQE_OK;
    bool eval(const double* x, double* f, double* g) {
        ++evals;
        const int rc = fn(ctx, n, x, f, g);
        if (rc != 0) {
            // keep a message set by the callback's own library call, if any
            status = (rc < 0) ? rc : VQE_EINVAL;
            if (g_last_error.empty()) g_last_error = "objective callback failed";
            return false;
        }
        if (!std::isfinite(*f) || !finite_all(g, n)) {
            status = VQE_ENUMERIC;
            g_last_error = "objective returned a non-finite value";
            return false;
        }
        return true;
    }
};

inline double dot(const std::vector<double>& a, const std::vector<double>& b) {
    double s = 0.0;
    for (size_t i = 0; i < a.size(); ++i) s += a[i] * b[i];
    return s;
}

// Minimiser of the cubic through (a, fa, da) and (b, fb, db); NaN if none.
double cubic_min(double a, double fa, double da, double b, double fb, double db) {
    const double d1 = da + db - 3.0 * (fa - fb) / (a - b);
    const double disc = d1 * d1 - da * db;
    if (!(disc >= 0.0)) return std::numeric_limits<double>::quiet_NaN();
    const double d2 = std::copysign(std::sqrt(disc), b - a);
    const double den = db - da + 2.0 * d2;
    if (den == 0.0) return std::numeric_limits<double>::quiet_NaN();
    return b - (b - a) * (db + d2 - d1) / den;
}

struct LinePoint {
    double a, f, d;
    std::vector<double> x, g;
};

// Strong-Wolfe line search: bracketing phase, then zoom with safeguarded
// cubic interpolation.  Returns false if no acceptable step was found.
bool line_search(Objective& obj, const std::vector<double>& x0, double f0,
                 const std::vector<double>& g0, const std::vector<double>& p, double a_init,
                 LinePoint& out) {
    const double c1 = 1e-4, c2 = 0.9;
    const double d0 = dot(g0, p);
    // Sufficient decrease is tested with a rounding allowance on f: near a
    // minimum the predicted decrease drops below the resolution of f, and the
    // (derivative-based) curvature condition then decides.
    const double epsf = 0x1p-46 * std::max(1.0, std::fabs(f0));
    const int n = int(x0.size());
    auto eval_at = [&](double a, LinePoint& pt) -> bool {
        pt.a = a;
        pt.x.resize(n);
        pt.g.resize(n);
        for (int i = 0; i < n; ++i) pt.x[i] = x0[i] + a * p[i];
        if (!obj.eval(pt.x.data(), &pt.f, pt.g.data())) return false;
        pt.d = dot(pt.g, p);
        return true;
    };
    LinePoint prev{0.0, f0, d0, x0, g0};
    LinePoint cur;
    double a = a_init;
    auto zoom = [&](LinePoint lo, LinePoint hi) -> bool {
        for (int it = 0; it < 30; ++it) {
            double aj = cubic_min(lo.a, lo.f, lo.d, hi.a, hi.f, hi.d);
            const double lo_b = std::min(lo.a, hi.a), hi_b = std::max(lo.a, hi.a);
            const double w = hi_b - lo_b;
            if (!std::isfinite(aj) || aj < lo_b + 0.1 * w || aj > hi_b - 0.1 * w)
                aj = 0.5 * (lo.a + hi.a);
            LinePoint pj;
            if (!eval_at(aj, pj)) return false;
            if (pj.f > f0 + c1 * aj * d0 + epsf || pj.f >= lo.f + epsf) {
                hi = std::move(pj);
            } else {
                if (std::fabs(pj.d) <= -c2 * d0) {
                    out = std::move(pj);
                    return true;
                }
                if (pj.d * (hi.a - lo.a) >= 0.0) hi = lo;
                lo = std::move(pj);
            }
            if (std::fabs(hi.a - lo.a) < 1e-16 * std::max(1.0, std::fabs(lo.a))) break;
        }
        // accept the best sufficient-decrease point seen if the bracket collapsed
        if (lo.a > 0.0 && lo.f <= f0 + epsf && std::fabs(lo.d) < std::fabs(d0)) {
            out = std::move(lo);
            return true;
        }
        return false;
    };
    for (int it = 0; it < 40; ++it) {
        if (!eval_at(a, cur)) return false;
        if (cur.f > f0 + c1 * a * d0 + epsf || (it > 0 && cur.f >= prev.f + epsf))
            return zoom(prev, cur);
        if (std::fabs(cur.d) <= -c2 * d0) {
            out = std::move(cur);
            return true;
        }
        if (cur.d >= 0.0) return zoom(cur, prev);
        prev = cur;
        a *= 2.0;
    }
    return false;
}

}  // namespace

extern "C" int vqe_minimize_bfgs(int n, vqe_objective_fn fn, void* ctx, const double* x0,
                                 const vqe_options* opts, double* x_out, double* trace_out,
                                 vqe_result* res) {
    if (!fn || !opts || !x_out || !res) return fail(VQE_EINVAL, "null pointer argument");
    if (n < 1) return fail(VQE_ERANGE, "n must be >= 1");
    if (opts->max_iter < 0) return fail(VQE_ERANGE, "max_iter < 0");
    if (!(opts->gtol >= 0.0) || !(opts->ftol >= 0.0))
        return fail(VQE_EINVAL, "gtol and ftol must be >= 0");
    std::vector<double> x(n, 0.0);
    if (x0) {
        if (!finite_all(x0, n)) return fail(VQE_EINVAL, "theta0 has a non-finite entry");
        std::copy(x0, x0 + n, x.begin());
    }
    clear_error();
    const auto t_start = std::chrono::steady_clock::now();
    auto elapsed = [&]() {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
    };
    if (trace_out)
        for (int i = 0; i <= opts->max_iter; ++i) trace_out[i] = std::numeric_limits<double>::quiet_NaN();
    Objective obj{fn, ctx, n};
    std::vector<double> g(n);
    double f = 0.0;
    *res = vqe_result{std::numeric_limits<double>::quiet_NaN(), 0, 0, 0};
    auto finish = [&](int status, int converged) {
        std::copy(x.begin(), x.end(), x_out);
        res->energy = f;
        res->n_evals = obj.evals;
        res->converged = converged;
        return status;
    };
    if (!obj.eval(x.data(), &f, g.data())) return finish(obj.status, 0);
    if (trace_out && opts->record_trace) trace_out[0] = f;
    std::vector<double> Hinv(size_t(n) * n, 0.0);
    for (int i = 0; i < n; ++i) Hinv[size_t(i) * n + i] = 1.0;
    std::vector<double> p(n), s(n), y(n), Hy(n);
    int k = 0;
    auto gmax = [&]() {
        double m = 0.0;
        for (double v : g) m = std::max(m, std::fabs(v));
        return m;
    };
    while (true) {
        if (gmax() <= opts->gtol) return finish(VQE_OK, 1);
        if (k >= opts->max_iter) return finish(VQE_OK, 0);
        if (opts->max_seconds > 0.0 && elapsed() > opts->max_seconds) return finish(VQE_OK, 0);
        for (int i = 0; i < n; ++i) {
            double acc = 0.0;
            const double* row = &Hinv[size_t(i) * n];
            for (int j = 0; j < n; ++j) acc -= row[j] * g[j];
            p[i] = acc;
        }
        if (dot(p, g) >= 0.0) {  // not a descent direction: restart from steepest descent
            for (int i = 0; i < n; ++i) {
                std::fill(&Hinv[size_t(i) * n], &Hinv[size_t(i) * n] + n, 0.0);
                Hinv[size_t(i) * n + i] = 1.0;
                p[i] = -g[i];
            }
        }
        LinePoint lp;
        bool found = line_search(obj, x, f, g, p, 1.0, lp);
        if (!found && obj.status == VQE_OK) {
            // retry once along steepest descent with a fresh Hessian model
            bool identity = true;
            for (int i = 0; i < n && identity; ++i)
                for (int j = 0; j < n; ++j)
                    if (Hinv[size_t(i) * n + j] != (i == j ? 1.0 : 0.0)) {
                        identity = false;
                        break;
                    }
            if (!identity) {
                for (int i = 0; i < n; ++i) {
                    std::fill(&Hinv[size_t(i) * n], &Hinv[size_t(i) * n] + n, 0.0);
                    Hinv[size_t(i) * n + i] = 1.0;
                    p[i] = -g[i];
                }
                found = line_search(obj, x, f, g, p, 1.0, lp);
            }
        }
        if (!found) {
            if (obj.status != VQE_OK) return finish(obj.status, 0);
            return finish(VQE_OK, 0);  // no further progress possible
        }
        for (int i = 0; i < n; ++i) {
            s[i] = lp.x[i] - x[i];
            y[i] = lp.g[i] - g[i];
        }
        const double f_old = f;
        x = lp.x;
        g = lp.g;
        f = lp.f;
        ++k;
        res->iters = k;
        if (trace_out && opts->record_trace) trace_out[k] = f;
        const double ys = dot(y, s);
        if (ys > 1e-300) {
            if (k == 1) {  // rescale H0 = (y's / y'y) I before the first update
                const double sc = ys / dot(y, y);
                for (auto& v : Hinv) v *= sc;
            }
            const double rho = 1.0 / ys;
            for (int i = 0; i < n; ++i) {
                double acc = 0.0;
                const double* row = &Hinv[size_t(i) * n];
                for (int j = 0; j < n; ++j) acc += row[j] * y[j];
                Hy[i] = acc;
            }
            const double yHy = dot(y, Hy);
            // H <- (I - rho s y') H (I - rho y s') + rho s s'
            //    = H - rho (s Hy' + Hy s') + (rho^2 y'Hy + rho) s s'
            const double c_ss = rho * rho * yHy + rho;
            for (int i = 0; i < n; ++i) {
                double* row = &Hinv[size_t(i) * n];
                for (int j = 0; j < n; ++j)
                    row[j] += -rho * (s[i] * Hy[j] + Hy[i] * s[j]) + c_ss * s[i] * s[j];
            }
        }
        if (opts->ftol > 0.0 && std::fabs(f_old - f) <= opts->ftol * std::max(1.0, std::fabs(f_old)))
            return finish(VQE_OK, 1);
    }
}

namespace {
struct RunCtx {
    const vqe_hamiltonian* H;
    const vqe_ansatz* A;
    int ne;
    void* stream;
};
int run_objective(void* ctx, int n, const double* x, double* f, double* g) {
    auto* c = static_cast<RunCtx*>(ctx);
    (void)n;
    return vqe_energy_grad(c->H, c->A, c->ne, x, f, g, c->stream);
}
}  // namespace

extern "C" int vqe_run(const vqe_hamiltonian* H, const vqe_ansatz* A, int n_electrons,
                       const double* theta0, const vqe_options* opts, double* theta_out,
                       double* trace_out, vqe_result* res, void* hip_stream) {
    if (!H || !A || !opts || !theta_out || !res) return fail(VQE_EINVAL, "null pointer argument");
    if (A->n_params < 1) return fail(VQE_ERANGE, "ansatz has no parameters");
    RunCtx ctx{H, A, n_electrons, hip_stream};
    return vqe_minimize_bfgs(A->n_params, run_objective, &ctx, theta0, opts, theta_out, trace_out,
                             res);
}

// ============================================================== ADAPT-VQE

namespace {
struct AnsatzHandle {
    vqe_ansatz* a = nullptr;
    ~AnsatzHandle() { vqe_ansatz_free(a); }
};
}  // namespace

// Sec. 2.1, "ADAPT-VQE algorithm": start from the identity ansatz, add the
// pool operator with the largest energy gradient (applied last, angle 0),
// re-optimise every angle, stop once the pool gradient is small.
extern "C" int vqe_adapt(const vqe_hamiltonian* H, const vqe_ansatz* pool, int n_electrons,
                         const vqe_adapt_options* opts, int32_t* selected, double* theta_out,
                         double* energy_trace, double* grad_norm_trace, vqe_adapt_result* res,
                         void* hip_stream) {
    if (!H || !pool || !opts || !res) return fail(VQE_EINVAL, "null pointer argument");
    if (opts->max_operators < 0) return fail(VQE_ERANGE, "max_operators is negative");
    if (opts->max_operators > 0 && (!selected || !theta_out))
        return fail(VQE_EINVAL, "null selected or theta_out");
    if (!(opts->grad_tol >= 0.0) || !(opts->tie_tol >= 0.0))
        return fail(VQE_EINVAL, "grad_tol and tie_tol must be non-negative");
    if (pool->n_params < 1) return fail(VQE_ERANGE, "pool has no parameters");
    *res = vqe_adapt_result{};
    const int cap = opts->max_operators;
    const size_t P = size_t(pool->n_params);
    std::vector<int32_t> sel;
    std::vector<double> theta, next, g(P);
    int evals = 0;
    for (;;) {
        AnsatzHandle A;
        if (int rc = vqe_ansatz_select(pool, int64_t(sel.size()), sel.data(), &A.a)) return rc;
        double e = 0.0;
        if (int rc = vqe_pool_gradient(H, A.a, pool, n_electrons, theta.data(), &e, g.data(),
                                       hip_stream))
            return rc;
        ++evals;
        double norm2 = 0.0, gmax = 0.0;
        for (double v : g) {
            norm2 += v * v;
            gmax = std::max(gmax, std::fabs(v));
        }
        const double norm = std::sqrt(norm2);
        const size_t k = sel.size();
        if (energy_trace) energy_trace[k] = e;
        if (grad_norm_trace) grad_norm_trace[k] = norm;
        res->energy = e;
        res->grad_norm = norm;
        res->n_operators = int32_t(k);
        res->n_evals = evals;
        if (norm < opts->grad_tol) {
            res->converged = 1;
            break;
        }
        if (int(k) >= cap) break;
        // the lowest pool index within tie_tol of the largest |gradient|
        size_t pick = 0;
        while (std::fabs(g[pick]) < gmax - opts->tie_tol) ++pick;
        sel.push_back(int32_t(pick));
        theta.push_back(0.0);
        AnsatzHandle B;
        if (int rc = vqe_ansatz_select(pool, int64_t(sel.size()), sel.data(), &B.a)) return rc;
        next.assign(theta.size(), 0.0);
        vqe_result r{};
        if (int rc = vqe_run(H, B.a, n_electrons, theta.data(), &opts->vqe, next.data(), nullptr, &r,
                             hip_stream))
            return rc;
        evals += r.n_evals;
        theta.swap(next);
        res->vqe_iters += r.iters;
    }
    for (size_t k = 0; k < sel.size(); ++k) {
        selected[k] = sel[k];
        theta_out[k] = theta[k];
    }
    return VQE_OK;
}
