// Internal structures shared by the host builders (vqe_host.cpp) and the
// device path (vqe_device.hip).  Not part of the C ABI.
#pragma once

#include <cstdint>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/vqe.h"

namespace vqe {

// ---------------------------------------------------------------- errors
int fail(int code, const std::string& msg);   // records the message, returns code
void clear_error();

// ---------------------------------------------------------------- Hamiltonian
//
// Terms are kept in folded form  c' X^x Z^z  (real c'), sorted by (x, z) and
// grouped by x.  For the device each x-group g is re-expressed relative to
// the OUTPUT index b' of lambda = H psi:
//   lambda[b'] = sum_g psi[b' ^ x_g] * D_g(b'),
//   D_g(b')    = sum_{s in sub(g)} (-1)^{popcount(b' & w_s)} * tab_s[pext(b', x_g)],
// where a subgroup s collects the terms of g whose z agrees outside x
// (w_s = z & ~x) and tab_s holds their combined coefficient for each pattern
// of the x bits of b'.  Groups whose x has more than kMaxTabBits bits use
// one subgroup per term with w = z and a one-entry table.
constexpr int kMaxTabBits = 4;

struct GroupDesc {
    uint32_t x;        // flip mask
    uint32_t pos;      // bits 0..2: k (table bits); then four 5-bit positions, the
                       // k table bits in ascending order, unused slots = 31
    int32_t sub_begin; // subgroup range [sub_begin, sub_end)
    int32_t sub_end;
};

struct SubDesc {
    uint32_t w;        // sign mask applied to the output index
    int32_t tab;       // offset of the 2^k-entry table in the table array
};

struct DevHam;  // device copy (vqe_device.hip)

}  // namespace vqe

struct vqe_hamiltonian {
    int n = 0;
    std::vector<uint32_t> x, z;       // sorted terms (folded form)
    std::vector<double> c;
    // group structure (host copy of what is uploaded)
    std::vector<vqe::GroupDesc> groups;
    std::vector<vqe::SubDesc> subs;
    std::vector<double> tabs;
    int32_t diag_group = -1;          // index of the x = 0 group, -1 if none
    mutable std::mutex mu;
    mutable std::map<int, vqe::DevHam*> dev;  // per device ordinal
    // this Hamiltonian in the occupation basis of an encoding (keyed by the
    // encoding's rows of beta^-1), made on first use
    mutable std::map<std::vector<uint32_t>, vqe_hamiltonian*> occ;
    ~vqe_hamiltonian();
};

namespace vqe {

enum GateType : int32_t { kExcitation = 0, kPauli = 1 };

// One gate of an ansatz program.
//  kExcitation: Givens rotation exp(theta (T - T^dag)) on the pairs
//    (D, E = D ^ x) with (D & x) == pd; sign s(D) = csign * (-1)^{popcount(D & chain)};
//    new D = cos*D - s*sin*E, new E = cos*E + s*sin*D, angle = scale * theta[param].
//  kPauli: exp(-i phi/2 P(x, z)), phi = scale * theta[param]; chain holds z.
struct GateDesc {
    uint32_t x;
    uint32_t pd;
    uint32_t chain;
    int32_t type;
    int32_t param;
    int32_t pad;
    double scale;
    double csign;
};
static_assert(sizeof(GateDesc) == 40, "GateDesc layout");

struct DevAnsatz;

}  // namespace vqe

struct vqe_ansatz {
    int n = 0;
    int n_electrons = -1;             // UCCSD reference, -1 for rotation lists
    int64_t ref_bits = -1;            // reference basis index; -1: the lowest n_electrons qubits
    int32_t n_params = 0;
    bool sector_conserving = false;   // every gate conserves N and S_z
    std::vector<vqe::GateDesc> gates;
    std::vector<int32_t> exc;         // 4 per gate for UCCSD (i, a, -1, -1) / (i, j, a, b)
    // UCCSD under a linear encoding b = beta n other than Jordan-Wigner: the
    // same excitations in the occupation basis (owned; null otherwise), with
    // the encoding's columns (enc_c[P]: the qubits that flip with n_P) and
    // the rows of beta^-1 (enc_r[P]: n_P as a parity of qubits)
    vqe_ansatz* occ = nullptr;
    uint32_t enc_c[32] = {}, enc_r[32] = {};
    mutable std::mutex mu;
    mutable std::map<int, vqe::DevAnsatz*> dev;
    ~vqe_ansatz();
};

namespace vqe {
// Host-side helpers used by both translation units.
bool finite_all(const double* v, int64_t n);
// H with every term's masks taken to the occupation basis of the encoding
// (enc_c, enc_r as in vqe_ansatz): X^x Z^z on encoded qubits acts on
// occupations as X^{beta^-1 x} Z^{beta^T z} with the same coefficient.
int hamiltonian_to_occupation(const vqe_hamiltonian* H, const uint32_t* enc_c, const uint32_t* enc_r,
                              vqe_hamiltonian** out);
}  // namespace vqe
