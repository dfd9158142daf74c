// Host-side construction of a quantum Tanner code from (G, A, B, C_A, C_B)
// (Sec. II-A, II-B of the LEAD paper) and of the tables the decoding kernels
// consume.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

namespace lead {

constexpr int kMaxDelta = 8;

// Tables of one check type (Z checks on V0 or X checks on V1).
struct TypeTables {
    int r = 0;                          // checks per vertex
    std::vector<uint64_t> mask;         // r masks over the delta^2 local variables
    std::vector<int32_t> view;          // order x delta^2 qubit ids
    std::vector<int32_t> csr_ptr, csr_idx;  // global H, rows g*r + rho
    int rank = 0;
    int eloc = 0;
    // Each qubit sits in exactly two views; partner[v*D2+j] = v'*D2+j' is the
    // other occurrence.  owned[v*D2+j] = 1 for the occurrence that owns the
    // qubit (computes its shared quantities).  On a Cayley complex the local
    // position of the other occurrence depends on j alone: sigma[j] = j' for
    // every view (sigma is empty when that does not hold).  Then position j
    // owns its qubit in every view when j < sigma[j]; the qubits at fixed
    // points of sigma (and every qubit when sigma is empty) are oriented
    // along Euler tours of the view multigraph.  Either way every view owns
    // at most ceil(D2/2) qubits.
    std::vector<int32_t> partner;
    std::vector<int32_t> sigma;
    std::vector<uint8_t> owned;
    int own_max = 0;
};

struct Code {
    int order = 0, delta = 0, n = 0, kA = 0, kB = 0, k = 0;
    std::vector<uint16_t> mul;
    std::vector<int32_t> A, B;
    uint64_t rrefA[kMaxDelta] = {}, rrefB[kMaxDelta] = {};    // RREF bases of C_A, C_B
    uint64_t dualA[kMaxDelta] = {}, dualB[kMaxDelta] = {};    // RREF bases of the duals
    TypeTables t[2];
};

// Returns 0 (LEAD_OK) or a negative lead_status; message in `err`.
int build_code(int order, const uint16_t *mul, int delta, const int32_t *A, const int32_t *B, int kA,
               const uint64_t *GA, int kB, const uint64_t *GB, Code &out, std::string &err);

}  // namespace lead
