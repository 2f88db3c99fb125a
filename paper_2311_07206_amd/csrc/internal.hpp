// Internal declarations shared by the host parts of the library.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace sdc {

constexpr int kMaxNodes = 6;
constexpr int kMaxDiag = 32;   // diagonal storage limit (distinct column offsets per instance)

struct Collocation {
  int M;
  double tau[kMaxNodes];
  double Q[kMaxNodes][kMaxNodes];
  double QI[kMaxNodes][kMaxNodes];
  double QE[kMaxNodes][kMaxNodes];
};

// Radau-IIA collocation data; returns 0 on success.
int collocation(int M, Collocation* c);

// Host P1 assembly result (CSR with sorted column indices per row).
struct HostSystem {
  int64_t n = 0;
  std::vector<int32_t> rowptr;  // n+1
  std::vector<int32_t> col;     // nnz
  std::vector<double> val;      // nnz, A
  std::vector<double> ml;       // n, lumped mass
  std::vector<int32_t> diag;    // n, position of the diagonal entry in its row
};

// Assemble ML and A from simplices; returns an empty string or an error message.
std::string assemble_p1(int dim, int64_t n_nodes, const double* coords, int64_t n_elems,
                        const int32_t* elems, const double* elem_tensor,
                        const double* node_sigma, HostSystem* out);

// Add node-pair couplings w_q (e_a - e_b)(e_a - e_b)^T to the assembled A:
// A_aa, A_bb += w_q, A_ab, A_ba -= w_q; pairs with w_q = 0 only extend the
// pattern.  Then A_ii += diag[i] (diag may be null).  Recomputes the
// diagonal positions.
std::string add_pair_couplings(HostSystem* hs, int64_t n_pairs, const int32_t* a, const int32_t* b,
                               const double* w, const double* diag);

// Off-diagonal entries Khat_T[a][b], a < b (lexicographic pairs), of every
// element's unit-conductivity stiffness |T| g_a . D_T g_b.  Because the rows
// of Khat_T sum to zero, psi^T Khat_T u = -sum_{a<b} Khat_ab (psi_a - psi_b)(u_a - u_b).
std::string element_pairs(int dim, const double* coords, int64_t ne, const int32_t* elems,
                          const double* elem_tensor, std::vector<double>* w);

}  // namespace sdc
