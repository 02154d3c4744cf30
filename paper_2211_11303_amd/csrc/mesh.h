// Kuhn-split cube mesh and its Nedelec Galerkin matrix (host, setup).
#pragma once
#include <cstdint>
#include <vector>

namespace hlu {

// A = K_beta - kappa^2 M on the interior edges of the n^3 Kuhn cube, or of
// the union of its cubes (i, j, k) flagged in mask[i + n (j + n k)]; CSR with
// sorted columns, doubled midpoints (N x 3).  beta_box (cube indices lo[3],
// hi[3], half-open; null: none): cubes whose curl-curl term is scaled by
// beta_in.
void kuhn_assemble(int n, double kappa, std::vector<int32_t>* row_ptr, std::vector<int32_t>* col,
                   std::vector<double>* val, std::vector<int32_t>* mid2, int32_t* N,
                   const int32_t* beta_box = nullptr, double beta_in = 1.0, const uint8_t* mask = nullptr);
// Bounding box of the tetrahedra holding each interior edge (doubled units).
void kuhn_support_boxes(int n, std::vector<int32_t>* lo2, std::vector<int32_t>* hi2,
                        const uint8_t* mask = nullptr);
// b_j = <J, Phi_j> for a constant field J.
void kuhn_load(int n, const double J[3], std::vector<double>* b, const uint8_t* mask = nullptr);

}  // namespace hlu
