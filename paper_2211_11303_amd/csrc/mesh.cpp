// Kuhn-split cube mesh and the lowest-order Nedelec Galerkin matrix
// A = K - kappa^2 M (Sec. 2.1, eq. (5), eq. (8)) on its interior edges.
//
// Every cube (i,j,k) of the n^3 grid (or of a union of its cubes) is cut into the six tetrahedra
// {c, c+e_p0, c+e_p0+e_p1, c+(1,1,1)}, one per axis permutation p.  Edges
// run from the lower vertex id to the higher; an edge is interior unless both
// ends lie in one boundary face plane.  The Whitney function of edge (a,b) is
// lambda_a grad(lambda_b) - lambda_b grad(lambda_a); its curl is
// 2 grad(lambda_a) x grad(lambda_b), and the mass integrals use
// int_T lambda_x lambda_y = |T| (1 + delta_xy) / 20, so both element
// matrices are exact.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>

#include "common.h"
#include "mesh.h"

namespace hlu {
namespace {

// The seven edge directions of the Kuhn mesh, ordered by the id offset they
// add (so that the outgoing edges of a vertex come in increasing head id).
const int kDir[7][3] = {{1, 0, 0}, {0, 1, 0}, {1, 1, 0}, {0, 0, 1},
                        {1, 0, 1}, {0, 1, 1}, {1, 1, 1}};

int dir_index(int dx, int dy, int dz) {
  for (int d = 0; d < 7; ++d)
    if (kDir[d][0] == dx && kDir[d][1] == dy && kDir[d][2] == dz) return d;
  return -1;
}

// Interior edges of the domain: the whole cube, or the union of the cubes
// (i, j, k) flagged in mask[i + n (j + n k)].  The edge from lattice point p
// to p + d (d one of kDir) lies in the cubes c with c_a = p_a where d_a = 1
// and c_a in {p_a - 1, p_a} where d_a = 0; it belongs to the mesh if one of
// them is in the domain.  It lies on the boundary if it lies in a boundary
// face: a square of a plane x_a = p_a (d_a = 0) with exactly one of its two
// cubes in the domain.  Such a square contains the edge if its lower corner
// q has q_b = p_b where d_b = 1 and q_b in {p_b - 1, p_b} where d_b = 0
// (the Kuhn split cuts every square along the diagonal from its lowest to
// its highest corner, which is the edge direction with two ones).
struct KuhnDofs {
  int n;
  const uint8_t* mask;
  int64_t nv;
  std::vector<int32_t> dof;  // [vertex * 7 + dir] -> interior dof or -1
  int32_t N = 0;

  bool in(int i, int j, int k) const {
    if (i < 0 || j < 0 || k < 0 || i >= n || j >= n || k >= n) return false;
    return !mask || mask[i + (int64_t)n * (j + (int64_t)n * k)] != 0;
  }

  KuhnDofs(int n_, const uint8_t* mask_) : n(n_), mask(mask_), nv((int64_t)(n_ + 1) * (n_ + 1) * (n_ + 1)) {
    dof.assign(nv * 7, -1);
    for (int64_t v = 0; v < nv; ++v) {
      int p[3] = {int(v % (n + 1)), int((v / (n + 1)) % (n + 1)), int(v / ((int64_t)(n + 1) * (n + 1)))};
      for (int d = 0; d < 7; ++d) {
        const int* e = kDir[d];
        // cube corners c_a in [lo_a, p_a]
        int lo[3];
        for (int a = 0; a < 3; ++a) lo[a] = p[a] + e[a] - 1;
        bool exists = false;
        for (int c2 = lo[2]; c2 <= p[2] && !exists; ++c2)
          for (int c1 = lo[1]; c1 <= p[1] && !exists; ++c1)
            for (int c0 = lo[0]; c0 <= p[0] && !exists; ++c0) exists = in(c0, c1, c2);
        if (!exists) continue;
        bool boundary = false;
        for (int a = 0; a < 3 && !boundary; ++a) {
          if (e[a] != 0) continue;
          const int b = (a + 1) % 3, c = (a + 2) % 3;
          for (int qb = lo[b]; qb <= p[b] && !boundary; ++qb)
            for (int qc = lo[c]; qc <= p[c] && !boundary; ++qc) {
              if (qb < 0 || qc < 0 || qb >= n || qc >= n) continue;
              int below[3], above[3];
              below[a] = p[a] - 1;
              above[a] = p[a];
              below[b] = above[b] = qb;
              below[c] = above[c] = qc;
              boundary = in(below[0], below[1], below[2]) != in(above[0], above[1], above[2]);
            }
        }
        if (!boundary) dof[v * 7 + d] = N++;
      }
    }
  }
  int64_t vid(int i, int j, int k) const { return i + (int64_t)(n + 1) * (j + (int64_t)(n + 1) * k); }
};

void cross(const double* a, const double* b, double* c) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}
double dot3(const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

const int kLocalEdge[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};

// Barycentric gradients g[4][3] of one tetrahedron with vertex coordinates
// x[4][3]; returns its volume.
double gradients(const double x[4][3], double g[4][3]) {
  double J[3][3];  // columns x1-x0, x2-x0, x3-x0
  for (int c = 0; c < 3; ++c)
    for (int r = 0; r < 3; ++r) J[r][c] = x[c + 1][r] - x[0][r];
  double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
               J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
               J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
  double vol = std::fabs(det) / 6.0;
  // rows of J^{-1} are the gradients of lambda_1..lambda_3
  double inv[3][3];
  inv[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) / det;
  inv[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
  inv[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
  inv[1][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) / det;
  inv[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
  inv[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
  inv[2][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) / det;
  inv[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
  inv[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
  for (int a = 0; a < 3; ++a) {
    g[a + 1][0] = inv[a][0];
    g[a + 1][1] = inv[a][1];
    g[a + 1][2] = inv[a][2];
  }
  for (int c = 0; c < 3; ++c) g[0][c] = -(g[1][c] + g[2][c] + g[3][c]);
  return vol;
}

// Local K and M of one tetrahedron with vertex coordinates x[4][3].
void element(const double x[4][3], double Kl[6][6], double Ml[6][6]) {
  double g[4][3];
  const double vol = gradients(x, g);
  auto I = [&](int p, int q) { return vol * (p == q ? 2.0 : 1.0) / 20.0; };
  for (int e = 0; e < 6; ++e) {
    int a = kLocalEdge[e][0], b = kLocalEdge[e][1];
    double ce[3];
    cross(g[a], g[b], ce);
    for (int f = 0; f < 6; ++f) {
      int c = kLocalEdge[f][0], d = kLocalEdge[f][1];
      double cf[3];
      cross(g[c], g[d], cf);
      Kl[e][f] = 4.0 * vol * dot3(ce, cf);
      Ml[e][f] = dot3(g[b], g[d]) * I(a, c) - dot3(g[b], g[c]) * I(a, d) -
                 dot3(g[a], g[d]) * I(b, c) + dot3(g[a], g[c]) * I(b, d);
    }
  }
}

struct Triplet {
  int32_t r, c;
  double v;
};

// Lattice vertices v[4][3] of tetrahedron p (axis permutation) of cube
// (i, j, k): the monotone path c, c + e_p0, c + e_p0 + e_p1, c + (1,1,1).
void tet_vertices(int i, int j, int k, int p, int v[4][3]) {
  static const int perms[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
  v[0][0] = i;
  v[0][1] = j;
  v[0][2] = k;
  for (int s = 0; s < 3; ++s) {
    for (int a = 0; a < 3; ++a) v[s + 1][a] = v[s][a];
    v[s + 1][perms[p][s]] += 1;
  }
}

// Interior dof of the local edges of a tetrahedron (-1: boundary edge).
void local_dofs(const KuhnDofs& D, const int v[4][3], int32_t ld[6]) {
  for (int e = 0; e < 6; ++e) {
    const int* va = v[kLocalEdge[e][0]];
    const int* vb = v[kLocalEdge[e][1]];
    const int d = dir_index(vb[0] - va[0], vb[1] - va[1], vb[2] - va[2]);
    ld[e] = D.dof[D.vid(va[0], va[1], va[2]) * 7 + d];
  }
}

// beta_box (cube indices lo[3], hi[3], half-open; null: none): the cubes
// whose tetrahedra carry the curl-curl coefficient beta_in (1 elsewhere).
void assemble(int n, double kappa, std::vector<int32_t>* row_ptr, std::vector<int32_t>* col,
              std::vector<double>* val, std::vector<int32_t>* mid2, int32_t* Nout, const int32_t* beta_box,
              double beta_in, const uint8_t* mask) {
  KuhnDofs D(n, mask);
  const int N = D.N;
  const double k2 = kappa * kappa;
  std::vector<Triplet> trip;
  trip.reserve((size_t)6 * n * n * n * 36);
  for (int k = 0; k < n; ++k)
    for (int j = 0; j < n; ++j)
      for (int i = 0; i < n; ++i)
        for (int p = 0; p < 6 && D.in(i, j, k); ++p) {
          int v[4][3];
          tet_vertices(i, j, k, p, v);
          double x[4][3];
          for (int s = 0; s < 4; ++s)
            for (int a = 0; a < 3; ++a) x[s][a] = double(v[s][a]) / n;
          double Kl[6][6], Ml[6][6];
          element(x, Kl, Ml);
          const bool in_box = beta_box && i >= beta_box[0] && i < beta_box[3] && j >= beta_box[1] &&
                              j < beta_box[4] && k >= beta_box[2] && k < beta_box[5];
          const double beta = in_box ? beta_in : 1.0;
          int32_t ld[6];
          local_dofs(D, v, ld);
          for (int e = 0; e < 6; ++e) {
            if (ld[e] < 0) continue;
            for (int f = 0; f < 6; ++f) {
              if (ld[f] < 0) continue;
              trip.push_back({ld[e], ld[f], beta * Kl[e][f] - k2 * Ml[e][f]});
            }
          }
        }
  std::sort(trip.begin(), trip.end(), [](const Triplet& a, const Triplet& b) {
    return a.r != b.r ? a.r < b.r : a.c < b.c;
  });
  row_ptr->assign(N + 1, 0);
  col->clear();
  val->clear();
  for (size_t t = 0; t < trip.size();) {
    size_t u = t;
    double s = 0.0;
    // sum duplicates in the order the elements were visited
    while (u < trip.size() && trip[u].r == trip[t].r && trip[u].c == trip[t].c) s += trip[u++].v;
    col->push_back(trip[t].c);
    val->push_back(s);
    (*row_ptr)[trip[t].r + 1]++;
    t = u;
  }
  for (int r = 0; r < N; ++r) (*row_ptr)[r + 1] += (*row_ptr)[r];
  if (mid2) {
    mid2->assign((size_t)3 * N, 0);
    for (int64_t vtx = 0; vtx < D.nv; ++vtx)
      for (int d = 0; d < 7; ++d) {
        int32_t q = D.dof[vtx * 7 + d];
        if (q < 0) continue;
        int p[3] = {int(vtx % (n + 1)), int((vtx / (n + 1)) % (n + 1)), int(vtx / ((int64_t)(n + 1) * (n + 1)))};
        for (int a = 0; a < 3; ++a) (*mid2)[3 * q + a] = 2 * p[a] + kDir[d][a];
      }
  }
  *Nout = N;
}

}  // namespace

void kuhn_assemble(int n, double kappa, std::vector<int32_t>* row_ptr, std::vector<int32_t>* col,
                   std::vector<double>* val, std::vector<int32_t>* mid2, int32_t* N, const int32_t* beta_box,
                   double beta_in, const uint8_t* mask) {
  assemble(n, kappa, row_ptr, col, val, mid2, N, beta_box, beta_in, mask);
}

// Support box of every interior edge's basis function: the bounding box of
// the tetrahedra that contain the edge, in doubled lattice units (the units
// of the midpoints), lo2 and hi2 N x 3.
void kuhn_support_boxes(int n, std::vector<int32_t>* lo2, std::vector<int32_t>* hi2, const uint8_t* mask) {
  KuhnDofs D(n, mask);
  lo2->assign((size_t)3 * D.N, INT32_MAX);
  hi2->assign((size_t)3 * D.N, INT32_MIN);
  for (int k = 0; k < n; ++k)
    for (int j = 0; j < n; ++j)
      for (int i = 0; i < n; ++i)
        for (int p = 0; p < 6 && D.in(i, j, k); ++p) {
          int v[4][3];
          tet_vertices(i, j, k, p, v);
          int32_t ld[6];
          local_dofs(D, v, ld);
          for (int e = 0; e < 6; ++e) {
            if (ld[e] < 0) continue;
            for (int s = 0; s < 4; ++s)
              for (int a = 0; a < 3; ++a) {
                int32_t& l = (*lo2)[3 * (size_t)ld[e] + a];
                int32_t& h = (*hi2)[3 * (size_t)ld[e] + a];
                l = std::min(l, 2 * v[s][a]);
                h = std::max(h, 2 * v[s][a]);
              }
          }
        }
}

// b_j = <J, Phi_j> for a constant field J (the right-hand side of the weak
// form, Sec. 2.1): the integral of a barycentric coordinate over T is |T|/4,
// so T adds |T|/4 J.(grad lambda_b - grad lambda_a) to its local edge (a, b).
void kuhn_load(int n, const double J[3], std::vector<double>* b, const uint8_t* mask) {
  KuhnDofs D(n, mask);
  b->assign(D.N, 0.0);
  for (int k = 0; k < n; ++k)
    for (int j = 0; j < n; ++j)
      for (int i = 0; i < n; ++i)
        for (int p = 0; p < 6 && D.in(i, j, k); ++p) {
          int v[4][3];
          tet_vertices(i, j, k, p, v);
          double x[4][3], g[4][3];
          for (int s = 0; s < 4; ++s)
            for (int a = 0; a < 3; ++a) x[s][a] = double(v[s][a]) / n;
          const double vol = gradients(x, g);
          int32_t ld[6];
          local_dofs(D, v, ld);
          for (int e = 0; e < 6; ++e) {
            if (ld[e] < 0) continue;
            const int a = kLocalEdge[e][0], c = kLocalEdge[e][1];
            double d[3] = {g[c][0] - g[a][0], g[c][1] - g[a][1], g[c][2] - g[a][2]};
            (*b)[ld[e]] += vol / 4.0 * dot3(J, d);
          }
        }
}

}  // namespace hlu
