// Oracle for the 3D crack element method step -- TEST INFRASTRUCTURE ONLY.
//
// Plain FP64 CPU implementation, written for readability, not speed.  Only the
// tests, the smoke check and the bench's CPU-baseline leg load it; the GPU
// library shares no code with it.  Each function names the passage of the
// paper it follows.  Readings of silent or garbled passages:
//   * energy density psi = lambda/2 (tr eps)^2 + mu eps:eps  (Section 2.1; the
//     printed density is garbled), so sigma = lambda tr(eps) I + 2 mu eps;
//   * smoothing-domain volume of edge k is V_k = (1/6) sum of the volumes of
//     the elements sharing the edge (expanded form of Eq. CSTet_fint);
//   * lumped mass m_i = sum rho V_e / 4 over the elements holding node i;
//   * face traction t on a boundary triangle of area A adds t A / 3 to each
//     vertex (the paper writes the load with a 2D line segment);
//   * Newmark beta = 0 with gamma = 1/2 (gamma is not printed);
//   * stretch test: |x_j - x_i| > |X_j - X_i| evaluated as
//     2 dX.du + |du|^2 > 0; the Heaviside step at 0 is 0;
//   * the "maximum principal stress vector" projected on n is taken as
//     sigma_1 |P_1 n| (P_1: projector on the eigenspace of the largest
//     eigenvalue; eigenvalues within 1e-6 max|lambda| of the largest count as
//     tied, because stresses computed in two different summation orders
//     differ by rounding and the eigenvector of a closer pair moves by that
//     rounding over the gap), or n.sigma.n (gsig = 1);
//     projected stretches enter as |delta.n|;
//   * crack front: a face of an intact tet shared with a split tet whose
//     partition cuts that face; the node alone on its side is N2, the other
//     face nodes N1 < N3 (local order), N4 the intact tet's opposite node;
//   * Griffith test G >= Gc (Section 2.1); ties go to the lower local face,
//     then pattern I before II; all splits of a step are decided on one state
//     and applied together in ascending tet id; a tet splits at most once;
//   * a split tet becomes two phantom-node copies (or is removed in erosion
//     mode); each copy keeps the parent's gradients, volume fraction 1/2
//     (2|2 partition) or 1/8 and 7/8 (1|3 partition, the lone side gets 1/8),
//     its own side's real nodes and fresh extra nodes for the other side,
//     which copy the twin's position and u, v, a; masses are rebuilt from the
//     elements (kept fixed in erosion mode);
//   * dissipated energy U_d = Gc * (midpoint crack area) summed over splits
//     decided by the G test (host pre-splits excluded);
//   * critical step dt_crit = 2 / sqrt(max_e (4/rho) lambda_max(B^T C B));
//   * a Young's modulus per tetrahedron (split copies keep their parent's)
//     enters the smoothing domain of edge k as C_k = sum_j w_jk C_j, the
//     volume average of the element matrices over the domain, so that
//     sigma_k = C_k eps_k;
//   * trilinear hexahedra (Eqs. hex_strain_discretization and
//     hex_fint_discretization): as Eq. strain_discretization states, hex j
//     enters the smoothing domain of edge k with its shape-function gradients
//     evaluated at that edge's point G_k, the midpoint of the hex edge; edges
//     are the 12 hex edges, the smoothing domain of edge k has
//     V_k = (1/12) sum of the volumes sharing it and the volume weights
//     w_jk = V_j / sum V; the hex volume is exact with 2 x 2 x 2 Gauss points;
//     the lumped mass is rho V / 8 per node;
//   * hex crack patterns (Section 3, the parallelepiped patterns; the figure
//     that draws them is missing from the text): cut planes are taken in the
//     hex's natural coordinates xi through edge midpoints, c . xi = d with
//     c in {-1, 0, 1}^3: the three mid-planes (d = 0), twelve wedge planes
//     (two nonzero c, d = 1, cutting off the prism around one hex edge) and
//     eight corner planes (three nonzero c, d = 2); a plane's cut edges are
//     the edges whose midpoints lie on it.  A crack front is a face of an
//     intact hex shared with a cracked hex whose plane cuts that face (at
//     two of its edges, G1 on the lower local edge, G2 on the other).  Two
//     opposite edges give III (the mid-plane through G1 G2, deactivating the
//     hex) and IV (the two wedge planes through G1 G2 tilted toward either
//     side), two neighbouring edges give V (the wedge plane through G1 G2
//     along the face normal) and VI (the corner plane through G1 G2 and the
//     midpoint G6 of the edge at their shared corner along the face normal).
//     G_III, G_IV, G_V take Eq. G-I over the quad G1 G2 G4 G3, with G3 (G4)
//     the fourth-edge point joined to G1 (G2), n the unit normal of the
//     quad's diagonals, delta_1 and delta_2 the stretches of the G1 and G2
//     edges; G_VI takes Eq. G-II over the triangle G1 G2 G6.  A III hex
//     carries no volume after it cracks; after IV, V or VI the hex keeps its
//     edge-point gradients and carries half its volume, the triangular prism
//     (three tetrahedra of its own nodes) on the far side of the crack; its
//     mass is kept; a hex cracks once; ties: larger G, then the lower local
//     face, then III, IV toward -1, IV toward +1, V, VI; the crack area for
//     U_d is that of the quad or the triangle;
//   * hex critical step: the element bound takes the largest stiffness over
//     the hex's edge points, (8 / rho) max_q lambda_max(B_q^T C B_q), which is
//     at least lambda_max of its edge-averaged stiffness;
//   * a prescribed velocity v0 r_v(t) on listed degrees of freedom, with the
//     ramp r_v = t / t0 up to t0 and 1 after (Section 4 examples), fixes the
//     displacement to u_ref + v0 S(t), S the integral of r_v, the velocity to
//     v0 r_v(t) and the acceleration to v0 dr_v/dt (1/t0 on the ramp, taken on
//     the ramp at t = t0, else 0); the reaction is m a + f_int - f_ext on those
//     degrees of freedom; extra nodes of split copies are not constrained;
//   * the gradient of a window of fixed-topology steps is the exact reverse
//     (discrete adjoint) of the Newmark update, with the per-tet modulus,
//     the initial displacement and the initial velocity as the inputs.
#include "oracle.h"

#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <map>
#include <string>
#include <thread>
#include <utility>
#include <vector>

namespace {

typedef std::array<double, 3> V3;

V3 sub(const V3& a, const V3& b) { return {a[0] - b[0], a[1] - b[1], a[2] - b[2]}; }
double dot(const V3& a, const V3& b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
V3 cross(const V3& a, const V3& b) {
  return {a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]};
}
double norm(const V3& a) { return std::sqrt(dot(a, a)); }

// Runs fn(lo, hi) over nt contiguous pieces of [0, n) on nt threads (the
// calling thread alone when nt <= 1).  Callers give each item to exactly one
// piece and keep every per-item sum in the serial order, so results do not
// depend on nt.
template <class Fn>
void par_range(int nt, size_t n, Fn fn) {
  if (nt <= 1 || n < 2) {
    fn((size_t)0, n);
    return;
  }
  std::vector<std::thread> th;
  for (int t = 0; t < nt; ++t) {
    size_t lo = n * t / nt, hi = n * (t + 1) / nt;
    th.emplace_back([=] { fn(lo, hi); });
  }
  for (auto& x : th) x.join();
}

// Cyclic Jacobi eigen-decomposition of a symmetric n x n matrix (row-major).
// On return w holds the eigenvalues and column i of vec the i-th eigenvector.
void jacobi_eig(int n, std::vector<double> A, double* w, double* vec) {
  std::vector<double> Vm(n * n, 0.0);
  for (int i = 0; i < n; ++i) Vm[i * n + i] = 1.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, diag = 0.0;
    for (int p = 0; p < n; ++p) {
      diag += A[p * n + p] * A[p * n + p];
      for (int q = p + 1; q < n; ++q) off += A[p * n + q] * A[p * n + q];
    }
    if (off == 0.0 || off <= 1e-36 * diag) break;
    for (int p = 0; p < n; ++p) {
      for (int q = p + 1; q < n; ++q) {
        double apq = A[p * n + q];
        if (apq == 0.0) continue;
        double theta = (A[q * n + q] - A[p * n + p]) / (2.0 * apq);
        double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < n; ++k) {  // A <- A G
          double akp = A[k * n + p], akq = A[k * n + q];
          A[k * n + p] = c * akp - s * akq;
          A[k * n + q] = s * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {  // A <- G^T A
          double apk = A[p * n + k], aqk = A[q * n + k];
          A[p * n + k] = c * apk - s * aqk;
          A[q * n + k] = s * apk + c * aqk;
        }
        for (int k = 0; k < n; ++k) {  // V <- V G
          double vkp = Vm[k * n + p], vkq = Vm[k * n + q];
          Vm[k * n + p] = c * vkp - s * vkq;
          Vm[k * n + q] = s * vkp + c * vkq;
        }
      }
    }
  }
  for (int i = 0; i < n; ++i) w[i] = A[i * n + i];
  if (vec)
    for (int i = 0; i < n * n; ++i) vec[i] = Vm[i];
}

struct Elem {
  int nn = 4;        // nodes: 4 (tet) or 8 (hex)
  int n[8];          // node ids (real or extra)
  double g[8][3];    // dN_l/dx of a tet, Section 2.2 (constant; hexes: per edge point, orc_ctx::hexg)
  double V;          // volume of the parent tetrahedron
  double Veff;       // volume the element carries (V, a fraction of V, or 0)
  int parent;        // original tet id
};

struct Event {
  int step, tet, mask, pattern;
  double G;
};

struct FrontRec {
  int c, face, lone;
  double GI, GII;
};

int popcount4(int m) { return (m & 1) + ((m >> 1) & 1) + ((m >> 2) & 1) + ((m >> 3) & 1); }

}  // namespace

struct orc_ctx {
  int status = 0;
  std::string err;
  double E = 0, nu = 0, rho = 0, Gc = 0, lam = 0, mu = 0;
  int mode = 0, gsig = 0;
  int N0 = 0, T0 = 0;
  double D = 6.0;  // V_k = (1/D) sum of the patch volumes: 6 (tets), 12 (hexes)
  std::vector<V3> X;
  std::vector<Elem> el;
  std::map<std::pair<int, int>, int> edge_of;
  std::vector<std::pair<int, int>> edge_nodes;
  std::vector<std::vector<int>> patch;
  std::vector<std::vector<int>> patch_q;  // local edge of each patch element on that edge
  // hexes: grad N_i at the midpoint of local edge q, [(q * 8 + i) * 3 + d]
  std::vector<std::array<double, 288>> hexg;
  std::vector<std::array<int, 4>> orig;  // original (oriented) connectivity
  std::vector<std::array<int, 4>> nbr, nbr_face;
  std::vector<std::array<int, 6>> hnbr, hnbr_face;  // hexes: neighbour across local face f
  std::vector<int> smask;  // per original tet: -1 intact, else side mask
  std::vector<double> m;
  std::vector<V3> F;
  std::vector<double> Et;  // Young's modulus of each original tet
  bool hetero = false;     // Et differs from the scalar E
  bool frozen = false;     // topology frozen: no crack pass
  int nthreads = 1;        // threads of the element, edge and node loops
  // prescribed velocities (Dirichlet), in groups: per constrained node its
  // group, dof mask (bit d), v0, u_ref and current reaction; per group the
  // ramp time, the reactions' work and a history row per step
  std::vector<int> bc_node, bc_mask, bc_group;
  std::vector<V3> bc_v0, bc_uref, bc_R;
  std::vector<double> grp_t0, grp_W;
  std::vector<std::vector<std::array<double, 6>>> grp_hist;  // step, t, R_x, R_y, R_z, S(t)
  double ramp_t0 = 0;
  double dt = 0;
  long step = 0;
  std::vector<V3> u, v, a;
  bool need_init = true;
  double W = 0, Ud = 0, Gmax = 0;
  int nfront = 0, nsplit = 0;
  std::vector<Event> events;
  bool replay = false;
  std::vector<Event> schedule;
  size_t cursor = 0;

  int fail(int code, const std::string& msg) {
    err = msg;
    return code;
  }
};

namespace {

// Linear elasticity, Section 2.1: Lame constants from E and nu.
void lame(double E, double nu, double* lam, double* mu) {
  *lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
  *mu = E / (2.0 * (1.0 + nu));
}

// 6x6 elasticity matrix in the paper's Voigt order
// (e11, e22, e33, g12, g23, g13) with engineering shear strains.
void cmat(double lam, double mu, double C[6][6]) {
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) C[i][j] = 0.0;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) C[i][j] = lam + (i == j ? 2.0 * mu : 0.0);
  for (int i = 3; i < 6; ++i) C[i][i] = mu;
}

// Linear tetrahedron geometry (Section 2.2): with J = [X1-X0 | X2-X0 | X3-X0],
// V = det J / 6 and dN_l/dx (l = 1..3) is row l of J^{-1}; dN_0 = -sum.
double tet_geometry(const V3 x[4], double g[4][3]) {
  double J[3][3];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) J[r][c] = x[c + 1][r] - x[0][r];
  double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
               J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
               J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
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
  for (int l = 1; l <= 3; ++l)
    for (int d = 0; d < 3; ++d) g[l][d] = inv[l - 1][d];
  for (int d = 0; d < 3; ++d) g[0][d] = -(g[1][d] + g[2][d] + g[3][d]);
  return det / 6.0;
}

// Strain-displacement matrix B (6 x 3nn) of Eqs. CSTet_strain_discretization
// and hex_strain_discretization, columns ordered (u_0, v_0, w_0, u_1, ...).
void bmat_of(const double (*g)[3], int nn, double B[6][24]) {
  for (int r = 0; r < 6; ++r)
    for (int c = 0; c < 24; ++c) B[r][c] = 0.0;
  for (int l = 0; l < nn; ++l) {
    double gx = g[l][0], gy = g[l][1], gz = g[l][2];
    int c = 3 * l;
    B[0][c + 0] = gx;
    B[1][c + 1] = gy;
    B[2][c + 2] = gz;
    B[3][c + 0] = gy;
    B[3][c + 1] = gx;
    B[4][c + 1] = gz;
    B[4][c + 2] = gy;
    B[5][c + 0] = gz;
    B[5][c + 2] = gx;
  }
}

void bmat(const Elem& e, double B[6][24]) { bmat_of(e.g, e.nn, B); }

// Strain-displacement matrix of element j in the smoothing domain of its local
// edge q: tets have one (constant gradients); a hex uses its gradients at the
// midpoint of edge q (Eq. strain_discretization evaluates them at G_k).
void elem_bmat(const orc_ctx* c, int j, int q, double B[6][24]) {
  if (c->el[j].nn == 8)
    bmat_of(reinterpret_cast<const double(*)[3]>(c->hexg[j].data() + 24 * q), 8, B);
  else
    bmat(c->el[j], B);
}

// Voigt stress vector (s11, s22, s33, s12, s23, s13) -> symmetric 3x3 tensor.
void voigt_to_tensor(const double* s, double T[9]) {
  T[0] = s[0]; T[1] = s[3]; T[2] = s[5];
  T[3] = s[3]; T[4] = s[1]; T[5] = s[4];
  T[6] = s[5]; T[7] = s[4]; T[8] = s[2];
}

// Stress term of Eqs. G-I / G-II: the component of the maximum principal
// stress along the crack normal n.  gsig 0: sigma_1 * |P_1 n| with P_1 the
// projector on the eigenspace of the largest eigenvalue; gsig 1: n.sigma.n.
double stress_term(const double* s6, const V3& n, int gsig) {
  double T[9];
  voigt_to_tensor(s6, T);
  if (gsig == 1) {
    double r = 0;
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) r += n[i] * T[3 * i + j] * n[j];
    return r;
  }
  std::vector<double> A(T, T + 9);
  double w[3], vec[9];
  jacobi_eig(3, A, w, vec);
  double lmax = std::max(w[0], std::max(w[1], w[2]));
  double amax = std::max(std::fabs(w[0]), std::max(std::fabs(w[1]), std::fabs(w[2])));
  double gap = 1e-6 * amax;
  double p2 = 0.0;
  for (int i = 0; i < 3; ++i) {
    if (w[i] >= lmax - gap) {
      double c = vec[0 * 3 + i] * n[0] + vec[1 * 3 + i] * n[1] + vec[2 * 3 + i] * n[2];
      p2 += c * c;
    }
  }
  return lmax * std::sqrt(p2);
}

double ramp(const orc_ctx* c, double t) {
  if (c->ramp_t0 > 0.0 && t < c->ramp_t0) return t / c->ramp_t0;
  return 1.0;
}

int find_or_add_edge(orc_ctx* c, int a, int b) {
  std::pair<int, int> key(std::min(a, b), std::max(a, b));
  auto it = c->edge_of.find(key);
  if (it != c->edge_of.end()) return it->second;
  int id = (int)c->edge_nodes.size();
  c->edge_of[key] = id;
  c->edge_nodes.push_back(key);
  c->patch.push_back({});
  c->patch_q.push_back({});
  return id;
}

const int kEdgeLocal[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};
// hex node order: bottom face 0-1-2-3 counter-clockwise, top face 4-7 above
const int kHexEdge[12][2] = {{0, 1}, {1, 2}, {2, 3}, {3, 0}, {4, 5}, {5, 6},
                             {6, 7}, {7, 4}, {0, 4}, {1, 5}, {2, 6}, {3, 7}};
// reference corner signs of the local nodes (Eq. hex_strain_discretization)
const int kHexSign[8][3] = {{-1, -1, -1}, {1, -1, -1}, {1, 1, -1}, {-1, 1, -1},
                            {-1, -1, 1},  {1, -1, 1},  {1, 1, 1},  {-1, 1, 1}};

int elem_edges(const Elem& e, const int (**tab)[2]) {
  *tab = e.nn == 8 ? kHexEdge : kEdgeLocal;
  return e.nn == 8 ? 12 : 6;
}

void add_elem_to_edges(orc_ctx* c, int e) {
  const int(*tab)[2];
  int ne = elem_edges(c->el[e], &tab);
  for (int q = 0; q < ne; ++q) {
    int k = find_or_add_edge(c, c->el[e].n[tab[q][0]], c->el[e].n[tab[q][1]]);
    c->patch[k].push_back(e);
    c->patch_q[k].push_back(q);
  }
}

void remove_elem_from_edges(orc_ctx* c, int e) {
  for (int q = 0; q < 6; ++q) {
    int a = c->el[e].n[kEdgeLocal[q][0]], b = c->el[e].n[kEdgeLocal[q][1]];
    int k = c->edge_of.at(std::make_pair(std::min(a, b), std::max(a, b)));
    auto& p = c->patch[k];
    auto& pq = c->patch_q[k];
    size_t at = std::find(p.begin(), p.end(), e) - p.begin();
    p.erase(p.begin() + at);
    pq.erase(pq.begin() + at);
  }
}

// Lumped (row-sum) mass, Eq. mass_discretization: m_i = sum rho V_e / 4.
void rebuild_masses(orc_ctx* c) {
  c->m.assign(c->X.size(), 0.0);
  for (const Elem& e : c->el)
    for (int l = 0; l < e.nn; ++l) c->m[e.n[l]] += c->rho * e.Veff / e.nn;
}

// Acceleration of node i under the net force g: g / m_i.  A node that no
// element holds has no mass, no internal force and no load; it is given zero
// acceleration and so keeps its velocity.
double accel(const orc_ctx* c, size_t i, double g) { return c->m[i] > 0 ? g / c->m[i] : 0.0; }

// Smoothed strain and stress of every edge (Eqs. strain_discretization and
// CSTet_strain_discretization): eps_k = sum_j w_jk B_j u_j with
// w_jk = V_j / sum V over the elements sharing edge k; sigma_k = C eps_k.
// Elasticity matrix of element j: that of its parent tet's modulus.
void elem_cmat(const orc_ctx* c, int j, double C[6][6]) {
  double lam, mu;
  lame(c->Et[c->el[j].parent], c->nu, &lam, &mu);
  cmat(lam, mu, C);
}

// Smoothing-domain elasticity of edge k: C_k = sum_j w_jk C_j (the volume
// average over the domain; C_k = C for a single modulus).
void edge_cmat(const orc_ctx* c, int k, double S, double Ck[6][6]) {
  if (!c->hetero) {
    cmat(c->lam, c->mu, Ck);
    return;
  }
  for (int r = 0; r < 6; ++r)
    for (int q = 0; q < 6; ++q) Ck[r][q] = 0.0;
  for (int j : c->patch[k]) {
    double Cj[6][6];
    elem_cmat(c, j, Cj);
    double w = c->el[j].Veff / S;
    for (int r = 0; r < 6; ++r)
      for (int q = 0; q < 6; ++q) Ck[r][q] += w * Cj[r][q];
  }
}

void edge_fields(const orc_ctx* c, const std::vector<V3>& u, std::vector<std::array<double, 6>>& eps,
                 std::vector<std::array<double, 6>>& sig, std::vector<double>& Vsum) {
  // strain of each element at the point of each of its smoothing domains:
  // one per tet (constant gradients), one per local edge of a hex
  const int per = c->D == 12.0 ? 12 : 1;
  std::vector<std::array<double, 6>> eps_el(c->el.size() * per);
  par_range(c->nthreads, c->el.size(), [&](size_t j0, size_t j1) {
    for (size_t j = j0; j < j1; ++j) {
      double ue[24];
      const int nc = 3 * c->el[j].nn;
      for (int l = 0; l < c->el[j].nn; ++l)
        for (int d = 0; d < 3; ++d) ue[3 * l + d] = u[c->el[j].n[l]][d];
      for (int pq = 0; pq < per; ++pq) {
        double B[6][24];
        elem_bmat(c, (int)j, pq, B);
        for (int r = 0; r < 6; ++r) {
          double s = 0;
          for (int q = 0; q < nc; ++q) s += B[r][q] * ue[q];
          eps_el[per * j + pq][r] = s;
        }
      }
    }
  });
  size_t nE = c->edge_nodes.size();
  eps.assign(nE, {0, 0, 0, 0, 0, 0});
  sig.assign(nE, {0, 0, 0, 0, 0, 0});
  Vsum.assign(nE, 0.0);
  par_range(c->nthreads, nE, [&](size_t k0, size_t k1) {
    for (size_t k = k0; k < k1; ++k) {
      double S = 0;
      for (int j : c->patch[k]) S += c->el[j].Veff;
      Vsum[k] = S;
      if (S == 0.0) continue;  // every element on the edge removed: no stress
      for (size_t i = 0; i < c->patch[k].size(); ++i) {
        int j = c->patch[k][i];
        int q = per == 1 ? 0 : c->patch_q[k][i];
        double w = c->el[j].Veff / S;
        for (int r = 0; r < 6; ++r) eps[k][r] += w * eps_el[per * j + q][r];
      }
      double C[6][6];
      edge_cmat(c, (int)k, S, C);
      for (int r = 0; r < 6; ++r) {
        double s = 0;
        for (int q = 0; q < 6; ++q) s += C[r][q] * eps[k][q];
        sig[k][r] = s;
      }
    }
  });
}

// Internal force, Eqs. fint_discretization / CSTet_fint_discretization in the
// expanded form: f = sum_k V_k sum_{j in patch k} w_jk B_j^T sigma_k with
// V_k = (1/6) sum_j V_j.  Written as the edge loop it states.
void internal_force(const orc_ctx* c, const std::vector<V3>& u, std::vector<V3>& f) {
  std::vector<std::array<double, 6>> eps, sig;
  std::vector<double> Vsum;
  edge_fields(c, u, eps, sig, Vsum);
  f.assign(c->X.size(), {0, 0, 0});
  // each thread owns a range of nodes and runs the whole edge loop, adding
  // only to its own nodes: every nodal sum keeps the serial order
  par_range(c->nthreads, c->X.size(), [&](size_t n0, size_t n1) {
    auto own = [&](int i) { return (size_t)i >= n0 && (size_t)i < n1; };
    for (size_t k = 0; k < c->edge_nodes.size(); ++k) {
      double S = Vsum[k];
      if (S == 0.0) continue;
      double Vk = S / c->D;
      for (size_t i = 0; i < c->patch[k].size(); ++i) {
        int j = c->patch[k][i];
        const Elem& e = c->el[j];
        bool any = false;
        for (int l = 0; l < e.nn; ++l) any = any || own(e.n[l]);
        if (!any) continue;
        double w = e.Veff / S;
        double B[6][24];
        elem_bmat(c, j, c->patch_q[k][i], B);
        for (int q = 0; q < 3 * e.nn; ++q) {
          if (!own(e.n[q / 3])) continue;
          double s = 0;
          for (int r = 0; r < 6; ++r) s += B[r][q] * sig[k][r];
          f[e.n[q / 3]][q % 3] += Vk * w * s;
        }
      }
    }
  });
}

// Fraction of the parent volume carried by the copy holding the nodes of one
// side: midpoint cuts leave 1/8 on the side of a lone node, 7/8 on the side of
// three nodes and 1/2 each for a 2|2 partition.
double side_fraction(int nodes_on_side) {
  if (nodes_on_side == 1) return 0.125;
  if (nodes_on_side == 3) return 0.875;
  return 0.5;
}

// Area of the midpoint crack surface of a tet cut by `mask`: the Varignon
// parallelogram (2|2, Appendix I) or the corner triangle (1|3).
double crack_area(const V3 x[4], int mask) {
  int nb = popcount4(mask);
  if (nb == 2) {
    int A[2], Bn[2], ia = 0, ib = 0;
    for (int l = 0; l < 4; ++l) {
      if ((mask >> l) & 1) Bn[ib++] = l; else A[ia++] = l;
    }
    return 0.25 * norm(cross(sub(x[A[1]], x[A[0]]), sub(x[Bn[1]], x[Bn[0]])));
  }
  // the three nodes on the larger side span the face parallel to the cut
  int big = (nb == 1) ? 0 : 1;
  int q[3], iq = 0;
  for (int l = 0; l < 4; ++l)
    if ((((mask >> l) & 1) ? 1 : 0) == big) q[iq++] = l;
  return 0.125 * norm(cross(sub(x[q[1]], x[q[0]]), sub(x[q[2]], x[q[0]])));
}

// Split (or erode) original tet t with side mask `mask` (bit l: local node l
// on side B).  s_index is the global split counter (extra nodes N0+4s+l).
void apply_split(orc_ctx* c, int t, int mask) {
  c->smask[t] = mask;
  Elem& par = c->el[t];
  int nb = popcount4(mask);
  if (c->mode == 1) {  // erosion: the element no longer carries volume
    par.Veff = 0.0;
    return;
  }
  remove_elem_from_edges(c, t);
  int base = (int)c->X.size();
  Elem copyB = par;
  for (int l = 0; l < 4; ++l) {
    int real = par.n[l];
    int extra = base + l;
    c->X.push_back(c->X[real]);
    c->u.push_back(c->u[real]);
    c->v.push_back(c->v[real]);
    c->a.push_back(c->a[real]);
    c->F.push_back({0, 0, 0});
    bool onB = (mask >> l) & 1;
    if (onB) {
      c->el[t].n[l] = extra;  // copy A sees an extra node for a B-side node
    } else {
      copyB.n[l] = extra;     // copy B sees an extra node for an A-side node
    }
  }
  c->el[t].Veff = side_fraction(4 - nb) * c->el[t].V;
  copyB.Veff = side_fraction(nb) * copyB.V;
  c->el.push_back(copyB);
  add_elem_to_edges(c, t);
  add_elem_to_edges(c, (int)c->el.size() - 1);
}

// ---- hexahedral crack patterns III-VI (Section 3, parallelepiped element)

// Natural coordinate d of the midpoint of local hex edge q: -1, 0 or 1.
int hex_mid(int q, int d) { return (kHexSign[kHexEdge[q][0]][d] + kHexSign[kHexEdge[q][1]][d]) / 2; }

// The axis a hex edge runs along (the coordinate its midpoint has at 0).
int hex_edge_axis(int q) {
  for (int d = 0; d < 3; ++d)
    if (hex_mid(q, d) == 0) return d;
  return -1;
}

// The hex edge along `axis` whose midpoint has the two other coordinates
// given (by axis: want[d] for d != axis).
int hex_edge_at(int axis, const int want[3]) {
  for (int q = 0; q < 12; ++q) {
    if (hex_edge_axis(q) != axis) continue;
    bool ok = true;
    for (int d = 0; d < 3; ++d)
      if (d != axis && hex_mid(q, d) != want[d]) ok = false;
    if (ok) return q;
  }
  return -1;
}

// Crack plane c . xi = d of index p: 0-2 mid-planes (axis p), 3-14 wedge
// planes (axis pair (0,1), (0,2), (1,2); signs of the two coefficients, the
// first one slower), 15-22 corner planes (signs of c0, c1, c2, c0 slowest).
void hex_plane(int p, int c[3], int* d) {
  c[0] = c[1] = c[2] = 0;
  if (p < 3) {
    c[p] = 1;
    *d = 0;
  } else if (p < 15) {
    const int pr[3][2] = {{0, 1}, {0, 2}, {1, 2}};
    int k = (p - 3) / 4, r = (p - 3) % 4;
    c[pr[k][0]] = (r & 2) ? 1 : -1;
    c[pr[k][1]] = (r & 1) ? 1 : -1;
    *d = 1;
  } else {
    int r = p - 15;
    c[0] = (r & 4) ? 1 : -1;
    c[1] = (r & 2) ? 1 : -1;
    c[2] = (r & 1) ? 1 : -1;
    *d = 2;
  }
}

int hex_plane_index(const int c[3], int d) {
  if (d == 0) return c[0] ? 0 : c[1] ? 1 : 2;
  if (d == 1) {
    int a = c[0] ? 0 : 1, b = c[2] ? 2 : 1;
    int k = (a == 0 && b == 1) ? 0 : (a == 0 ? 1 : 2);
    return 3 + 4 * k + 2 * (c[a] > 0) + (c[b] > 0);
  }
  return 15 + 4 * (c[0] > 0) + 2 * (c[1] > 0) + (c[2] > 0);
}

// Cut edges of plane p: bit q set when the midpoint of edge q lies on it.
int hex_plane_mask(int p) {
  int c[3], d, m = 0;
  hex_plane(p, c, &d);
  for (int q = 0; q < 12; ++q)
    if (c[0] * hex_mid(q, 0) + c[1] * hex_mid(q, 1) + c[2] * hex_mid(q, 2) == d) m |= 1 << q;
  return m;
}

// Volume fraction a hex keeps after cracking with plane p: none after III
// (mid-plane), the triangular-prism half after IV, V and VI.
double hex_plane_fraction(int p) { return p < 3 ? 0.0 : 0.5; }

// Local face f = 2 axis + (side > 0): its four edges, as a bit mask.
int hex_face_mask(int f) {
  int axis = f / 2, side = (f & 1) ? 1 : -1, m = 0;
  for (int q = 0; q < 12; ++q)
    if (kHexSign[kHexEdge[q][0]][axis] == side && kHexSign[kHexEdge[q][1]][axis] == side) m |= 1 << q;
  return m;
}

// One candidate of a hex front: its plane, pattern (3-6) and the local
// edges of G1, G2 and G3, G4 (G-I quads) or G6 (G-II triangle, in G3).
struct HexCand {
  int plane, pattern, q1, q2, q3, q4;
};

// Candidates of the front on face f through the midpoints of local edges
// qa < qb, in tie order: III, IV toward -1, IV toward +1 (opposite edges);
// V, VI (neighbouring edges).
std::vector<HexCand> hex_candidates(int f, int qa, int qb) {
  std::vector<HexCand> out;
  const int k = f / 2, s = (f & 1) ? 1 : -1;
  const int i = hex_edge_axis(qa), j2 = hex_edge_axis(qb);
  if (i == j2) {  // opposite edges, both along axis i
    const int j = 3 - i - k;
    int w3[3] = {0, 0, 0}, w4[3] = {0, 0, 0};
    // III: the mid-plane xi_i = 0; G3, G4 on the i-edges of the opposite face
    w3[j] = hex_mid(qa, j); w3[k] = -s;
    w4[j] = hex_mid(qb, j); w4[k] = -s;
    out.push_back({i, 3, qa, qb, hex_edge_at(i, w3), hex_edge_at(i, w4)});
    // IV: sigma xi_i + s xi_k = 1; G3, G4 on the k-edges at xi_i = sigma
    for (int sg = -1; sg <= 1; sg += 2) {
      int c[3] = {0, 0, 0};
      c[i] = sg;
      c[k] = s;
      w3[i] = sg; w3[j] = hex_mid(qa, j);
      w4[i] = sg; w4[j] = hex_mid(qb, j);
      out.push_back({hex_plane_index(c, 1), 4, qa, qb, hex_edge_at(k, w3), hex_edge_at(k, w4)});
    }
  } else {  // neighbouring edges: qa along i at xi_j = p, qb along j at xi_i = r
    const int j = j2, p = hex_mid(qa, j), r = hex_mid(qb, i);
    int c[3] = {0, 0, 0};
    c[i] = r;
    c[j] = p;
    int w3[3] = {0, 0, 0}, w4[3] = {0, 0, 0};
    w3[j] = p; w3[k] = -s;
    w4[i] = r; w4[k] = -s;
    out.push_back({hex_plane_index(c, 1), 5, qa, qb, hex_edge_at(i, w3), hex_edge_at(j, w4)});
    c[k] = s;
    int w6[3] = {0, 0, 0};
    w6[i] = r; w6[j] = p;
    out.push_back({hex_plane_index(c, 2), 6, qa, qb, hex_edge_at(k, w6), -1});
  }
  return out;
}

// Reference midpoint of local edge q of hex t.
V3 hex_edge_point_x(const orc_ctx* c, int t, int q) {
  const V3& a = c->X[c->el[t].n[kHexEdge[q][0]]];
  const V3& b = c->X[c->el[t].n[kHexEdge[q][1]]];
  return {0.5 * (a[0] + b[0]), 0.5 * (a[1] + b[1]), 0.5 * (a[2] + b[2])};
}

int hex_global_edge(const orc_ctx* c, int t, int q) {
  int a = c->el[t].n[kHexEdge[q][0]], b = c->el[t].n[kHexEdge[q][1]];
  return c->edge_of.at(std::make_pair(std::min(a, b), std::max(a, b)));
}

// Eq. stretch-delta on local edge q of hex t: its end-to-end displacement
// difference if the edge lengthens, else 0.
V3 hex_stretch(const orc_ctx* c, const std::vector<V3>& u, int t, int q) {
  int a = c->el[t].n[kHexEdge[q][0]], b = c->el[t].n[kHexEdge[q][1]];
  V3 du = sub(u[b], u[a]);
  V3 dX = sub(c->X[b], c->X[a]);
  if (2.0 * dot(dX, du) + dot(du, du) > 0.0) return du;
  return {0, 0, 0};
}

// Crack normal and surface area of candidate k of hex t: the quad G1 G2 G4 G3
// (normal of its diagonals G1G4 and G2G3, area half their cross product) or
// the triangle G1 G2 G6.
void hex_cand_geometry(const orc_ctx* c, int t, const HexCand& k, V3* n, double* area) {
  V3 P1 = hex_edge_point_x(c, t, k.q1), P2 = hex_edge_point_x(c, t, k.q2);
  V3 P3 = hex_edge_point_x(c, t, k.q3);
  V3 nn;
  if (k.pattern == 6) {
    nn = cross(sub(P2, P1), sub(P3, P1));
  } else {
    V3 P4 = hex_edge_point_x(c, t, k.q4);
    nn = cross(sub(P4, P1), sub(P3, P2));
  }
  double l = norm(nn);
  *area = 0.5 * l;
  *n = {nn[0] / l, nn[1] / l, nn[2] / l};
}

// Release rate of candidate k of hex t (Eq. G-I for III, IV, V; Eq. G-II for VI).
double hex_cand_G(const orc_ctx* c, const std::vector<V3>& u,
                  const std::vector<std::array<double, 6>>& sig, int t, const HexCand& k) {
  V3 n;
  double area;
  hex_cand_geometry(c, t, k, &n, &area);
  V3 d1 = hex_stretch(c, u, t, k.q1), d2 = hex_stretch(c, u, t, k.q2);
  double a1 = std::fabs(dot(d1, n)), a2 = std::fabs(dot(d2, n));
  double s3 = stress_term(sig[hex_global_edge(c, t, k.q3)].data(), n, c->gsig);
  if (k.pattern == 6) return 0.5 * s3 * (a1 + a2);
  double s4 = stress_term(sig[hex_global_edge(c, t, k.q4)].data(), n, c->gsig);
  return 0.5 * (s3 * a1 + s4 * a2);
}

// Fronts of a hex mesh: per face of a cracked hex cut at two edges, the intact
// hex across it, its local face and its two local edges (qa * 16 + qb,
// qa < qb, in `lone`).  Sorted by (hex, face).
std::vector<FrontRec> hex_fronts(const orc_ctx* c) {
  std::vector<FrontRec> fr;
  for (int s = 0; s < c->T0; ++s) {
    if (c->smask[s] < 0) continue;
    const int cut = hex_plane_mask(c->smask[s]);
    for (int f = 0; f < 6; ++f) {
      int on = cut & hex_face_mask(f);
      if (__builtin_popcount(on) != 2) continue;
      int nb = c->hnbr[s][f];
      if (nb < 0 || c->smask[nb] >= 0) continue;
      int qs[2], k = 0;
      for (int q = 0; q < 12; ++q)
        if ((on >> q) & 1) qs[k++] = q;
      int ql[2];
      for (int r = 0; r < 2; ++r) {
        int g = hex_global_edge(c, s, qs[r]);
        ql[r] = -1;
        for (int q = 0; q < 12; ++q)
          if (hex_global_edge(c, nb, q) == g) ql[r] = q;
      }
      FrontRec r;
      r.c = nb;
      r.face = c->hnbr_face[s][f];
      r.lone = std::min(ql[0], ql[1]) * 16 + std::max(ql[0], ql[1]);
      r.GI = r.GII = 0;
      fr.push_back(r);
    }
  }
  std::sort(fr.begin(), fr.end(), [](const FrontRec& x, const FrontRec& y) {
    return x.c != y.c ? x.c < y.c : x.face < y.face;
  });
  return fr;
}

// Area of the crack surface of plane p in hex t: the triangle of its three
// cut-edge midpoints, or the quad of four, whose diagonals join the
// midpoints farthest apart in natural coordinates.
double hex_plane_area(const orc_ctx* c, int t, int p) {
  int qs[4], n = 0;
  const int cut = hex_plane_mask(p);
  for (int q = 0; q < 12; ++q)
    if ((cut >> q) & 1) qs[n++] = q;
  V3 P[4];
  for (int r = 0; r < n; ++r) P[r] = hex_edge_point_x(c, t, qs[r]);
  if (n == 3) return 0.5 * norm(cross(sub(P[1], P[0]), sub(P[2], P[0])));
  int far = 1, best = -1;
  for (int r = 1; r < 4; ++r) {
    int d2 = 0;
    for (int d = 0; d < 3; ++d) {
      int x = hex_mid(qs[r], d) - hex_mid(qs[0], d);
      d2 += x * x;
    }
    if (d2 > best) { best = d2; far = r; }
  }
  int o[2], k = 0;
  for (int r = 1; r < 4; ++r)
    if (r != far) o[k++] = r;
  return 0.5 * norm(cross(sub(P[far], P[0]), sub(P[o[1]], P[o[0]])));
}

// Crack hex t with plane p: it carries the volume fraction the plane leaves.
void apply_hex_crack(orc_ctx* c, int t, int p) {
  c->smask[t] = p;
  c->el[t].Veff = hex_plane_fraction(p) * c->el[t].V;
}

// Crack front list (Section 3): faces of intact tets shared with a split tet
// whose partition cuts that face.  Each record names the intact tet c, its
// local face (opposite local node `face`) and the real node of the face that
// lies alone on its side of the cut (N2).  Sorted by (c, face).
std::vector<FrontRec> fronts(const orc_ctx* c) {
  if (c->D == 12.0) return hex_fronts(c);
  std::vector<FrontRec> fr;
  for (int s = 0; s < c->T0; ++s) {
    int m = c->smask[s];
    if (m < 0) continue;
    for (int f = 0; f < 4; ++f) {
      int nbt = c->nbr[s][f];
      if (nbt < 0 || c->smask[nbt] >= 0) continue;
      int fl[3], k = 0;
      for (int l = 0; l < 4; ++l)
        if (l != f) fl[k++] = l;
      int b0 = (m >> fl[0]) & 1, b1 = (m >> fl[1]) & 1, b2 = (m >> fl[2]) & 1;
      if (b0 == b1 && b1 == b2) continue;  // face not cut
      int lone = (b1 == b2) ? fl[0] : (b0 == b2) ? fl[1] : fl[2];
      FrontRec r;
      r.c = nbt;
      r.face = c->nbr_face[s][f];
      r.lone = c->orig[s][lone];
      r.GI = r.GII = 0;
      fr.push_back(r);
    }
  }
  std::sort(fr.begin(), fr.end(), [](const FrontRec& x, const FrontRec& y) {
    return x.c != y.c ? x.c < y.c : x.face < y.face;
  });
  return fr;
}

// Release rates of one front (Eqs. stretch-delta, G-I, G-II).  Candidate tet
// c, its face `face` (opposite local node `face`) lies on the crack front;
// `lone` is the node of that face alone on its side (N2).
void front_G(const orc_ctx* c, const std::vector<V3>& u, const std::vector<std::array<double, 6>>& sig,
             const FrontRec& fr, double* GI, double* GII, int* maskI, int* maskII) {
  const auto& tn = c->orig[fr.c];
  int lN2 = -1, lN4 = fr.face, lN1 = -1, lN3 = -1;
  for (int l = 0; l < 4; ++l) {
    if (l == fr.face) continue;
    if (tn[l] == fr.lone) lN2 = l;
    else if (lN1 < 0) lN1 = l;
    else lN3 = l;
  }
  int N1 = tn[lN1], N2 = tn[lN2], N3 = tn[lN3], N4 = tn[lN4];
  const V3 &X1 = c->X[N1], &X2 = c->X[N2], &X3 = c->X[N3], &X4 = c->X[N4];
  auto stretch = [&](int i, int j) -> V3 {
    V3 du = sub(u[j], u[i]);
    V3 dX = sub(c->X[j], c->X[i]);
    double d = 2.0 * dot(dX, du) + dot(du, du);
    if (d > 0.0) return du;
    return {0, 0, 0};
  };
  V3 d1 = stretch(N1, N2), d2 = stretch(N2, N3);
  auto unit = [](V3 x) {
    double l = norm(x);
    return V3{x[0] / l, x[1] / l, x[2] / l};
  };
  V3 nI = unit(cross(sub(X3, X1), sub(X4, X2)));
  V3 nII = unit(cross(sub(X3, X1), sub(X4, X1)));
  auto edge = [&](int a, int b) { return c->edge_of.at(std::make_pair(std::min(a, b), std::max(a, b))); };
  double s3 = stress_term(sig[edge(N1, N4)].data(), nI, c->gsig);
  double s4 = stress_term(sig[edge(N3, N4)].data(), nI, c->gsig);
  double s6 = stress_term(sig[edge(N2, N4)].data(), nII, c->gsig);
  *GI = 0.5 * (s3 * std::fabs(dot(d1, nI)) + s4 * std::fabs(dot(d2, nI)));
  *GII = 0.5 * s6 * (std::fabs(dot(d1, nII)) + std::fabs(dot(d2, nII)));
  *maskI = (1 << lN2) | (1 << lN4);
  *maskII = (1 << lN2);
}

// Prescribed-velocity history with ramp time t0: the velocity factor
// r_v(t) = t / t0 up to t0, then 1 (t0 = 0: 1 from the start), its integral S
// and its derivative.
double bc_vel(double t0, double t) { return (t0 > 0 && t <= t0) ? t / t0 : 1.0; }
double bc_disp(double t0, double t) {
  if (t0 > 0 && t <= t0) return t * t / (2.0 * t0);
  return t0 > 0 ? t - 0.5 * t0 : t;
}
double bc_acc(double t0, double t) { return (t0 > 0 && t <= t0) ? 1.0 / t0 : 0.0; }

// Constrained components of u (if set_u), v and a at time t.
void apply_bc(orc_ctx* c, double t, std::vector<V3>& u, bool set_u) {
  for (size_t b = 0; b < c->bc_node.size(); ++b) {
    int i = c->bc_node[b];
    double t0 = c->grp_t0[c->bc_group[b]];
    for (int d = 0; d < 3; ++d) {
      if (!((c->bc_mask[b] >> d) & 1)) continue;
      if (set_u) u[i][d] = c->bc_uref[b][d] + c->bc_v0[b][d] * bc_disp(t0, t);
      c->v[i][d] = c->bc_v0[b][d] * bc_vel(t0, t);
      c->a[i][d] = c->bc_v0[b][d] * bc_acc(t0, t);
    }
  }
}

// Support reaction on the constrained components: m a + f_int - r F.
void bc_reactions(orc_ctx* c, const std::vector<V3>& f, double r, std::vector<V3>& R) {
  R.assign(c->bc_node.size(), {0, 0, 0});
  for (size_t b = 0; b < c->bc_node.size(); ++b) {
    int i = c->bc_node[b];
    for (int d = 0; d < 3; ++d)
      if ((c->bc_mask[b] >> d) & 1) R[b][d] = c->m[i] * c->a[i][d] + f[i][d] - r * c->F[i][d];
  }
}

int initialize(orc_ctx* c) {
  double t = c->step * c->dt;
  apply_bc(c, t, c->u, true);
  std::vector<V3> f;
  internal_force(c, c->u, f);
  double r = ramp(c, t);
  for (size_t i = 0; i < c->X.size(); ++i)
    for (int d = 0; d < 3; ++d) c->a[i][d] = accel(c, i, r * c->F[i][d] - f[i][d]);
  apply_bc(c, t, c->u, false);
  bc_reactions(c, f, r, c->bc_R);
  c->need_init = false;
  return 0;
}

// Decide the splits of this step on the current state (Section 3; Griffith
// test of Section 2.1).  Returns (tet, mask, pattern, G) sorted by tet.
std::vector<Event> decide_splits(orc_ctx* c) {
  std::vector<Event> out;
  std::vector<std::array<double, 6>> eps, sig;
  std::vector<double> Vsum;
  edge_fields(c, c->u, eps, sig, Vsum);
  std::vector<FrontRec> fr = fronts(c);
  c->nfront = (int)fr.size();
  c->Gmax = 0.0;
  bool any = false;
  size_t i = 0;
  while (i < fr.size()) {
    size_t j = i;
    double best = -INFINITY;
    int bmask = 0, bpat = 0;
    for (; j < fr.size() && fr[j].c == fr[i].c; ++j) {
      if (c->D == 12.0) {  // hex: candidates III-VI of this face, in tie order
        for (const HexCand& k : hex_candidates(fr[j].face, fr[j].lone / 16, fr[j].lone % 16)) {
          double G = hex_cand_G(c, c->u, sig, fr[j].c, k);
          if (G > best) { best = G; bmask = k.plane; bpat = k.pattern; }
        }
        continue;
      }
      double GI, GII;
      int mI, mII;
      front_G(c, c->u, sig, fr[j], &GI, &GII, &mI, &mII);
      if (GI > best) { best = GI; bmask = mI; bpat = 1; }
      if (GII > best) { best = GII; bmask = mII; bpat = 2; }
    }
    if (!any || best > c->Gmax) c->Gmax = best;
    any = true;
    if (best >= c->Gc) out.push_back({0, fr[i].c, bmask, bpat, best});
    i = j;
  }
  if (!any) c->Gmax = 0.0;
  return out;
}

// Apply the splits decided in a step.  Each opens a crack surface and so
// dissipates Gc times its area (pre-splits, applied by orc_presplit, do not).
void apply_events(orc_ctx* c, const std::vector<Event>& evs) {
  const auto& on = c->orig;
  for (const Event& e : evs) {
    if (c->D == 12.0) {
      c->Ud += c->Gc * hex_plane_area(c, e.tet, e.mask);
      apply_hex_crack(c, e.tet, e.mask);
      c->events.push_back(e);
      c->events.back().step = (int)c->step;
      c->nsplit++;
      continue;
    }
    V3 x[4];
    for (int l = 0; l < 4; ++l) x[l] = c->X[on[e.tet][l]];
    c->Ud += c->Gc * crack_area(x, e.mask);
    apply_split(c, e.tet, e.mask);
    c->events.push_back(e);
    c->events.back().step = (int)c->step;
    c->nsplit++;
  }
  if (!evs.empty() && c->mode == 0 && c->D == 6.0) rebuild_masses(c);
}

// One explicit Newmark step (beta = 0, gamma = 1/2), then the crack pass.
void one_step(orc_ctx* c) {
  if (c->need_init) initialize(c);
  double dt = c->dt;
  double tn = c->step * dt, tn1 = (c->step + 1) * dt;
  double rn = ramp(c, tn), rn1 = ramp(c, tn1);
  size_t N = c->X.size();
  std::vector<V3> u1(N);
  for (size_t i = 0; i < N; ++i)
    for (int d = 0; d < 3; ++d)
      u1[i][d] = c->u[i][d] + dt * c->v[i][d] + 0.5 * dt * dt * c->a[i][d];
  // prescribed components follow their history exactly
  for (size_t b = 0; b < c->bc_node.size(); ++b)
    for (int d = 0; d < 3; ++d)
      if ((c->bc_mask[b] >> d) & 1)
        u1[c->bc_node[b]][d] =
            c->bc_uref[b][d] + c->bc_v0[b][d] * bc_disp(c->grp_t0[c->bc_group[b]], tn1);
  std::vector<V3> f;
  internal_force(c, u1, f);
  std::vector<V3> u0 = c->u;
  for (size_t i = 0; i < N; ++i)
    for (int d = 0; d < 3; ++d) c->W += 0.5 * (rn + rn1) * c->F[i][d] * (u1[i][d] - c->u[i][d]);
  par_range(c->nthreads, N, [&](size_t i0, size_t i1) {
    for (size_t i = i0; i < i1; ++i) {
      for (int d = 0; d < 3; ++d) {
        double an1 = accel(c, i, rn1 * c->F[i][d] - f[i][d]);
        c->v[i][d] = c->v[i][d] + 0.5 * dt * (c->a[i][d] + an1);
        c->a[i][d] = an1;
        c->u[i][d] = u1[i][d];
      }
    }
  });
  if (!c->grp_t0.empty()) {
    apply_bc(c, tn1, c->u, false);
    std::vector<V3> R;
    bc_reactions(c, f, rn1, R);
    size_t G = c->grp_t0.size();
    std::vector<std::array<double, 6>> rows(G);
    for (size_t g = 0; g < G; ++g) rows[g] = {(double)(c->step + 1), tn1, 0, 0, 0, bc_disp(c->grp_t0[g], tn1)};
    for (size_t b = 0; b < R.size(); ++b) {
      int i = c->bc_node[b], g = c->bc_group[b];
      for (int d = 0; d < 3; ++d) {
        c->grp_W[g] += 0.5 * (c->bc_R[b][d] + R[b][d]) * (c->u[i][d] - u0[i][d]);
        rows[g][2 + d] += R[b][d];
      }
    }
    c->bc_R = R;
    for (size_t g = 0; g < G; ++g) c->grp_hist[g].push_back(rows[g]);
  }
  c->step += 1;
  std::vector<Event> evs;
  if (c->replay) {
    // forced schedule: splits listed for this step, G test not used
    std::vector<Event> tmp = decide_splits(c);  // keeps Gmax / n_front readbacks
    (void)tmp;
    while (c->cursor < c->schedule.size() && c->schedule[c->cursor].step < c->step) c->cursor++;
    while (c->cursor < c->schedule.size() && c->schedule[c->cursor].step == c->step) {
      Event e = c->schedule[c->cursor++];
      if (c->smask[e.tet] >= 0) continue;
      e.pattern = popcount4(e.mask) == 2 ? 1 : 2;
      e.G = 0.0;
      evs.push_back(e);
    }
  } else if (c->frozen) {
    // fixed-topology window: no crack pass
  } else if (c->Gc < INFINITY) {
    evs = decide_splits(c);
  } else {
    c->nfront = (int)fronts(c).size();
  }
  apply_events(c, evs);
}

double strain_energy(const orc_ctx* c) {
  std::vector<std::array<double, 6>> eps, sig;
  std::vector<double> Vsum;
  edge_fields(c, c->u, eps, sig, Vsum);
  double se = 0;
  for (size_t k = 0; k < eps.size(); ++k) {
    double s = 0;
    for (int r = 0; r < 6; ++r) s += sig[k][r] * eps[k][r];
    se += 0.5 * (Vsum[k] / c->D) * s;
  }
  return se;
}

// lambda^T (dK/dE_j) u for every original tet j, times `scale`, added to
// out[j].  With C_k = sum_j w_jk C_j and C_j = E_j Chat (Chat: the matrix at
// unit modulus), dK/dE_j = sum_{k : j in patch k} V_k w_jk Bt_k^T Chat Bt_k,
// so the term is sum_k V_k w_jk eps_k(lambda) . Chat eps_k(u) with eps_k the
// smoothed strain of edge k.  Split copies add to their parent tet.
void modulus_term(const orc_ctx* c, const std::vector<V3>& lam, const std::vector<V3>& u, double scale,
                  std::vector<double>& out) {
  std::vector<std::array<double, 6>> el, sl, eu, su;
  std::vector<double> Vs;
  edge_fields(c, lam, el, sl, Vs);
  edge_fields(c, u, eu, su, Vs);
  double lh, mh, Ch[6][6];
  lame(1.0, c->nu, &lh, &mh);
  cmat(lh, mh, Ch);
  for (size_t k = 0; k < Vs.size(); ++k) {
    double S = Vs[k];
    if (S == 0.0) continue;
    double q = 0;
    for (int r = 0; r < 6; ++r)
      for (int p = 0; p < 6; ++p) q += el[k][r] * Ch[r][p] * eu[k][p];
    double Vk = S / c->D;
    for (int j : c->patch[k]) out[c->el[j].parent] += scale * Vk * (c->el[j].Veff / S) * q;
  }
}

// Sensitivity of J = gu . u_N + gv . v_N to the modulus of every tet and to
// the initial state, over n steps of fixed topology taken from the current
// state.  The forward step (Newmark beta = 0, gamma = 1/2, end of
// Section 2.2) is
//   u_{n+1} = u_n + dt v_n + dt^2/2 a_n,
//   a_{n+1} = M^-1 (r_{n+1} F - K u_{n+1}),
//   v_{n+1} = v_n + dt/2 (a_n + a_{n+1}),
// with a_0 = M^-1 (r_0 F - K u_0).  Reversing these three assignments with
// sensitivities ub, vb, ab (K is symmetric, M diagonal) gives per step
//   ab_{n+1} += dt/2 vb_{n+1};  lambda = M^-1 ab_{n+1};
//   ub_{n+1} -= K lambda;  Eb_j -= lambda^T dK/dE_j u_{n+1};
//   ub_n += ub_{n+1};  vb_n += vb_{n+1} + dt ub_{n+1};
//   ab_n += dt/2 vb_{n+1} + dt^2/2 ub_{n+1},
// and a_0 takes the treatment of a_{n+1} once more at the end.
int window_gradient(orc_ctx* c, int n, const double* gu, const double* gv, double* gu0, double* gv0,
                    double* gE) {
  if (c->need_init) initialize(c);
  bool was = c->frozen;
  c->frozen = true;
  std::vector<std::vector<V3>> us;
  us.push_back(c->u);
  for (int s = 0; s < n; ++s) {
    one_step(c);
    us.push_back(c->u);
  }
  c->frozen = was;
  size_t N = c->X.size();
  const double dt = c->dt;
  std::vector<V3> ub(N), vb(N), ab(N, V3{0, 0, 0}), lam(N), f;
  for (size_t i = 0; i < N; ++i)
    for (int d = 0; d < 3; ++d) {
      ub[i][d] = gu ? gu[3 * i + d] : 0.0;
      vb[i][d] = gv ? gv[3 * i + d] : 0.0;
    }
  std::vector<double> Eb(c->T0, 0.0);
  auto invm = [&](size_t i) { return c->m[i] > 0 ? 1.0 / c->m[i] : 0.0; };
  for (int s = n - 1; s >= -1; --s) {
    // the acceleration of index s + 1 (s = -1: a_0 of the initial state)
    for (size_t i = 0; i < N; ++i)
      for (int d = 0; d < 3; ++d) {
        if (s >= 0) ab[i][d] += 0.5 * dt * vb[i][d];
        lam[i][d] = invm(i) * ab[i][d];
      }
    internal_force(c, lam, f);
    for (size_t i = 0; i < N; ++i)
      for (int d = 0; d < 3; ++d) ub[i][d] -= f[i][d];
    modulus_term(c, lam, us[s + 1], -1.0, Eb);
    if (s < 0) break;
    for (size_t i = 0; i < N; ++i)
      for (int d = 0; d < 3; ++d) {
        double u1 = ub[i][d], v1 = vb[i][d];
        vb[i][d] = v1 + dt * u1;
        ab[i][d] = 0.5 * dt * v1 + 0.5 * dt * dt * u1;
        // ub_n = ub_{n+1}: unchanged
      }
  }
  for (size_t i = 0; i < N; ++i)
    for (int d = 0; d < 3; ++d) {
      if (gu0) gu0[3 * i + d] = ub[i][d];
      if (gv0) gv0[3 * i + d] = vb[i][d];
    }
  if (gE)
    for (int t = 0; t < c->T0; ++t) gE[t] = Eb[t];
  return 0;
}


// grad N_i = J^{-T} grad_xi N_i of the eight shape functions at the natural
// point xi (J[r][c] = dx_r / dxi_c); returns det J.
double hex_point_gradients(const V3 x[8], const double xi[3], double g[8][3]) {
  const int(*sg)[3] = kHexSign;
  double dN[8][3];  // dN_i / d(xi, eta, zeta)
  for (int i = 0; i < 8; ++i) {
    double f[3];
    for (int d = 0; d < 3; ++d) f[d] = 1.0 + xi[d] * sg[i][d];
    dN[i][0] = sg[i][0] * f[1] * f[2] / 8.0;
    dN[i][1] = f[0] * sg[i][1] * f[2] / 8.0;
    dN[i][2] = f[0] * f[1] * sg[i][2] / 8.0;
  }
  double J[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  for (int i = 0; i < 8; ++i)
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) J[r][c] += x[i][r] * dN[i][c];
  double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
               J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
               J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
  double inv[3][3];  // J^{-1}
  inv[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) / det;
  inv[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
  inv[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
  inv[1][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) / det;
  inv[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
  inv[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
  inv[2][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) / det;
  inv[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
  inv[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
  for (int i = 0; i < 8; ++i)
    for (int d = 0; d < 3; ++d) {
      double s = 0;
      for (int c = 0; c < 3; ++c) s += inv[c][d] * dN[i][c];
      g[i][d] = s;
    }
  return det;
}

// Volume (2 x 2 x 2 Gauss points, exact for the trilinear map), the
// smallest Jacobian determinant over the Gauss and edge points, and the
// gradients at the midpoint of each local edge q (ge[(q * 8 + i) * 3 + d]).
double hex_geometry(const V3 x[8], double* ge, double* min_det) {
  const int(*sg)[3] = kHexSign;
  const double a = 1.0 / std::sqrt(3.0);
  double V = 0, g[8][3];
  *min_det = INFINITY;
  for (int p = 0; p < 8; ++p) {
    double xi[3] = {sg[p][0] * a, sg[p][1] * a, sg[p][2] * a};
    double det = hex_point_gradients(x, xi, g);
    *min_det = std::min(*min_det, det);
    V += det;  // Gauss weights 1
  }
  for (int q = 0; q < 12; ++q) {
    int p0 = kHexEdge[q][0], p1 = kHexEdge[q][1];
    double xi[3];
    for (int d = 0; d < 3; ++d) xi[d] = 0.5 * (sg[p0][d] + sg[p1][d]);
    double det = hex_point_gradients(x, xi, g);
    *min_det = std::min(*min_det, det);
    for (int i = 0; i < 8; ++i)
      for (int d = 0; d < 3; ++d) ge[(q * 8 + i) * 3 + d] = g[i][d];
  }
  return V;
}

}  // namespace

extern "C" {

void orc_lame(double E, double nu, double* lam, double* mu) { lame(E, nu, lam, mu); }

orc_ctx* orc_create(int n_nodes, const double* X, int n_tets, const int* tets, double E, double nu,
                    double rho, double Gc, int split_mode, int gsig) {
  orc_ctx* c = new orc_ctx();
  c->E = E; c->nu = nu; c->rho = rho; c->Gc = Gc;
  c->mode = split_mode; c->gsig = gsig;
  lame(E, nu, &c->lam, &c->mu);
  c->N0 = n_nodes;
  c->T0 = n_tets;
  c->X.resize(n_nodes);
  for (int i = 0; i < n_nodes; ++i) c->X[i] = {X[3 * i], X[3 * i + 1], X[3 * i + 2]};
  // mean edge length for the degeneracy test
  double lsum = 0;
  long lcnt = 0;
  for (int t = 0; t < n_tets; ++t)
    for (int q = 0; q < 6; ++q) {
      int a = tets[4 * t + kEdgeLocal[q][0]], b = tets[4 * t + kEdgeLocal[q][1]];
      if (a < 0 || a >= n_nodes || b < 0 || b >= n_nodes) {
        c->status = -5;
        c->err = "node id out of range";
        return c;
      }
      lsum += norm(sub(c->X[a], c->X[b]));
      lcnt++;
    }
  double lmean = lcnt ? lsum / lcnt : 0;
  std::vector<std::array<int, 4>> orig(n_tets);
  c->el.resize(n_tets);
  for (int t = 0; t < n_tets; ++t) {
    Elem& e = c->el[t];
    for (int l = 0; l < 4; ++l) e.n[l] = tets[4 * t + l];
    V3 x[4];
    for (int l = 0; l < 4; ++l) x[l] = c->X[e.n[l]];
    double V = tet_geometry(x, e.g);
    if (V < 0) {  // orient: swap local nodes 2 and 3
      std::swap(e.n[2], e.n[3]);
      for (int l = 0; l < 4; ++l) x[l] = c->X[e.n[l]];
      V = tet_geometry(x, e.g);
    }
    if (!(std::fabs(V) > 1e-12 * lmean * lmean * lmean)) {
      c->status = -5;
      c->err = "degenerate tetrahedron " + std::to_string(t);
      return c;
    }
    e.V = V;
    e.Veff = V;
    e.parent = t;
    for (int l = 0; l < 4; ++l) orig[t][l] = e.n[l];
  }
  c->orig = orig;
  for (int t = 0; t < n_tets; ++t) add_elem_to_edges(c, t);
  // face adjacency of the original mesh
  c->nbr.assign(n_tets, {-1, -1, -1, -1});
  c->nbr_face.assign(n_tets, {-1, -1, -1, -1});
  std::map<std::array<int, 3>, std::vector<std::pair<int, int>>> faces;
  for (int t = 0; t < n_tets; ++t)
    for (int f = 0; f < 4; ++f) {
      std::array<int, 3> k;
      int q = 0;
      for (int l = 0; l < 4; ++l)
        if (l != f) k[q++] = orig[t][l];
      std::sort(k.begin(), k.end());
      faces[k].push_back({t, f});
    }
  for (auto& kv : faces) {
    if (kv.second.size() > 2) {
      c->status = -5;
      c->err = "face shared by more than two tetrahedra";
      return c;
    }
    if (kv.second.size() == 2) {
      auto p = kv.second[0], q = kv.second[1];
      c->nbr[p.first][p.second] = q.first;
      c->nbr_face[p.first][p.second] = q.second;
      c->nbr[q.first][q.second] = p.first;
      c->nbr_face[q.first][q.second] = p.second;
    }
  }
  c->smask.assign(n_tets, -1);
  c->Et.assign(n_tets, E);
  c->u.assign(n_nodes, {0, 0, 0});
  c->v.assign(n_nodes, {0, 0, 0});
  c->a.assign(n_nodes, {0, 0, 0});
  c->F.assign(n_nodes, {0, 0, 0});
  rebuild_masses(c);
  return c;
}

// Trilinear hexahedral mesh (node order: bottom face 0-1-2-3 counter-clockwise
// seen from above, top face 4-7 above them).  A hex with negative Jacobian
// determinants throughout is mirrored (local nodes 1 <-> 3, 5 <-> 7); one
// with mixed signs is rejected.  Cracks start from precracked hexes
// (orc_presplit with crack plane indices).
orc_ctx* orc_create_hex(int n_nodes, const double* X, int n_hex, const int* hex, double E, double nu,
                        double rho, double Gc, int gsig) {
  orc_ctx* c = new orc_ctx();
  c->E = E; c->nu = nu; c->rho = rho; c->Gc = Gc;
  c->gsig = gsig;
  c->D = 12.0;
  lame(E, nu, &c->lam, &c->mu);
  c->N0 = n_nodes;
  c->T0 = n_hex;
  c->X.resize(n_nodes);
  for (int i = 0; i < n_nodes; ++i) c->X[i] = {X[3 * i], X[3 * i + 1], X[3 * i + 2]};
  c->el.resize(n_hex);
  c->hexg.resize(n_hex);
  for (int t = 0; t < n_hex; ++t) {
    Elem& e = c->el[t];
    e.nn = 8;
    for (int l = 0; l < 8; ++l)
      for (int d = 0; d < 3; ++d) e.g[l][d] = 0.0;  // hexes use their edge-point gradients
    for (int l = 0; l < 8; ++l) {
      e.n[l] = hex[8 * t + l];
      if (e.n[l] < 0 || e.n[l] >= n_nodes) {
        c->status = -5;
        c->err = "node id out of range";
        return c;
      }
    }
    V3 x[8];
    for (int l = 0; l < 8; ++l) x[l] = c->X[e.n[l]];
    double mind;
    double V = hex_geometry(x, c->hexg[t].data(), &mind);
    if (V < 0) {
      std::swap(e.n[1], e.n[3]);
      std::swap(e.n[5], e.n[7]);
      for (int l = 0; l < 8; ++l) x[l] = c->X[e.n[l]];
      V = hex_geometry(x, c->hexg[t].data(), &mind);
    }
    if (!(mind > 0)) {
      c->status = -5;
      c->err = "degenerate or inverted hexahedron " + std::to_string(t);
      return c;
    }
    e.V = V;
    e.Veff = V;
    e.parent = t;
  }
  for (int t = 0; t < n_hex; ++t) add_elem_to_edges(c, t);
  c->orig.assign(n_hex, {0, 0, 0, 0});
  c->nbr.assign(n_hex, {-1, -1, -1, -1});
  c->nbr_face.assign(n_hex, {-1, -1, -1, -1});
  // face adjacency (local face f = 2 axis + (side > 0))
  c->hnbr.assign(n_hex, {-1, -1, -1, -1, -1, -1});
  c->hnbr_face.assign(n_hex, {-1, -1, -1, -1, -1, -1});
  std::map<std::array<int, 4>, std::vector<std::pair<int, int>>> faces;
  for (int t = 0; t < n_hex; ++t)
    for (int f = 0; f < 6; ++f) {
      std::array<int, 4> k;
      int q = 0;
      for (int l = 0; l < 8; ++l)
        if (kHexSign[l][f / 2] == ((f & 1) ? 1 : -1)) k[q++] = c->el[t].n[l];
      std::sort(k.begin(), k.end());
      faces[k].push_back({t, f});
    }
  for (auto& kv : faces) {
    if (kv.second.size() > 2) {
      c->status = -5;
      c->err = "face shared by more than two hexahedra";
      return c;
    }
    if (kv.second.size() == 2) {
      auto p = kv.second[0], q = kv.second[1];
      c->hnbr[p.first][p.second] = q.first;
      c->hnbr_face[p.first][p.second] = q.second;
      c->hnbr[q.first][q.second] = p.first;
      c->hnbr_face[q.first][q.second] = p.second;
    }
  }
  c->smask.assign(n_hex, -1);
  c->Et.assign(n_hex, E);
  c->u.assign(n_nodes, {0, 0, 0});
  c->v.assign(n_nodes, {0, 0, 0});
  c->a.assign(n_nodes, {0, 0, 0});
  c->F.assign(n_nodes, {0, 0, 0});
  rebuild_masses(c);
  return c;
}

int orc_create_status(const orc_ctx* c) { return c->status; }
const char* orc_error(const orc_ctx* c) { return c->err.c_str(); }
void orc_destroy(orc_ctx* c) { delete c; }

// External force (Eq. for f_ext): each loaded boundary triangle adds t A / 3
// to its three vertices.
int orc_set_traction(orc_ctx* c, int n_faces, const int* tri, const double* t, double ramp_t0) {
  for (auto& x : c->F) x = {0, 0, 0};
  for (int f = 0; f < n_faces; ++f) {
    int a = tri[3 * f], b = tri[3 * f + 1], d = tri[3 * f + 2];
    if (a < 0 || b < 0 || d < 0 || a >= c->N0 || b >= c->N0 || d >= c->N0)
      return c->fail(-1, "traction face node out of range");
    double A = 0.5 * norm(cross(sub(c->X[b], c->X[a]), sub(c->X[d], c->X[a])));
    for (int q = 0; q < 3; ++q) {
      int n = tri[3 * f + q];
      for (int k = 0; k < 3; ++k) c->F[n][k] += t[3 * f + k] * A / 3.0;
    }
  }
  c->ramp_t0 = ramp_t0;
  c->need_init = true;
  return 0;
}

int orc_presplit(orc_ctx* c, int n, const int* tet, const unsigned char* mask) {
  if (c->D == 12.0) {  // hexes: mask holds the crack plane index
    std::vector<std::pair<int, int>> lst;
    for (int i = 0; i < n; ++i) {
      if (tet[i] < 0 || tet[i] >= c->T0) return c->fail(-1, "precrack hex out of range");
      if (mask[i] >= 23) return c->fail(-1, "crack plane index out of range");
      lst.push_back({tet[i], mask[i]});
    }
    std::sort(lst.begin(), lst.end());
    for (auto& p : lst) {
      if (c->smask[p.first] >= 0) continue;
      apply_hex_crack(c, p.first, p.second);
      c->events.push_back({(int)c->step, p.first, p.second, 0, 0.0});
      c->nsplit++;
    }
    c->need_init = true;
    return 0;
  }
  std::vector<std::pair<int, int>> lst;
  for (int i = 0; i < n; ++i) {
    int nb = popcount4(mask[i] & 15);
    if (tet[i] < 0 || tet[i] >= c->T0) return c->fail(-1, "presplit tet out of range");
    if ((mask[i] & ~15) || nb == 0 || nb == 4) return c->fail(-1, "presplit mask is not a partition");
    lst.push_back({tet[i], mask[i]});
  }
  std::sort(lst.begin(), lst.end());
  for (auto& p : lst) {
    if (c->smask[p.first] >= 0) continue;
    apply_split(c, p.first, p.second);
    c->events.push_back({(int)c->step, p.first, p.second, 0, 0.0});
    c->nsplit++;
  }
  if (c->mode == 0) rebuild_masses(c);
  c->need_init = true;
  return 0;
}

// Critical step: dt_crit = 2 / omega_hat, omega_hat^2 the largest element
// eigenvalue of M_e^{-1} K_e with K_e = V B^T C B and M_e = rho V / 4 I.
int orc_critical_dt(orc_ctx* c, double* dt_crit) {
  std::vector<double> lam(c->T0);
  orc_elem_lambda_max(c, lam.data());
  double lmax = 0;
  for (double l : lam) lmax = std::max(lmax, l);
  // M_e = rho V / nn per node: omega^2 = (nn / rho) lambda_max(B^T C B)
  *dt_crit = 2.0 / std::sqrt(c->el[0].nn / c->rho * lmax);
  return 0;
}

// Largest eigenvalue of B^T C B for one strain-displacement matrix of nc
// columns (dense cyclic Jacobi).
double lambda_max_btcb(const double B[6][24], int nc, const double C[6][6]) {
  std::vector<double> K(nc * nc, 0.0);
  for (int i = 0; i < nc; ++i)
    for (int j = 0; j < nc; ++j) {
      double s = 0;
      for (int r = 0; r < 6; ++r)
        for (int q = 0; q < 6; ++q) s += B[r][i] * C[r][q] * B[q][j];
      K[nc * i + j] = s;
    }
  double w[24];
  jacobi_eig(nc, K, w, nullptr);
  double lm = w[0];
  for (int i = 1; i < nc; ++i) lm = std::max(lm, w[i]);
  return lm;
}

int orc_elem_lambda_max(orc_ctx* c, double* lam) {
  double C[6][6];
  cmat(c->lam, c->mu, C);
  if (c->D == 12.0) {
    // hexes: the largest over the edge points, max_q lambda_max(B_q^T C B_q),
    // bounds lambda_max of the edge-averaged (1/12) sum_q B_q^T C B_q
    std::map<std::array<double, 288>, double> hmemo;
    for (int t = 0; t < c->T0; ++t) {
      auto it = hmemo.find(c->hexg[t]);
      if (it != hmemo.end()) {
        lam[t] = it->second;
        continue;
      }
      double lm = 0;
      for (int q = 0; q < 12; ++q) {
        double B[6][24];
        elem_bmat(c, t, q, B);
        lm = std::max(lm, lambda_max_btcb(B, 24, C));
      }
      hmemo[c->hexg[t]] = lm;
      lam[t] = lm;
    }
    return 0;
  }
  std::map<std::array<double, 24>, double> memo;  // identical shapes repeat
  for (int t = 0; t < c->T0; ++t) {
    const int nc = 3 * c->el[t].nn;
    std::array<double, 24> key{};
    for (int l = 0; l < c->el[t].nn; ++l)
      for (int d = 0; d < 3; ++d) key[3 * l + d] = c->el[t].g[l][d];
    auto it = memo.find(key);
    if (it != memo.end()) {
      lam[t] = it->second;
      continue;
    }
    double B[6][24];
    bmat(c->el[t], B);
    std::vector<double> K(nc * nc, 0.0);
    for (int i = 0; i < nc; ++i)
      for (int j = 0; j < nc; ++j) {
        double s = 0;
        for (int r = 0; r < 6; ++r)
          for (int q = 0; q < 6; ++q) s += B[r][i] * C[r][q] * B[q][j];
        K[nc * i + j] = s;
      }
    double w[24];
    jacobi_eig(nc, K, w, nullptr);
    double lm = w[0];
    for (int i = 1; i < nc; ++i) lm = std::max(lm, w[i]);
    memo[key] = lm;
    lam[t] = lm;
  }
  // C_t = (E_t / E) C, and the eigenvalues of B^T C_t B scale with it
  for (int t = 0; t < c->T0; ++t) lam[t] *= c->Et[t] / c->E;
  return 0;
}

int orc_set_dt(orc_ctx* c, double dt) {
  if (!(dt > 0)) return c->fail(-1, "dt must be positive");
  c->dt = dt;
  return 0;
}

int orc_counts(orc_ctx* c, int* out) {
  out[0] = (int)c->X.size();
  out[1] = (int)c->el.size();
  int ne = 0;
  for (const auto& p : c->patch) ne += p.empty() ? 0 : 1;
  out[2] = ne;
  out[3] = c->nsplit;
  out[4] = (int)fronts(c).size();
  return 0;
}

int orc_set_state(orc_ctx* c, const double* u, const double* v) {
  for (size_t i = 0; i < c->X.size(); ++i)
    for (int d = 0; d < 3; ++d) {
      if (u) c->u[i][d] = u[3 * i + d];
      if (v) c->v[i][d] = v[3 * i + d];
    }
  c->need_init = true;
  return 0;
}

int orc_get_state(orc_ctx* c, double* u, double* v, double* a) {
  if (c->need_init && c->dt > 0) initialize(c);
  for (size_t i = 0; i < c->X.size(); ++i)
    for (int d = 0; d < 3; ++d) {
      if (u) u[3 * i + d] = c->u[i][d];
      if (v) v[3 * i + d] = c->v[i][d];
      if (a) a[3 * i + d] = c->a[i][d];
    }
  return 0;
}

int orc_internal_force(orc_ctx* c, const double* u, double* f) {
  std::vector<V3> uu(c->X.size());
  for (size_t i = 0; i < uu.size(); ++i) uu[i] = {u[3 * i], u[3 * i + 1], u[3 * i + 2]};
  std::vector<V3> ff;
  internal_force(c, uu, ff);
  for (size_t i = 0; i < ff.size(); ++i)
    for (int d = 0; d < 3; ++d) f[3 * i + d] = ff[i][d];
  return 0;
}

int orc_step(orc_ctx* c, int n_steps) {
  if (!(c->dt > 0)) return c->fail(-7, "dt not set");
  for (int s = 0; s < n_steps; ++s) one_step(c);
  return 0;
}

int orc_energy(orc_ctx* c, double* out) {
  if (c->need_init && c->dt > 0) initialize(c);
  double ke = 0;
  for (size_t i = 0; i < c->X.size(); ++i) ke += 0.5 * c->m[i] * dot(c->v[i], c->v[i]);
  out[0] = (double)c->step;
  out[1] = c->step * c->dt;
  out[2] = ke;
  out[3] = strain_energy(c);
  out[4] = c->W;
  out[5] = c->Ud;
  out[6] = c->Gmax;
  out[7] = c->nsplit;
  out[8] = c->nfront;
  out[9] = (double)c->X.size();
  return 0;
}

int orc_splits(orc_ctx* c, int cap, int* ev4, double* G, int* n_out) {
  int n = (int)c->events.size();
  *n_out = n;
  for (int i = 0; i < n && i < cap; ++i) {
    ev4[4 * i + 0] = c->events[i].step;
    ev4[4 * i + 1] = c->events[i].tet;
    ev4[4 * i + 2] = c->events[i].mask;
    ev4[4 * i + 3] = c->events[i].pattern;
    G[i] = c->events[i].G;
  }
  return 0;
}

int orc_front_G(orc_ctx* c, int cap, int* tfl3, double* g2, int* n_out) {
  std::vector<std::array<double, 6>> eps, sig;
  std::vector<double> Vsum;
  edge_fields(c, c->u, eps, sig, Vsum);
  std::vector<FrontRec> fr = fronts(c);
  if (c->D == 12.0) {  // one row per candidate: (hex, face, plane), (G, pattern)
    int n = 0;
    for (const FrontRec& r : fr)
      for (const HexCand& k : hex_candidates(r.face, r.lone / 16, r.lone % 16)) {
        if (n < cap) {
          tfl3[3 * n] = r.c;
          tfl3[3 * n + 1] = r.face;
          tfl3[3 * n + 2] = k.plane;
          g2[2 * n] = hex_cand_G(c, c->u, sig, r.c, k);
          g2[2 * n + 1] = k.pattern;
        }
        n++;
      }
    *n_out = n;
    return 0;
  }
  *n_out = (int)fr.size();
  for (int i = 0; i < (int)fr.size() && i < cap; ++i) {
    double GI, GII;
    int mI, mII;
    front_G(c, c->u, sig, fr[i], &GI, &GII, &mI, &mII);
    tfl3[3 * i] = fr[i].c;
    tfl3[3 * i + 1] = fr[i].face;
    tfl3[3 * i + 2] = fr[i].lone;
    g2[2 * i] = GI;
    g2[2 * i + 1] = GII;
  }
  return 0;
}

int orc_replay(orc_ctx* c, int n, const int* ev3) {
  if (c->D == 12.0) return c->fail(-7, "a forced schedule is for tetrahedral meshes");
  c->schedule.clear();
  for (int i = 0; i < n; ++i) c->schedule.push_back({ev3[3 * i], ev3[3 * i + 1], ev3[3 * i + 2], 0, 0.0});
  std::stable_sort(c->schedule.begin(), c->schedule.end(), [](const Event& x, const Event& y) {
    return x.step != y.step ? x.step < y.step : x.tet < y.tet;
  });
  c->cursor = 0;
  c->replay = true;
  return 0;
}

int orc_hex_plane_masks(int* out23) {
  for (int p = 0; p < 23; ++p) out23[p] = hex_plane_mask(p);
  return 0;
}

int orc_masses(orc_ctx* c, double* m) {
  for (size_t i = 0; i < c->m.size(); ++i) m[i] = c->m[i];
  return 0;
}

int orc_loads(orc_ctx* c, double* F) {
  for (size_t i = 0; i < c->F.size(); ++i)
    for (int d = 0; d < 3; ++d) F[3 * i + d] = c->F[i][d];
  return 0;
}

int orc_elements(orc_ctx* c, int* nodes4, double* Veff, double* V, int* parent) {
  for (size_t e = 0; e < c->el.size(); ++e) {
    for (int l = 0; l < 4; ++l)
      if (nodes4) nodes4[4 * e + l] = c->el[e].n[l];
    if (Veff) Veff[e] = c->el[e].Veff;
    if (V) V[e] = c->el[e].V;
    if (parent) parent[e] = c->el[e].parent;
  }
  return 0;
}

int orc_grad(orc_ctx* c, double* g12) {
  for (size_t e = 0; e < c->el.size(); ++e)
    for (int l = 0; l < 4; ++l)
      for (int d = 0; d < 3; ++d) g12[12 * e + 3 * l + d] = c->el[e].g[l][d];
  return 0;
}

// Edges of the current element set (node pairs with a non-empty patch) with
// their smoothed strain and stress at displacement u (current state if null).
int orc_edges(orc_ctx* c, const double* u, int* nodes2, double* eps6, double* sig6) {
  std::vector<V3> uu = c->u;
  if (u)
    for (size_t i = 0; i < uu.size(); ++i) uu[i] = {u[3 * i], u[3 * i + 1], u[3 * i + 2]};
  std::vector<std::array<double, 6>> eps, sig;
  std::vector<double> Vsum;
  edge_fields(c, uu, eps, sig, Vsum);
  int q = 0;
  for (size_t k = 0; k < eps.size(); ++k) {
    if (c->patch[k].empty()) continue;
    if (nodes2) {
      nodes2[2 * q] = c->edge_nodes[k].first;
      nodes2[2 * q + 1] = c->edge_nodes[k].second;
    }
    for (int r = 0; r < 6; ++r) {
      if (eps6) eps6[6 * q + r] = eps[k][r];
      if (sig6) sig6[6 * q + r] = sig[k][r];
    }
    q++;
  }
  return 0;
}

int orc_sym_eig3(const double* s6, double* lam3, double* vec9) {
  double T[9];
  voigt_to_tensor(s6, T);
  jacobi_eig(3, std::vector<double>(T, T + 9), lam3, vec9);
  return 0;
}

double orc_stress_term(const double* s6, const double* n, int gsig) {
  return stress_term(s6, V3{n[0], n[1], n[2]}, gsig);
}

double orc_crack_area(const double* X4, int mask) {
  V3 x[4];
  for (int l = 0; l < 4; ++l) x[l] = {X4[3 * l], X4[3 * l + 1], X4[3 * l + 2]};
  return crack_area(x, mask);
}

int orc_set_modulus(orc_ctx* c, const double* E_tet) {
  if (c->D != 6.0) return c->fail(-7, "per-element modulus is for tetrahedra");
  for (int t = 0; t < c->T0; ++t) {
    if (!(E_tet[t] > 0)) return c->fail(-1, "modulus must be positive");
  }
  bool het = false;
  for (int t = 0; t < c->T0; ++t) {
    c->Et[t] = E_tet[t];
    het = het || E_tet[t] != c->E;
  }
  c->hetero = het;
  c->need_init = true;
  return 0;
}

int orc_set_frozen(orc_ctx* c, int on) {
  c->frozen = on != 0;
  return 0;
}

int orc_set_threads(orc_ctx* c, int n) {
  if (n < 1) return c->fail(-1, "thread count must be positive");
  c->nthreads = n;
  return 0;
}

int orc_window_gradient(orc_ctx* c, int n_steps, const double* gu, const double* gv, double* gu0,
                        double* gv0, double* gE) {
  if (!(c->dt > 0)) return c->fail(-7, "dt not set");
  if (n_steps < 0) return c->fail(-1, "negative step count");
  if (!c->grp_t0.empty()) return c->fail(-7, "windows with prescribed velocities are not supported");
  return window_gradient(c, n_steps, gu, gv, gu0, gv0, gE);
}

int orc_add_velocity_bc(orc_ctx* c, int n, const int* node, const int* mask, const double* v0,
                        double t0, int* group) {
  if (c->step != 0) return c->fail(-7, "prescribed velocities must precede the first step");
  if (!(t0 >= 0)) return c->fail(-1, "ramp time must be >= 0");
  int g = (int)c->grp_t0.size();
  for (int b = 0; b < n; ++b) {
    if (node[b] < 0 || node[b] >= c->N0) return c->fail(-1, "constrained node out of range");
    if (mask[b] < 1 || mask[b] > 7) return c->fail(-1, "dof mask must be 1..7");
    for (int q = 0; q < b; ++q)
      if (node[q] == node[b]) return c->fail(-1, "node listed twice");
    if (std::find(c->bc_node.begin(), c->bc_node.end(), node[b]) != c->bc_node.end())
      return c->fail(-1, "node already constrained");
  }
  for (int b = 0; b < n; ++b) {
    c->bc_node.push_back(node[b]);
    c->bc_mask.push_back(mask[b]);
    c->bc_group.push_back(g);
    c->bc_v0.push_back({v0[3 * b], v0[3 * b + 1], v0[3 * b + 2]});
    c->bc_uref.push_back(c->u[node[b]]);
    c->bc_R.push_back({0, 0, 0});
  }
  c->grp_t0.push_back(t0);
  c->grp_W.push_back(0.0);
  c->grp_hist.push_back({});
  c->need_init = true;
  if (group) *group = g;
  return 0;
}

int orc_reactions(orc_ctx* c, int group, int cap, double* rows6, int* n_out, double* work) {
  if (group < 0 || group >= (int)c->grp_t0.size()) return c->fail(-1, "no such group");
  const auto& h = c->grp_hist[group];
  int n = (int)h.size();
  *n_out = n;
  for (int i = 0; i < n && i < cap; ++i)
    for (int k = 0; k < 6; ++k) rows6[6 * i + k] = h[i][k];
  if (work) *work = c->grp_W[group];
  return 0;
}

int orc_strain_energy_grad(orc_ctx* c, const double* u, double* gE) {
  // explicit sensitivity of SE = 1/2 u^T K(E) u to each tet's modulus at fixed
  // u: 1/2 u^T (dK/dE_j) u (the same edge sum as the window's modulus term)
  std::vector<V3> uu = c->u;
  if (u)
    for (size_t i = 0; i < uu.size(); ++i) uu[i] = {u[3 * i], u[3 * i + 1], u[3 * i + 2]};
  std::vector<double> out(c->T0, 0.0);
  modulus_term(c, uu, uu, 0.5, out);
  for (int t = 0; t < c->T0; ++t) gE[t] = out[t];
  return 0;
}

}  // extern "C"
