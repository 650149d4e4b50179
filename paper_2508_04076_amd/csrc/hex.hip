// HIP kernels (gfx950) for trilinear hexahedra: the ES-H-FEM form of
// Eqs. hex_strain_discretization and hex_fint_discretization.
//
// Hex e enters the smoothing domain of each of its 12 edges q with its
// shape-function gradients at the edge's point G_q, the midpoint of the hex
// edge (Eq. strain_discretization evaluates dN/dx at G_i).  The gradients are
// recomputed from the corner coordinates where they are needed, twelve
// Jacobians per hex and pass, not stored:
//   strain  per hex: V_e eps_e(G_q) for q = 0..11, one record per (hex, edge)
//           (the patch entries of a hex mesh name 12 e + q);
//   edge    shared with the tetrahedra: eps_k = sum_patch V eps / sum_patch V,
//           sigma_k = C eps_k;
//   force   per hex: the eight nodal terms
//           (V_e / 12) sum_q grad N_i(G_q)^T sigma_{k(q)}
//           (w_ek V_k = V_e / 12), written at the (hex, local) positions of the
//           node lists, which the node pass sums per node in list order
//           (shared with the tetrahedra's term layout).
#include "hex_crack.h"

namespace cem {

// hex node order: bottom face 0-1-2-3 counter-clockwise seen from above, top
// face 4-7 above them; reference corner signs and the twelve edges
// (compile-time tables: with the edge-point loops unrolled, the shape-function
// derivatives at each edge midpoint are constants, and their zeros fold away)
constexpr signed char kHexSign[8][3] = {{-1, -1, -1}, {1, -1, -1}, {1, 1, -1}, {-1, 1, -1},
                                        {-1, -1, 1},  {1, -1, 1},  {1, 1, 1},  {-1, 1, 1}};
constexpr signed char kHexEdgeL[12][2] = {{0, 1}, {1, 2}, {2, 3}, {3, 0}, {4, 5}, {5, 6},
                                          {6, 7}, {7, 4}, {0, 4}, {1, 5}, {2, 6}, {3, 7}};

__device__ __forceinline__ void hex_nodes(const Mesh& m, int e, int* nd) {
  int4 a = m.hnodes[2 * e], b = m.hnodes[2 * e + 1];
  nd[0] = a.x; nd[1] = a.y; nd[2] = a.z; nd[3] = a.w;
  nd[4] = b.x; nd[5] = b.y; nd[6] = b.z; nd[7] = b.w;
}

__device__ __forceinline__ void hex_coords(const Mesh& m, const int* nd, double (&x)[8][3]) {
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    double4 p = m.X[nd[i]];
    x[i][0] = p.x; x[i][1] = p.y; x[i][2] = p.z;
  }
}

// Gradients of the eight shape functions at the natural point xi, scaled by
// the Jacobian determinant: gd_i = adj(J)^T dN_i/dxi = det J * J^-T dN_i/dxi
// (J[r][c] = dx_r / dxi_c).  Returns det J.
__device__ __forceinline__ double hex_grad_at(const double (&x)[8][3], const double* xi,
                                              double (&gd)[8][3]) {
  double dN[8][3];
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    double f0 = 1.0 + xi[0] * kHexSign[i][0], f1 = 1.0 + xi[1] * kHexSign[i][1],
           f2 = 1.0 + xi[2] * kHexSign[i][2];
    dN[i][0] = 0.125 * kHexSign[i][0] * f1 * f2;
    dN[i][1] = 0.125 * f0 * kHexSign[i][1] * f2;
    dN[i][2] = 0.125 * f0 * f1 * kHexSign[i][2];
  }
  double J[3][3] = {};
#pragma unroll
  for (int i = 0; i < 8; ++i)
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int cc = 0; cc < 3; ++cc) J[r][cc] += x[i][r] * dN[i][cc];
  double A[3][3];  // cofactor matrix: A[r][c] = cofactor of J[r][c]
  A[0][0] = J[1][1] * J[2][2] - J[1][2] * J[2][1];
  A[0][1] = J[1][2] * J[2][0] - J[1][0] * J[2][2];
  A[0][2] = J[1][0] * J[2][1] - J[1][1] * J[2][0];
  A[1][0] = J[0][2] * J[2][1] - J[0][1] * J[2][2];
  A[1][1] = J[0][0] * J[2][2] - J[0][2] * J[2][0];
  A[1][2] = J[0][1] * J[2][0] - J[0][0] * J[2][1];
  A[2][0] = J[0][1] * J[1][2] - J[0][2] * J[1][1];
  A[2][1] = J[0][2] * J[1][0] - J[0][0] * J[1][2];
  A[2][2] = J[0][0] * J[1][1] - J[0][1] * J[1][0];
  // det J * J^-T = cofactor matrix
#pragma unroll
  for (int i = 0; i < 8; ++i)
#pragma unroll
    for (int d = 0; d < 3; ++d) gd[i][d] = A[d][0] * dN[i][0] + A[d][1] * dN[i][1] + A[d][2] * dN[i][2];
  return J[0][0] * A[0][0] + J[0][1] * A[0][1] + J[0][2] * A[0][2];
}

// natural coordinates of the midpoint of local edge q
__device__ __forceinline__ void hex_edge_point(int q, double* xi) {
  const int a = kHexEdgeL[q][0], b = kHexEdgeL[q][1];
#pragma unroll
  for (int d = 0; d < 3; ++d) xi[d] = 0.5 * (kHexSign[a][d] + kHexSign[b][d]);
}

// Volume: sum of det J over the 2 x 2 x 2 Gauss points (weights 1; exact for
// the trilinear map).
__global__ __launch_bounds__(kBlock) void k_hex_geometry(Mesh m) {
  int e = blockIdx.x * kBlock + threadIdx.x;
  if (e >= m.T0) return;
  int nd[8];
  hex_nodes(m, e, nd);
  double x[8][3];
  hex_coords(m, nd, x);
  const double a = 0.57735026918962576451;  // 1 / sqrt(3)
  double V = 0;
#pragma unroll 1
  for (int gp = 0; gp < 8; ++gp) {
    double xi[3] = {kHexSign[gp][0] * a, kHexSign[gp][1] * a, kHexSign[gp][2] * a};
    double gd[8][3];
    V += hex_grad_at(x, xi, gd);
  }
  m.vol[e] = V;
}

// V_e eps_e(G_q) = (V_e / det J) sum_{i=1..7} sym(gd_i (x) (u_i - u_0)) for each
// local edge q (sum_i grad N_i = 0); the differences are taken in float64
// before any conversion to R.
template <class R>
__global__ __launch_bounds__(kBlock) void k_strain_hex(Mesh m, const double4* __restrict__ u,
                                                       Six<R>* __restrict__ veps,
                                                       const Counters* __restrict__ c) {
  if (c->err) return;
  Chunks it(m.T0);
  for (int e; it.next(e);) {
    if (e >= m.T0) continue;
    int nd[8];
    hex_nodes(m, e, nd);
    double x[8][3];
    hex_coords(m, nd, x);
    R du[8][3];
    const double4 u0 = u[nd[0]];
#pragma unroll
    for (int i = 1; i < 8; ++i) {
      double4 ui = u[nd[i]];
      du[i][0] = (R)(ui.x - u0.x);
      du[i][1] = (R)(ui.y - u0.y);
      du[i][2] = (R)(ui.z - u0.z);
    }
    const double V = m.vol[e];
#pragma unroll
    for (int q = 0; q < 12; ++q) {
      double xi[3], gd[8][3];
      hex_edge_point(q, xi);
      const double s = V / hex_grad_at(x, xi, gd);
      R o[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll
      for (int i = 1; i < 8; ++i) {
        R gx = (R)(gd[i][0] * s), gy = (R)(gd[i][1] * s), gz = (R)(gd[i][2] * s);
        R dx = du[i][0], dy = du[i][1], dz = du[i][2];
        o[0] += gx * dx;
        o[1] += gy * dy;
        o[2] += gz * dz;
        o[3] += gy * dx + gx * dy;
        o[4] += gz * dy + gy * dz;
        o[5] += gz * dx + gx * dz;
      }
      store6(veps + 12 * (size_t)e + q, o);
    }
  }
}

// The eight nodal terms of hex e, (V_e / 12) sum_q grad N_i(G_q)^T sigma_{k(q)},
// written at the node-list positions of its (hex, local) entries.  The first
// fg workgroups (dispatched first, so they run beside the element workgroups)
// take the crack pass: both read the edge stresses and write disjoint data.
template <class R>
__global__ __launch_bounds__(kBlock) void k_elem_force_hex(Mesh m, const Six<R>* __restrict__ esig,
                                                           R* __restrict__ contrib,
                                                           const double4* __restrict__ uh,
                                                           Counters* __restrict__ c, int fg,
                                                           int flagging) {
  if (c->err) return;
  if ((int)blockIdx.x < fg) {
    __shared__ unsigned long long red[kBlock];
    hex_front_block<R>(m, uh, esig, c, flagging, blockIdx.x, fg, red);
    return;
  }
  Chunks it(m.T0, (int)gridDim.x - fg, fg);
  for (int e; it.next(e);) {
    if (e >= m.T0) continue;
    int nd[8];
    hex_nodes(m, e, nd);
    double x[8][3];
    hex_coords(m, nd, x);
    const double w = m.vol[e] / 12.0;
    double f[8][3] = {};
#pragma unroll
    for (int q = 0; q < 12; ++q) {
      const int2 k2 = m.he2e[6 * (size_t)e + (q >> 1)];
      const Six<R> sg = load6(esig + ((q & 1) ? k2.y : k2.x));
      double xi[3], gd[8][3];
      hex_edge_point(q, xi);
      const double s = w / hex_grad_at(x, xi, gd);
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        R gx = (R)(gd[i][0] * s), gy = (R)(gd[i][1] * s), gz = (R)(gd[i][2] * s);
        f[i][0] += (double)(gx * sg.v[0] + gy * sg.v[3] + gz * sg.v[5]);
        f[i][1] += (double)(gy * sg.v[1] + gx * sg.v[3] + gz * sg.v[4]);
        f[i][2] += (double)(gz * sg.v[2] + gy * sg.v[4] + gx * sg.v[5]);
      }
    }
    const int4 pa = m.epos[2 * (size_t)e], pb = m.epos[2 * (size_t)e + 1];
    const int pos[8] = {pa.x, pa.y, pa.z, pa.w, pb.x, pb.y, pb.z, pb.w};
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      R* o = contrib + 3 * (size_t)pos[i];
      o[0] = (R)f[i][0];
      o[1] = (R)f[i][1];
      o[2] = (R)f[i][2];
    }
  }
}

// Element bound of the largest frequency: (8 / rho) max_q lambda_max(B_q^T C B_q)
// over the hex's edge points (at least lambda_max of the edge-averaged
// stiffness), each via the 6 x 6 matrix (L^T B_q)(L^T B_q)^T with C = L L^T.
__global__ __launch_bounds__(kBlock) void k_dtcrit_hex(Mesh m, Counters* __restrict__ c) {
  __shared__ unsigned long long red[kBlock];
  double lmax = 0;
  int e = blockIdx.x * kBlock + threadIdx.x;
  if (e < m.T0) {
    int nd[8];
    hex_nodes(m, e, nd);
    double x[8][3];
    hex_coords(m, nd, x);
    double a = m.lam + 2 * m.mu, b = m.lam;
    double L11 = sqrt(a), L21 = b / L11, L31 = b / L11;
    double L22 = sqrt(a - L21 * L21), L32 = (b - L31 * L21) / L22;
    double L33 = sqrt(a - L31 * L31 - L32 * L32);
    double sm = sqrt(m.mu);
#pragma unroll 1
    for (int q = 0; q < 12; ++q) {
      double xi[3], gd[8][3];
      hex_edge_point(q, xi);
      const double iv = 1.0 / hex_grad_at(x, xi, gd);
      double Xm[6][24];
      for (int i = 0; i < 8; ++i) {
        double gx = gd[i][0] * iv, gy = gd[i][1] * iv, gz = gd[i][2] * iv;
        // rows of B for node i (columns 3i, 3i+1, 3i+2), premultiplied by L^T
        double B[6][3] = {{gx, 0, 0}, {0, gy, 0}, {0, 0, gz}, {gy, gx, 0}, {0, gz, gy}, {gz, 0, gx}};
        for (int r = 0; r < 3; ++r) {
          Xm[0][3 * i + r] = L11 * B[0][r] + L21 * B[1][r] + L31 * B[2][r];
          Xm[1][3 * i + r] = L22 * B[1][r] + L32 * B[2][r];
          Xm[2][3 * i + r] = L33 * B[2][r];
          Xm[3][3 * i + r] = sm * B[3][r];
          Xm[4][3 * i + r] = sm * B[4][r];
          Xm[5][3 * i + r] = sm * B[5][r];
        }
      }
      double A[6][6];
      for (int i = 0; i < 6; ++i)
        for (int j = 0; j < 6; ++j) {
          double s = 0;
          for (int r = 0; r < 24; ++r) s += Xm[i][r] * Xm[j][r];
          A[i][j] = s;
        }
      lmax = fmax(lmax, jacobi_lmax6(A));
    }
  }
  red[threadIdx.x] = dkey(lmax);
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w)
      red[threadIdx.x] = red[threadIdx.x] > red[threadIdx.x + w] ? red[threadIdx.x] : red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicMax(&c->lam_key, red[0]);
}

// ---------------------------------------------------------------- launchers

hipError_t launch_hex_geometry(const Mesh& m, hipStream_t s) {
  hipLaunchKernelGGL(k_hex_geometry, dim3(grid_for(m.T0)), dim3(kBlock), 0, s, m);
  return hipGetLastError();
}

template <class R>
hipError_t launch_strain_hex(const Mesh& m, const double4* u, void* veps, Counters* c,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_strain_hex<R>, dim3(persistent_grid(m, m.T0)), dim3(kBlock), 0, s, m, u,
                     (Six<R>*)veps, c);
  return hipGetLastError();
}

template <class R>
hipError_t launch_elem_force_hex(const Mesh& m, const void* esig, void* contrib, const double4* uh,
                                 Counters* c, int fg, int flagging, hipStream_t s) {
  hipLaunchKernelGGL(k_elem_force_hex<R>, dim3(fg + persistent_grid(m, m.T0)), dim3(kBlock), 0, s, m,
                     (const Six<R>*)esig, (R*)contrib, uh, c, fg, flagging);
  return hipGetLastError();
}

template hipError_t launch_strain_hex<double>(const Mesh&, const double4*, void*, Counters*, hipStream_t);
template hipError_t launch_strain_hex<float>(const Mesh&, const double4*, void*, Counters*, hipStream_t);
template hipError_t launch_elem_force_hex<double>(const Mesh&, const void*, void*, const double4*,
                                                  Counters*, int, int, hipStream_t);
template hipError_t launch_elem_force_hex<float>(const Mesh&, const void*, void*, const double4*,
                                                 Counters*, int, int, hipStream_t);

hipError_t launch_dtcrit_hex(const Mesh& m, Counters* c, hipStream_t s) {
  hipLaunchKernelGGL(k_dtcrit_hex, dim3(grid_for(m.T0)), dim3(kBlock), 0, s, m, c);
  return hipGetLastError();
}

}  // namespace cem
