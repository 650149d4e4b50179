// HIP kernels (gfx950) for trilinear hexahedra: the ES-H-FEM form of
// Eqs. hex_strain_discretization and hex_fint_discretization.
//
// Each hex enters the edge smoothing with one gradient per node, the volume
// average of grad N_i over the element; the kernels keep G_i = V grad N_i =
// integral of grad N_i (computed once, 2 x 2 x 2 Gauss points).  The edge
// smoothing domain has V_k = (1/12) sum of the patch volumes, and the force
// identity reads
//   sum_k V_k Bt_k^T sigma_k = sum_e (1/12) [G_e]^T sum_{k in edges(e)} sigma_k,
// so the strain, edge and node passes keep the structure of the tetrahedral
// path (the edge and node passes are shared with it).
#include "device_util.h"

namespace cem {

// hex node order: bottom face 0-1-2-3 counter-clockwise seen from above, top
// face 4-7 above them; reference corner signs
__device__ __constant__ signed char kHexSign[8][3] = {{-1, -1, -1}, {1, -1, -1}, {1, 1, -1},
                                                       {-1, 1, -1},  {-1, -1, 1}, {1, -1, 1},
                                                       {1, 1, 1},    {-1, 1, 1}};

__device__ __forceinline__ void hex_nodes(const Mesh& m, int e, int* nd) {
  int4 a = m.hnodes[2 * e], b = m.hnodes[2 * e + 1];
  nd[0] = a.x; nd[1] = a.y; nd[2] = a.z; nd[3] = a.w;
  nd[4] = b.x; nd[5] = b.y; nd[6] = b.z; nd[7] = b.w;
}

// G_i (8 x 3) packed row-major into six double4 per hex.
__device__ __forceinline__ void load_hgrad(const Mesh& m, int e, double* G) {
  const double4* p = m.hgrad + 6 * (size_t)e;
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    double4 v = p[q];
    G[4 * q] = v.x; G[4 * q + 1] = v.y; G[4 * q + 2] = v.z; G[4 * q + 3] = v.w;
  }
}

// Volume and G_i = sum over the Gauss points of J^-T dN_i/dxi det J.
__global__ __launch_bounds__(kBlock) void k_hex_geometry(Mesh m) {
  int e = blockIdx.x * kBlock + threadIdx.x;
  if (e >= m.T0) return;
  int nd[8];
  hex_nodes(m, e, nd);
  double x[8][3];
  for (int i = 0; i < 8; ++i) {
    double4 p = m.X[nd[i]];
    x[i][0] = p.x; x[i][1] = p.y; x[i][2] = p.z;
  }
  const double a = 0.57735026918962576451;  // 1 / sqrt(3)
  double G[8][3] = {};
  double V = 0;
  for (int gp = 0; gp < 8; ++gp) {
    double xi[3] = {kHexSign[gp][0] * a, kHexSign[gp][1] * a, kHexSign[gp][2] * a};
    double dN[8][3];
    for (int i = 0; i < 8; ++i) {
      double f0 = 1.0 + xi[0] * kHexSign[i][0], f1 = 1.0 + xi[1] * kHexSign[i][1],
             f2 = 1.0 + xi[2] * kHexSign[i][2];
      dN[i][0] = 0.125 * kHexSign[i][0] * f1 * f2;
      dN[i][1] = 0.125 * f0 * kHexSign[i][1] * f2;
      dN[i][2] = 0.125 * f0 * f1 * kHexSign[i][2];
    }
    double J[3][3] = {};
    for (int i = 0; i < 8; ++i)
      for (int r = 0; r < 3; ++r)
        for (int cc = 0; cc < 3; ++cc) J[r][cc] += x[i][r] * dN[i][cc];
    // adj(J)^T dN_i = det J * J^-T dN_i: no division needed
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
    V += J[0][0] * A[0][0] + J[0][1] * A[0][1] + J[0][2] * A[0][2];
    // det J * J^-T = cofactor matrix
    for (int i = 0; i < 8; ++i)
      for (int d = 0; d < 3; ++d)
        G[i][d] += A[d][0] * dN[i][0] + A[d][1] * dN[i][1] + A[d][2] * dN[i][2];
  }
  double4* out = m.hgrad + 6 * (size_t)e;
  const double* g = &G[0][0];
  for (int q = 0; q < 6; ++q)
    out[q] = make_double4(g[4 * q], g[4 * q + 1], g[4 * q + 2], g[4 * q + 3]);
  m.vol[e] = V;
}

// V eps = sum_{i=1..7} sym(G_i (x) (u_i - u_0))  (sum_i G_i = 0); the
// differences are taken in float64 before any conversion to R.
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
    double G[24];
    load_hgrad(m, e, G);
    double4 u0 = u[nd[0]];
    R o[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int i = 1; i < 8; ++i) {
      double4 ui = u[nd[i]];
      R dx = (R)(ui.x - u0.x), dy = (R)(ui.y - u0.y), dz = (R)(ui.z - u0.z);
      R gx = (R)G[3 * i], gy = (R)G[3 * i + 1], gz = (R)G[3 * i + 2];
      o[0] += gx * dx;
      o[1] += gy * dy;
      o[2] += gz * dz;
      o[3] += gy * dx + gx * dy;
      o[4] += gz * dy + gy * dz;
      o[5] += gz * dx + gx * dz;
    }
    store6(veps + e, o);
  }
}

// Per hex, s_e = (1/12) sum_{k in edges(e)} sigma_k.  The nodal terms
// c_{e,i} = G_i^T s_e are formed by the node pass, which gathers s_e and G_i
// per node-list entry: 48 bytes written per hex instead of eight 24-byte
// terms, and G read once, by the node pass.
template <class R>
__global__ __launch_bounds__(kBlock) void k_elem_force_hex(Mesh m, const Six<R>* __restrict__ esig,
                                                           R* __restrict__ contrib,
                                                           Counters* __restrict__ c) {
  if (c->err) return;
  Chunks it(m.T0);
  for (int e; it.next(e);) {
    if (e >= m.T0) continue;
    R sg[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      int2 k2 = m.he2e[6 * (size_t)e + q];
      Six<R> a = load6(esig + k2.x), b = load6(esig + k2.y);
#pragma unroll
      for (int r = 0; r < 6; ++r) sg[r] += a.v[r] + b.v[r];
    }
    const R w = (R)(1.0 / 12.0);
#pragma unroll
    for (int r = 0; r < 6; ++r) sg[r] *= w;
    store6((Six<R>*)contrib + e, sg);
  }
}

// Largest eigenvalue of Bbar^T C Bbar per hex (Bbar from G / V), via the
// 6 x 6 matrix (L^T Bbar)(L^T Bbar)^T with C = L L^T.
__global__ __launch_bounds__(kBlock) void k_dtcrit_hex(Mesh m, Counters* __restrict__ c) {
  __shared__ unsigned long long red[kBlock];
  double lmax = 0;
  int e = blockIdx.x * kBlock + threadIdx.x;
  if (e < m.T0) {
    double G[24];
    load_hgrad(m, e, G);
    double iv = 1.0 / m.vol[e];
    double Xm[6][24];
    double a = m.lam + 2 * m.mu, b = m.lam;
    double L11 = sqrt(a), L21 = b / L11, L31 = b / L11;
    double L22 = sqrt(a - L21 * L21), L32 = (b - L31 * L21) / L22;
    double L33 = sqrt(a - L31 * L31 - L32 * L32);
    double sm = sqrt(m.mu);
    for (int i = 0; i < 8; ++i) {
      double gx = G[3 * i] * iv, gy = G[3 * i + 1] * iv, gz = G[3 * i + 2] * iv;
      // rows of B for node i (columns 3i, 3i+1, 3i+2), premultiplied by L^T
      double B[6][3] = {{gx, 0, 0}, {0, gy, 0}, {0, 0, gz}, {gy, gx, 0}, {0, gz, gy}, {gz, 0, gx}};
      for (int q = 0; q < 3; ++q) {
        Xm[0][3 * i + q] = L11 * B[0][q] + L21 * B[1][q] + L31 * B[2][q];
        Xm[1][3 * i + q] = L22 * B[1][q] + L32 * B[2][q];
        Xm[2][3 * i + q] = L33 * B[2][q];
        Xm[3][3 * i + q] = sm * B[3][q];
        Xm[4][3 * i + q] = sm * B[4][q];
        Xm[5][3 * i + q] = sm * B[5][q];
      }
    }
    double A[6][6];
    for (int i = 0; i < 6; ++i)
      for (int j = 0; j < 6; ++j) {
        double s = 0;
        for (int q = 0; q < 24; ++q) s += Xm[i][q] * Xm[j][q];
        A[i][j] = s;
      }
    lmax = jacobi_lmax6(A);
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
hipError_t launch_elem_force_hex(const Mesh& m, const void* esig, void* contrib, Counters* c,
                                 hipStream_t s) {
  hipLaunchKernelGGL(k_elem_force_hex<R>, dim3(persistent_grid(m, m.T0)), dim3(kBlock), 0, s, m,
                     (const Six<R>*)esig, (R*)contrib, c);
  return hipGetLastError();
}

template hipError_t launch_strain_hex<double>(const Mesh&, const double4*, void*, Counters*, hipStream_t);
template hipError_t launch_strain_hex<float>(const Mesh&, const double4*, void*, Counters*, hipStream_t);
template hipError_t launch_elem_force_hex<double>(const Mesh&, const void*, void*, Counters*, hipStream_t);
template hipError_t launch_elem_force_hex<float>(const Mesh&, const void*, void*, Counters*, hipStream_t);

hipError_t launch_dtcrit_hex(const Mesh& m, Counters* c, hipStream_t s) {
  hipLaunchKernelGGL(k_dtcrit_hex, dim3(grid_for(m.T0)), dim3(kBlock), 0, s, m, c);
  return hipGetLastError();
}

}  // namespace cem
