// Device helpers shared by the kernel files of the step and of its adjoint.
#ifndef CEM_DEVICE_UTIL_H
#define CEM_DEVICE_UTIL_H

#include "cem_device.h"

#include <float.h>
#include <math.h>

// patch entries gathered together by the edge passes
#ifndef CEM_EDGE_BATCH
#define CEM_EDGE_BATCH 6
#endif
// unroll factor of the per-node entry loops of the node pass: 2 keeps two
// entries' gathers in flight per lane (same sum order; 3-5% faster than 1 on
// the plate and the blocks, 4 no better)
#ifndef CEM_NODE_UNROLL
#define CEM_NODE_UNROLL 2
#endif
#define CEM_PRAGMA_(x) _Pragma(#x)
#define CEM_PRAGMA(x) CEM_PRAGMA_(x)
// fewest dead entries before the crack-front candidate list is compacted
#ifndef CEM_CAND_COMPACT_MIN
#define CEM_CAND_COMPACT_MIN 64
#endif

namespace cem {

// ---------------------------------------------------------------- helpers

// Persistent grid-stride launch: the grid (a multiple of 8 workgroups) is
// sized to the chip, not to the data.  Chunks of kBlock items are split into
// eight contiguous ranges, one per XCD (workgroup b runs on XCD b % 8), and
// the workgroups of an XCD stride through its range.  The item count is read
// on the device, so a captured graph stays valid as splits add elements.
struct Chunks {
  int ch, hi, stride;
  // nblocks: the workgroups that share the items, starting at workgroup b0
  // (a multiple of 8, so that each keeps its XCD); default the whole grid
  __device__ __forceinline__ Chunks(long long count, int nblocks = 0, int b0 = 0) {
    long long nch = (count + kBlock - 1) / kBlock;
    int b = (int)blockIdx.x - b0;
    int x = b % 8, j = b / 8;
    stride = (nblocks > 0 ? nblocks : (int)gridDim.x) / 8;
    ch = (int)(nch * x / 8) + j;
    hi = (int)(nch * (x + 1) / 8);
  }
  __device__ __forceinline__ bool next(int& item) {
    if (ch >= hi) return false;
    item = ch * kBlock + threadIdx.x;
    ch += stride;
    return true;
  }
};

__device__ __forceinline__ double frac_of(int code) {
  return code == FR_ONE ? 1.0 : code == FR_HALF ? 0.5 : code == FR_EIGHTH ? 0.125
       : code == FR_SEVEN8 ? 0.875 : 0.0;
}

__device__ __forceinline__ int pack0(int node, int code) { return node | (code << kNodeBits); }

__device__ __forceinline__ unsigned long long dkey(double x) {
  unsigned long long b = (unsigned long long)__double_as_longlong(x);
  return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}
__host__ __device__ inline double key_to_double(unsigned long long k) {
  unsigned long long b = (k >> 63) ? (k & 0x7fffffffffffffffull) : ~k;
  union { unsigned long long u; double d; } x;
  x.u = b;
  return x.d;
}

template <class R> __device__ __forceinline__ Six<R> load6(const Six<R>* p) { return *p; }
template <class R> __device__ __forceinline__ void store6(Six<R>* p, const R* v) {
  Six<R> s;
#pragma unroll
  for (int i = 0; i < 6; ++i) s.v[i] = v[i];
  *p = s;
}

// Time step of node i (one per instance in a batch).
__device__ __forceinline__ double node_dt(const Mesh& m, int i) {
  return m.n_inst ? m.dti[m.inst[i]] : m.dt;
}

__device__ __forceinline__ double ramp(const Mesh& m, double t) {
  return (m.ramp_t0 > 0.0 && t < m.ramp_t0) ? t / m.ramp_t0 : 1.0;
}

__device__ __forceinline__ int n_split_now(const Counters* c) { return c->n_split; }
__device__ __forceinline__ int elems_now(const Mesh& m, const Counters* c) {
  return m.T0 + (m.mode == MODE_PHANTOM ? c->n_split : 0);
}
__device__ __forceinline__ int nodes_now(const Mesh& m, const Counters* c) {
  return m.N0 + (m.mode == MODE_PHANTOM ? 4 * c->n_split : 0);
}
__device__ __forceinline__ int edges_now(const Mesh& m, const Counters* c) {
  return m.E0 + (m.mode == MODE_PHANTOM ? 10 * c->n_split : 0);
}

// g_l = 6 V grad N_l (l = 1..3) as face cross products of c_l = X_l - X_0:
// g_1 = c2 x c3, g_2 = c3 x c1, g_3 = c1 x c2.  Differences in float64.
template <class R>
__device__ __forceinline__ void face_normals(double4 x0, double4 x1, double4 x2, double4 x3,
                                             R g[3][3]) {
  R c1x = (R)(x1.x - x0.x), c1y = (R)(x1.y - x0.y), c1z = (R)(x1.z - x0.z);
  R c2x = (R)(x2.x - x0.x), c2y = (R)(x2.y - x0.y), c2z = (R)(x2.z - x0.z);
  R c3x = (R)(x3.x - x0.x), c3y = (R)(x3.y - x0.y), c3z = (R)(x3.z - x0.z);
  g[0][0] = c2y * c3z - c2z * c3y; g[0][1] = c2z * c3x - c2x * c3z; g[0][2] = c2x * c3y - c2y * c3x;
  g[1][0] = c3y * c1z - c3z * c1y; g[1][1] = c3z * c1x - c3x * c1z; g[1][2] = c3x * c1y - c3y * c1x;
  g[2][0] = c1y * c2z - c1z * c2y; g[2][1] = c1z * c2x - c1x * c2z; g[2][2] = c1x * c2y - c1y * c2x;
}

// The float32 corner normals of element slot e from the table (the values
// face_normals<float> gives for its corners).
__device__ __forceinline__ void table_normals(const Mesh& m, int e, float g[3][3]) {
  const float* p = m.gtab + 9 * (size_t)e;
#pragma unroll
  for (int l = 0; l < 3; ++l)
#pragma unroll
    for (int d = 0; d < 3; ++d) g[l][d] = p[3 * l + d];
}

// g_1..g_3 of element slot e with corners nd: from the table in float32,
// from the coordinates in float64.
template <class R>
__device__ __forceinline__ void slot_normals(const Mesh& m, int e, int4 nd, R g[3][3]) {
  if constexpr (sizeof(R) == 4) {
    table_normals(m, e, g);
  } else {
    face_normals(m.X[nd.x & kNodeMask], m.X[nd.y], m.X[nd.z], m.X[nd.w], g);
  }
}

// d_l = u_l - u_0 (l = 1..3), taken in float64 before any conversion to R.
template <class R>
__device__ __forceinline__ void node_diffs(double4 u0, double4 u1, double4 u2, double4 u3,
                                           R d[3][3]) {
  d[0][0] = (R)(u1.x - u0.x); d[0][1] = (R)(u1.y - u0.y); d[0][2] = (R)(u1.z - u0.z);
  d[1][0] = (R)(u2.x - u0.x); d[1][1] = (R)(u2.y - u0.y); d[1][2] = (R)(u2.z - u0.z);
  d[2][0] = (R)(u3.x - u0.x); d[2][1] = (R)(u3.y - u0.y); d[2][2] = (R)(u3.z - u0.z);
}

// f sum_l sym(g_l (x) d_l) in Voigt order (xx, yy, zz, xy, yz, xz; engineering shear).
template <class R>
__device__ __forceinline__ void sym_grad(const R g[3][3], const R d[3][3], R f, R* out) {
  out[0] = f * (g[0][0] * d[0][0] + g[1][0] * d[1][0] + g[2][0] * d[2][0]);
  out[1] = f * (g[0][1] * d[0][1] + g[1][1] * d[1][1] + g[2][1] * d[2][1]);
  out[2] = f * (g[0][2] * d[0][2] + g[1][2] * d[1][2] + g[2][2] * d[2][2]);
  out[3] = f * (g[0][1] * d[0][0] + g[0][0] * d[0][1] + g[1][1] * d[1][0] + g[1][0] * d[1][1] +
                g[2][1] * d[2][0] + g[2][0] * d[2][1]);
  out[4] = f * (g[0][2] * d[0][1] + g[0][1] * d[0][2] + g[1][2] * d[1][1] + g[1][1] * d[1][2] +
                g[2][2] * d[2][1] + g[2][1] * d[2][2]);
  out[5] = f * (g[0][2] * d[0][0] + g[0][0] * d[0][2] + g[1][2] * d[1][0] + g[1][0] * d[1][2] +
                g[2][2] * d[2][0] + g[2][0] * d[2][2]);
}

// Sum of V_eff eps over the patch of edge k, in patch order.  Entry ids are
// fetched in batches so that the element gathers of a batch are in flight
// together.
template <class R>
__device__ __forceinline__ void edge_sum(const Mesh& m, const Six<R>* __restrict__ veps, int k,
                                         R* acc) {
  constexpr int B = CEM_EDGE_BATCH;
  int p0 = m.poff[k], p1 = m.poff[k + 1];
#pragma unroll
  for (int i = 0; i < 6; ++i) acc[i] = 0;
  for (int base = p0; base < p1; base += B) {
    int ids[B];
#pragma unroll
    for (int j = 0; j < B; ++j) ids[j] = base + j < p1 ? m.pent[base + j] : -1;
    Six<R> v[B];
#pragma unroll
    for (int j = 0; j < B; ++j) {
      if (ids[j] >= 0) v[j] = load6(veps + ids[j]);
      else
#pragma unroll
        for (int i = 0; i < 6; ++i) v[j].v[i] = 0;
    }
#pragma unroll
    for (int j = 0; j < B; ++j)
#pragma unroll
      for (int i = 0; i < 6; ++i) acc[i] += v[j].v[i];
  }
}

template <class R>
__device__ __forceinline__ void hooke(R lam, R mu, const R* eps, R* sig) {
  R tr = eps[0] + eps[1] + eps[2];
  sig[0] = lam * tr + 2 * mu * eps[0];
  sig[1] = lam * tr + 2 * mu * eps[1];
  sig[2] = lam * tr + 2 * mu * eps[2];
  sig[3] = mu * eps[3];
  sig[4] = mu * eps[4];
  sig[5] = mu * eps[5];
}

// Weighted stress sum of element e: s_e = (f / 36) sum_{k in edges(e)} sigma_k
// (f = V_eff / V), so that the nodal term is c_{e,l} = G_l^T s_e.
template <class R>
__device__ __forceinline__ void elem_ssum(const Mesh& m, int e, int code,
                                          const Six<R>* __restrict__ esig, R sg[6]) {
  int2 q01 = m.et2e[3 * e], q23 = m.et2e[3 * e + 1], q45 = m.et2e[3 * e + 2];
  Six<R> s0 = load6(esig + q01.x), s1 = load6(esig + q01.y), s2 = load6(esig + q23.x);
  Six<R> s3 = load6(esig + q23.y), s4 = load6(esig + q45.x), s5 = load6(esig + q45.y);
  const R w = (R)(frac_of(code) / 36.0);
#pragma unroll
  for (int r = 0; r < 6; ++r) sg[r] = w * (s0.v[r] + s1.v[r] + s2.v[r] + s3.v[r] + s4.v[r] + s5.v[r]);
}

// Nodal terms of element e: c_{e,l} = (V_eff / 6) B_l^T sum_{k in edges(e)} sigma_k
// = (f / 36) G_l^T s with G_l = 6 V grad N_l (G_0 = -(G_1 + G_2 + G_3)).
template <class R>
__device__ __forceinline__ void elem_terms(const Mesh& m, int e, int4 nd, int code,
                                           const Six<R>* __restrict__ esig, R out[4][3]) {
  int2 q01 = m.et2e[3 * e], q23 = m.et2e[3 * e + 1], q45 = m.et2e[3 * e + 2];
  double4 x0 = m.X[nd.x & kNodeMask], x1 = m.X[nd.y], x2 = m.X[nd.z], x3 = m.X[nd.w];
  R sg[6];
  {
    Six<R> s0 = load6(esig + q01.x), s1 = load6(esig + q01.y), s2 = load6(esig + q23.x);
    Six<R> s3 = load6(esig + q23.y), s4 = load6(esig + q45.x), s5 = load6(esig + q45.y);
#pragma unroll
    for (int r = 0; r < 6; ++r) sg[r] = s0.v[r] + s1.v[r] + s2.v[r] + s3.v[r] + s4.v[r] + s5.v[r];
  }
  R g[4][3];
  face_normals(x0, x1, x2, x3, g + 1);
#pragma unroll
  for (int d = 0; d < 3; ++d) g[0][d] = -(g[1][d] + g[2][d] + g[3][d]);
  R w = (R)(frac_of(code) / 36.0);
#pragma unroll
  for (int l = 0; l < 4; ++l) {
    R gx = g[l][0], gy = g[l][1], gz = g[l][2];
    out[l][0] = w * (gx * sg[0] + gy * sg[3] + gz * sg[5]);
    out[l][1] = w * (gy * sg[1] + gx * sg[3] + gz * sg[4]);
    out[l][2] = w * (gz * sg[2] + gy * sg[4] + gx * sg[5]);
  }
}

// One nodal force term per node-list entry: three values of R, packed (a
// quarter less traffic than padding to four for the float64 terms, the same
// speed for float32).
template <class R>
__device__ __forceinline__ void put_term(R* __restrict__ contrib, int p, R x, R y, R z) {
  R* q = contrib + 3 * (size_t)p;
  q[0] = x;
  q[1] = y;
  q[2] = z;
}
template <class R>
__device__ __forceinline__ void get_term(const R* __restrict__ contrib, int p, R& x, R& y, R& z) {
  const R* q = contrib + 3 * (size_t)p;
  x = q[0];
  y = q[1];
  z = q[2];
}

// Store the four nodal terms at the element's positions in the node lists.
template <class R>
__device__ __forceinline__ void store_terms(R* __restrict__ contrib, int4 pos, const R out[4][3]) {
  put_term(contrib, pos.x, out[0][0], out[0][1], out[0][2]);
  put_term(contrib, pos.y, out[1][0], out[1][1], out[1][2]);
  put_term(contrib, pos.z, out[2][0], out[2][1], out[2][2]);
  put_term(contrib, pos.w, out[3][0], out[3][1], out[3][2]);
}

// Tetrahedra: node i's force from its (tet, local) entries, each term
// G_l^T s_e formed from the tet's weighted stress sum s_e and
// G_l = 6 V grad N_l = (X_b - X_a) x (X_c - X_a) over the face (a, b, c)
// opposite corner l, oriented as G_1 = c2 x c3, G_2 = c3 x c1, G_3 = c1 x c2
// (c_j = X_j - X_0) and G_0 = (X_3 - X_1) x (X_2 - X_1).  Coordinate
// differences in float64; lanes and sum order as node_gather.
template <class R, int G>
__device__ __forceinline__ void node_gather_tet(const Mesh& m, const R* __restrict__ ts, int i,
                                                bool active, int g, double& fx, double& fy,
                                                double& fz) {
  fx = fy = fz = 0;
  const int p0 = active ? m.noff[i] : 0, p1 = active ? m.noff[i + 1] : 0;
  CEM_PRAGMA(unroll CEM_NODE_UNROLL)
  for (int p = p0 + g; p < p1; p += G) {
    const int ent = m.nent[p], e = ent >> 2, l = ent & 3;
    const int4 nd = m.enodes[e];
    const int n0 = nd.x & kNodeMask;
    const int na = l == 0 ? nd.y : n0;
    const int nb = l == 0 ? nd.w : l == 1 ? nd.z : l == 2 ? nd.w : nd.y;
    const int nc = l == 0 ? nd.z : l == 1 ? nd.w : l == 2 ? nd.y : nd.z;
    const double4 xa = m.X[na], xb = m.X[nb], xc = m.X[nc];
    Six<R> s = load6((const Six<R>*)ts + e);
    const R bx = (R)(xb.x - xa.x), by = (R)(xb.y - xa.y), bz = (R)(xb.z - xa.z);
    const R cx = (R)(xc.x - xa.x), cy = (R)(xc.y - xa.y), cz = (R)(xc.z - xa.z);
    const R gx = by * cz - bz * cy, gy = bz * cx - bx * cz, gz = bx * cy - by * cx;
    fx += (double)(gx * s.v[0] + gy * s.v[3] + gz * s.v[5]);
    fy += (double)(gy * s.v[1] + gx * s.v[3] + gz * s.v[4]);
    fz += (double)(gz * s.v[2] + gy * s.v[4] + gx * s.v[5]);
  }
#pragma unroll
  for (int off = G / 2; off > 0; off >>= 1) {
    fx += __shfl_xor(fx, off, G);
    fy += __shfl_xor(fy, off, G);
    fz += __shfl_xor(fz, off, G);
  }
}

// Sum of node i's contiguous terms by G lanes (lane g takes entries g, g + G,
// ...), combined by a fixed butterfly of shuffles, so the sum is the same on
// every run.  Every lane of the group must call it.
template <class R, int G>
__device__ __forceinline__ void node_gather(const Mesh& m, const R* __restrict__ contrib, int i,
                                            bool active, int g, double& fx, double& fy,
                                            double& fz) {
  fx = fy = fz = 0;
  const int p0 = active ? m.noff[i] : 0, p1 = active ? m.noff[i + 1] : 0;
  CEM_PRAGMA(unroll CEM_NODE_UNROLL)
  for (int p = p0 + g; p < p1; p += G) {
    R qx, qy, qz;
    get_term(contrib, p, qx, qy, qz);
    fx += (double)qx;
    fy += (double)qy;
    fz += (double)qz;
  }
#pragma unroll
  for (int off = G / 2; off > 0; off >>= 1) {
    fx += __shfl_xor(fx, off, G);
    fy += __shfl_xor(fy, off, G);
    fz += __shfl_xor(fz, off, G);
  }
}

// Prescribed-velocity history with ramp time t0: the velocity factor
// V(t) = t / t0 up to t0, then 1 (t0 = 0: 1 from the start), its integral S
// and its derivative A (taken on the ramp at t = t0).
__device__ __forceinline__ void bc_history(double t0, double t, double& S, double& V, double& A) {
  if (t0 > 0 && t <= t0) {
    S = t * t / (2.0 * t0);
    V = t / t0;
    A = 1.0 / t0;
  } else {
    S = t0 > 0 ? t - 0.5 * t0 : t;
    V = 1.0;
    A = 0.0;
  }
}

// Largest eigenvalue of a symmetric 6 x 6 matrix by cyclic Jacobi rotations
// (A is overwritten).
__device__ __forceinline__ double jacobi_lmax6(double A[6][6]) {
  for (int sweep = 0; sweep < 30; ++sweep) {
    double off = 0, dg = 0;
#pragma unroll
    for (int p = 0; p < 6; ++p) {
      dg += A[p][p] * A[p][p];
#pragma unroll
      for (int q = p + 1; q < 6; ++q) off += A[p][q] * A[p][q];
    }
    if (off <= 1e-36 * dg) break;
#pragma unroll
    for (int p = 0; p < 6; ++p)
#pragma unroll
      for (int q = p + 1; q < 6; ++q) {
        double apq = A[p][q];
        if (apq != 0.0) {
          double theta = (A[q][q] - A[p][p]) / (2.0 * apq);
          double tt = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
          double cs = 1.0 / sqrt(tt * tt + 1.0), sn = tt * cs;
#pragma unroll
          for (int k = 0; k < 6; ++k) {
            double akp = A[k][p], akq = A[k][q];
            A[k][p] = cs * akp - sn * akq;
            A[k][q] = sn * akp + cs * akq;
          }
#pragma unroll
          for (int k = 0; k < 6; ++k) {
            double apk = A[p][k], aqk = A[q][k];
            A[p][k] = cs * apk - sn * aqk;
            A[q][k] = sn * apk + cs * aqk;
          }
        }
      }
  }
  double lmax = 0;
#pragma unroll
  for (int i = 0; i < 6; ++i) lmax = fmax(lmax, A[i][i]);
  return lmax;
}

// Persistent grid: enough workgroups for the largest item count the launch
// can see (capacity), capped at m.grid_cap; always a multiple of 8.
static inline int persistent_grid(const Mesh& m, long long items) {
  long long g = (items + kBlock - 1) / kBlock;
  g = g < 8 ? 8 : g;
  g = g > m.grid_cap ? m.grid_cap : g;
  return (int)((g + 7) / 8 * 8);
}

// One Jacobi rotation in the (p, q) plane of the symmetric 3x3 tensor a, with
// the tangent of the stable 2x2 symmetric Schur decomposition (Golub and Van
// Loan, the classical Jacobi method): a_pq becomes 0, the diagonal moves by
// t a_pq, the third row/column and the columns p, q of v rotate.
template <int p, int q>
__device__ __forceinline__ void jacobi_rot(double (&a)[3][3], double (&v)[3][3]) {
  constexpr int r = 3 - p - q;
  double apq = a[p][q];
  if (apq == 0.0) return;
  double th = (a[q][q] - a[p][p]) / (2.0 * apq);
  double t = fabs(th) > 1e150 ? 0.5 / th
                               : (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
  double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
  a[p][p] -= t * apq;
  a[q][q] += t * apq;
  a[p][q] = a[q][p] = 0.0;
  double arp = a[r][p], arq = a[r][q];
  a[r][p] = a[p][r] = c * arp - s * arq;
  a[r][q] = a[q][r] = s * arp + c * arq;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    double vp = v[k][p], vq = v[k][q];
    v[k][p] = c * vp - s * vq;
    v[k][q] = s * vp + c * vq;
  }
}

// Stress term of Eqs. G-I / G-II for the smoothed edge stress s (Voigt) and the
// unit crack normal n.  gsig 0: sigma_1 |P_1 n|, P_1 the projector on the
// eigenspace of the largest eigenvalue; eigenvalues within 1e-6 max|lambda| of
// it count as equal (two evaluations of one edge stress in different summation
// orders differ by rounding, and the eigenvector of a closer pair moves by that
// rounding over the gap).  The eigenpairs come from cyclic Jacobi sweeps,
// accurate to rounding for the eigenvalues and to rounding over the gap for
// the eigenvectors.  gsig 1: n . sigma . n.
__device__ inline double stress_term(const double* s, double nx, double ny, double nz, int gsig) {
  if (gsig == 1) {
    return nx * (s[0] * nx + s[3] * ny + s[5] * nz) + ny * (s[3] * nx + s[1] * ny + s[4] * nz) +
           nz * (s[5] * nx + s[4] * ny + s[2] * nz);
  }
  double a[3][3] = {{s[0], s[3], s[5]}, {s[3], s[1], s[4]}, {s[5], s[4], s[2]}};
  double v[3][3] = {{1.0, 0.0, 0.0}, {0.0, 1.0, 0.0}, {0.0, 0.0, 1.0}};
  for (int sweep = 0; sweep < 16; ++sweep) {
    double off = a[0][1] * a[0][1] + a[0][2] * a[0][2] + a[1][2] * a[1][2];
    double dia = a[0][0] * a[0][0] + a[1][1] * a[1][1] + a[2][2] * a[2][2];
    if (!(off > 1e-36 * dia)) break;
    jacobi_rot<0, 1>(a, v);
    jacobi_rot<0, 2>(a, v);
    jacobi_rot<1, 2>(a, v);
  }
  double w[3] = {a[0][0], a[1][1], a[2][2]};
  double lmax = fmax(w[0], fmax(w[1], w[2]));
  double amax = fmax(fabs(w[0]), fmax(fabs(w[1]), fabs(w[2])));
  double gap = 1e-6 * amax;
  double p2 = 0.0;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    double c = v[0][i] * nx + v[1][i] * ny + v[2][i] * nz;
    if (w[i] >= lmax - gap) p2 += c * c;
  }
  return lmax * sqrt(p2);
}

template <class R> __device__ __forceinline__ void load_sig(const Six<R>* esig, int k, double* s) {
  Six<R> v = load6(esig + k);
#pragma unroll
  for (int i = 0; i < 6; ++i) s[i] = (double)v.v[i];
}

}  // namespace cem

#endif
