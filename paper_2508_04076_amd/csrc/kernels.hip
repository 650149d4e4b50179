// HIP kernels (gfx950) of the ES-T-FEM crack-element step.
//
// One explicit step is a chain of gather passes with no floating-point
// atomics, so results are deterministic:
//   strain      per element slot: V_eff * eps_e = V_eff B_e u_e          (6 values)
//   edge_stress per edge: eps_k = sum_patch(V_eff eps) / sum_patch V_eff, sigma_k = C eps_k
//   elem_force  per element: its four nodal force terms; extra workgroups of
//               the same launch take the crack-front candidates (G_I, G_II,
//               Griffith test, flags appended to the split list)
//   node        per node: f_i = sum_{(e,l) ni i} (V_eff,e / 6) B_{e,l}^T sum_{k in edges(e)} sigma_k,
//               then the Newmark update
//   topology    one workgroup sorts the flags and applies the step's splits
// The node force uses the identity
//   sum_k V_k Bt_k^T sigma_k = sum_e (V_eff,e / 6) B_e^T sum_{k in edges(e)} sigma_k
// (Bt_k = sum_patch w_ek B_e, V_k = (1/6) sum_patch V_eff, w_ek V_k = V_eff,e / 6),
// which turns the edge-smoothed force of Eq. CSTet_fint_discretization into
// a node-ordered gather.  Gradients are not stored: V grad N_l is a face
// cross product over 6, so no element needs a determinant or a division.
#include "hex_crack.h"

#ifndef CEM_WPE_STRAIN
#define CEM_WPE_STRAIN 1
#endif
#ifndef CEM_WPE_EDGE
#define CEM_WPE_EDGE 1
#endif
#ifndef CEM_WPE_ELEM
#define CEM_WPE_ELEM 1
#endif
#ifndef CEM_WPE_NODE
#define CEM_WPE_NODE 1
#endif

namespace cem {

// local edge q of a tet joins local nodes (kEA[q], kEB[q])
__device__ __constant__ int kEA[6] = {0, 0, 0, 1, 1, 2};
__device__ __constant__ int kEB[6] = {1, 2, 3, 2, 3, 3};
__device__ __forceinline__ int local_edge(int a, int b) {
  int lo = a < b ? a : b, hi = a < b ? b : a;
  return lo == 0 ? hi - 1 : (lo == 1 ? hi + 1 : 5);
}

__device__ __forceinline__ double tet_volume(double4 x0, double4 x1, double4 x2, double4 x3) {
  double ax = x1.x - x0.x, ay = x1.y - x0.y, az = x1.z - x0.z;
  double bx = x2.x - x0.x, by = x2.y - x0.y, bz = x2.z - x0.z;
  double cx = x3.x - x0.x, cy = x3.y - x0.y, cz = x3.z - x0.z;
  return (ax * (by * cz - bz * cy) + ay * (bz * cx - bx * cz) + az * (bx * cy - by * cx)) / 6.0;
}

__device__ __forceinline__ double elem_volume(const Mesh& m, int4 nd) {
  int n0 = nd.x & kNodeMask;
  return tet_volume(m.X[n0], m.X[nd.y], m.X[nd.z], m.X[nd.w]);
}

// ---------------------------------------------------------------- strain pass

// V_eff eps_e = (frac / 6) sum_{l=1..3} sym(g_l (x) (u_l - u_0)),
// g_1 = c2 x c3, g_2 = c3 x c1, g_3 = c1 x c2, c_l = X_l - X_0 (g_l = 6 V grad N_l).
// Differences are taken in float64 before any conversion to R.
template <class R>
__global__ __launch_bounds__(kBlock, CEM_WPE_STRAIN) void k_strain(Mesh m, const double4* __restrict__ u,
                                                   Six<R>* __restrict__ veps,
                                                   const Counters* __restrict__ c) {
  if (c->err) return;
  // the edge pass that follows takes max |sigma| afresh (fixed-point tiles)
  if (m.tiled == 2 && blockIdx.x == 0 && threadIdx.x < kSigSlots) m.sig_slot[threadIdx.x * kSigStride] = 0;
  const int Tn = elems_now(m, c);
  Chunks it(Tn);
  for (int e; it.next(e);) {
  if (e >= Tn) continue;
  int4 nd = m.enodes[e];
  int code = (unsigned)nd.x >> kNodeBits;
  int n0 = nd.x & kNodeMask;
  R out[6] = {0, 0, 0, 0, 0, 0};
  if (code != FR_ZERO) {
    R g[3][3], d[3][3];
    slot_normals<R>(m, e, nd, g);
    node_diffs(u[n0], u[nd.y], u[nd.z], u[nd.w], d);
    sym_grad(g, d, (R)(frac_of(code) / 6.0), out);
  }
  store6(veps + e, out);
  }
}

// ---------------------------------------------------------------- edge stress pass

template <class R>
__global__ __launch_bounds__(kBlock, CEM_WPE_EDGE) void k_edge_stress(Mesh m, const Six<R>* __restrict__ veps,
                                                        const R* __restrict__ einvV,
                                                        Six<R>* __restrict__ esig,
                                                        const Counters* __restrict__ c) {
  if (c->err) return;
  const int En = edges_now(m, c);
  double smax = 0.0;  // max |sigma| component (scale of the fixed-point tiles)
  Chunks it(En);
  for (int k; it.next(k);) {
    if (k >= En) continue;
    R acc[6], eps[6], sig[6];
    edge_sum(m, veps, k, acc);
    R iv = einvV[k];
#pragma unroll
    for (int i = 0; i < 6; ++i) eps[i] = acc[i] * iv;
    hooke((R)m.lam, (R)m.mu, eps, sig);
    store6(esig + k, sig);
    if (m.tiled == 2)
#pragma unroll
      for (int i = 0; i < 6; ++i) smax = fmax(smax, fabs((double)sig[i]));
  }
  if (m.tiled == 2) {
    // one atomic per workgroup, on the slot of its residue: on a small mesh
    // every workgroup ends at once, and thousands of atomics on one address
    // would outlast the pass itself
    __shared__ double wmax[kBlock / 64];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) smax = fmax(smax, __shfl_xor(smax, off));
    if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = smax;
    __syncthreads();
    if (threadIdx.x == 0) {
      double b = wmax[0];
#pragma unroll
      for (int w = 1; w < kBlock / 64; ++w) b = fmax(b, wmax[w]);
      if (b > 0.0) atomicMax(m.sig_slot + (blockIdx.x % kSigSlots) * kSigStride, dkey(b));
    }
  }
}

// Strain energy 1/2 sum_k V_k sigma_k . eps_k; V_k eps_k = acc_k / 6.
template <class R>
__global__ __launch_bounds__(kBlock) void k_strain_energy(Mesh m, const Six<R>* __restrict__ veps,
                                                          const R* __restrict__ einvV,
                                                          double* __restrict__ partial,
                                                          const Counters* __restrict__ c,
                                                          int want) {
  __shared__ double red[kBlock];
  double s = 0;
  int En = edges_now(m, c);
  for (int k = blockIdx.x * kBlock + threadIdx.x; k < En; k += gridDim.x * kBlock) {
    if (want >= 0 && m.einst[k] != want) continue;
    R acc[6], eps[6], sig[6];
    edge_sum(m, veps, k, acc);
    R iv = einvV[k];
#pragma unroll
    for (int i = 0; i < 6; ++i) eps[i] = acc[i] * iv;
    hooke((R)m.lam, (R)m.mu, eps, sig);
    double d = 0;
#pragma unroll
    for (int i = 0; i < 6; ++i) d += (double)sig[i] * (double)acc[i];
    s += 0.5 * d / (m.etype == 8 ? 12.0 : 6.0);  // V_k = S_k / 6 (tets), S_k / 12 (hexes)
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// ---------------------------------------------------------------- node pass

// Element force pass: for element e with effective volume fraction f,
//   c_{e,l} = (V_eff / 6) B_l^T sum_{k in edges(e)} sigma_k = (f / 36) G_l^T s,
// G_l = 6 V grad N_l (face cross products).  Two layouts of what the node
// pass receives (chosen per context, Mesh::ssum):
//  - terms (default): the four 3-vectors at the element's positions in the
//    node lists (epos), so the node pass reads each node's terms contiguously;
//  - stress sums: s_e = (f / 36) s, one coalesced row per element, and the
//    node pass forms G_l^T s_e itself from the corner coordinates.  Fewer
//    bytes written, more gathered: faster where the coordinates and element
//    rows stay in cache and the terms are wide (float64).
// More tets flagged than split capacity left: raise the error before the
// force passes touch the state, so it stays at the start of the step.
__device__ __forceinline__ bool over_capacity(const Mesh& m, Counters* c) {
  if (c->n_flag <= m.S_cap - c->n_split) return false;
  if (blockIdx.x == 0 && threadIdx.x == 0) c->err = -5;
  return true;
}

template <class R>
__device__ __forceinline__ void elem_force_items(const Mesh& m, const Six<R>* __restrict__ esig,
                                                 R* __restrict__ contrib,
                                                 const Counters* __restrict__ c, int nblocks,
                                                 int b0) {
  const int Tn = elems_now(m, c);
  Chunks it(Tn, nblocks, b0);
  for (int e; it.next(e);) {
  if (e >= Tn) continue;
  int4 nd = m.enodes[e];
  int code = (unsigned)nd.x >> kNodeBits;
  if (m.ssum) {
    R sg[6] = {0, 0, 0, 0, 0, 0};
    if (code != FR_ZERO) elem_ssum(m, e, code, esig, sg);
    store6((Six<R>*)contrib + e, sg);
    continue;
  }
  int4 pos = m.epos[e];
  R out[4][3];
  if (code == FR_ZERO) {
#pragma unroll
    for (int l = 0; l < 4; ++l) out[l][0] = out[l][1] = out[l][2] = 0;
  } else {
    elem_terms(m, e, nd, code, esig, out);
  }
  store_terms(contrib, pos, out);
  }
}

template <class R>
__global__ __launch_bounds__(kBlock, CEM_WPE_ELEM) void k_elem_force(Mesh m, const Six<R>* __restrict__ esig,
                                                       R* __restrict__ contrib,
                                                       Counters* __restrict__ c) {
  if (c->err || over_capacity(m, c)) return;
  elem_force_items(m, esig, contrib, c, 0, 0);
}

// Prescribed components of constrained slot b at time t: velocity v0 V(t),
// acceleration v0 A(t), the predictor for t_next from the history, and the
// reaction m a + f - r F on those components (0 on the free ones).
__device__ __forceinline__ void bc_override(const Mesh& m, int b, double t, double t_next,
                                            double im, double fx, double fy, double fz, double r,
                                            double4 F, double4& v, double4& a, double4& uh,
                                            double4& R) {
  const int mk = m.bmask[b];
  double S, V, A, S2, V2, A2;
  bc_history(m.gt0[mk >> 4], t, S, V, A);
  bc_history(m.gt0[mk >> 4], t_next, S2, V2, A2);
  const double4 w = m.bv0[b], ref = m.bref[b];
  const double mass = im > 0 ? 1.0 / im : 0.0;
  R = make_double4(0, 0, 0, 0);
  if (mk & 1) {
    v.x = w.x * V; a.x = w.x * A; uh.x = ref.x + w.x * S2;
    R.x = mass * a.x + fx - r * F.x;
  }
  if (mk & 2) {
    v.y = w.y * V; a.y = w.y * A; uh.y = ref.y + w.y * S2;
    R.y = mass * a.y + fy - r * F.y;
  }
  if (mk & 4) {
    v.z = w.z * V; a.z = w.z * A; uh.z = ref.z + w.z * S2;
    R.z = mass * a.z + fz - r * F.z;
  }
}

// Node pass: G lanes per node sum the node's contributions (lane g takes
// entries g, g + G, ...; a fixed butterfly of shuffles combines the lanes, so
// the sum is the same on every run), then the Newmark update.
// KIND: 0 = contiguous terms (tets or hexes), 2 = tet stress sums
// Newmark update of node i from its internal force f (MODE NODE_STEP), the
// initial acceleration (NODE_INIT) or f alone (NODE_FORCE); constrained
// components follow their prescribed history (BC).
template <int MODE, bool BC>
__device__ __forceinline__ void node_update(const Mesh& m, const State& st, double4* __restrict__ fout,
                                            Counters* __restrict__ c, int i, double fx, double fy,
                                            double fz) {
  if (MODE == NODE_FORCE) {
    fout[i] = make_double4(fx, fy, fz, 0.0);
    return;
  }
  const double dt = node_dt(m, i);
  const long long n = c->step;
  int ls = m.lslot[i];
  double4 F = ls >= 0 ? m.Fload[ls] : make_double4(0, 0, 0, 0);
  double im = m.invm[i];
  const int bs = BC ? m.bslot[i] : -1;
  if (MODE == NODE_INIT) {
    const double t = (double)n * dt;
    double r = ramp(m, t);
    double4 u0 = st.u[i], v0 = st.v[i];
    double ax = (r * F.x - fx) * im, ay = (r * F.y - fy) * im, az = (r * F.z - fz) * im;
    double h = 0.5 * dt * dt;
    double4 uh = make_double4(u0.x + dt * v0.x + h * ax, u0.y + dt * v0.y + h * ay,
                              u0.z + dt * v0.z + h * az, 0.0);
    if (bs >= 0) {
      double4 vv = v0, aa = make_double4(ax, ay, az, 0.0), rc;
      bc_override(m, bs, t, t + dt, im, fx, fy, fz, r, F, vv, aa, uh, rc);
      st.v[i] = vv;
      ax = aa.x; ay = aa.y; az = aa.z;
      m.breact[bs] = rc;
    }
    st.a[i] = make_double4(ax, ay, az, 0.0);
    st.uh[i] = uh;
    return;
  }
  // NODE_STEP: f was evaluated at u_{n+1} = uh
  double r0 = ramp(m, (double)n * dt), r1 = ramp(m, (double)(n + 1) * dt);
  double4 u1 = st.uh[i], v0 = st.v[i], a0 = st.a[i];
  double ax = (r1 * F.x - fx) * im, ay = (r1 * F.y - fy) * im, az = (r1 * F.z - fz) * im;
  double hdt = 0.5 * dt;
  double vx = v0.x + hdt * (a0.x + ax), vy = v0.y + hdt * (a0.y + ay), vz = v0.z + hdt * (a0.z + az);
  if (ls >= 0) {
    double4 u0 = st.u[i];
    m.wacc[ls] += 0.5 * (r0 + r1) * (F.x * (u1.x - u0.x) + F.y * (u1.y - u0.y) + F.z * (u1.z - u0.z));
  }
  double h = 0.5 * dt * dt;
  double4 uh = make_double4(u1.x + dt * vx + h * ax, u1.y + dt * vy + h * ay, u1.z + dt * vz + h * az,
                            0.0);
  if (bs >= 0) {
    // prescribed components: velocity, acceleration and the next predictor
    // from the history; the reaction and its work (trapezoid)
    double4 vv = make_double4(vx, vy, vz, 0.0), aa = make_double4(ax, ay, az, 0.0), rc;
    double t1 = (double)(n + 1) * dt;
    bc_override(m, bs, t1, t1 + dt, im, fx, fy, fz, r1, F, vv, aa, uh, rc);
    vx = vv.x; vy = vv.y; vz = vv.z;
    ax = aa.x; ay = aa.y; az = aa.z;
    double4 u0 = st.u[i], r0c = m.breact[bs];
    m.bwork[bs] += 0.5 * (r0c.x + rc.x) * (u1.x - u0.x) + 0.5 * (r0c.y + rc.y) * (u1.y - u0.y) +
                   0.5 * (r0c.z + rc.z) * (u1.z - u0.z);
    m.breact[bs] = rc;
  }
  st.u[i] = u1;
  st.v[i] = make_double4(vx, vy, vz, 0.0);
  st.a[i] = make_double4(ax, ay, az, 0.0);
  st.uh[i] = uh;
  bool bad = !(fabs(ax) <= DBL_MAX && fabs(ay) <= DBL_MAX && fabs(az) <= DBL_MAX) ||
             !(fabs(u1.x) <= m.umax && fabs(u1.y) <= m.umax && fabs(u1.z) <= m.umax);
  if (bad) atomicCAS(&c->err, 0, -6);
}

template <class R, int MODE, int G, bool BC, int KIND>
__global__ __launch_bounds__(kBlock, CEM_WPE_NODE) void k_node(Mesh m, State st, const R* __restrict__ contrib,
                                                 double4* __restrict__ fout,
                                                 Counters* __restrict__ c, int first) {
  if (c->err || over_capacity(m, c)) return;
  const int Nn = nodes_now(m, c);
  if (Nn <= first) return;
  Chunks it((long long)(Nn - first) * G);
  const int g = (int)threadIdx.x % G;
  for (int item; it.next(item);) {
    const int i = first + item / G;
    const bool active = i < Nn;
    double fx, fy, fz;
    if (KIND == 2) node_gather_tet<R, G>(m, contrib, i, active, g, fx, fy, fz);
    else node_gather<R, G>(m, contrib, i, active, g, fx, fy, fz);
    if (!active || g != 0) continue;
    node_update<MODE, BC>(m, st, fout, c, i, fx, fy, fz);
  }
}

// ---------------------------------------------------------------- crack pass


// Release rates of the front on local face `f` of intact tet c whose lone node
// (alone on its side of the neighbour's cut) is global node `lone`:
// N2 = lone, N4 = local node f, N1 < N3 the other face nodes (local order);
// stretches on N1N2 and N2N3 (Eq. stretch-delta: only lengthening edges),
// stresses at the edge points of N1N4, N3N4 (pattern I) and N2N4 (pattern II).
template <class R>
__device__ void front_rates(const Mesh& m, const double4* __restrict__ u,
                            const Six<R>* __restrict__ esig, const int* nd, const int* ed,
                            int f, int lone, double& GI, double& GII, int& maskI, int& maskII) {
  int l2 = -1, l1 = -1, l3 = -1;
  for (int l = 0; l < 4; ++l) {
    if (l == f) continue;
    if (nd[l] == lone) l2 = l;
    else if (l1 < 0) l1 = l;
    else l3 = l;
  }
  int l4 = f;
  if (l1 < 0 || l2 < 0 || l3 < 0) {  // the lone node is not on this face: no front
    GI = GII = -INFINITY;
    maskI = maskII = 0;
    return;
  }
  double4 X1 = m.X[nd[l1]], X2 = m.X[nd[l2]], X3 = m.X[nd[l3]], X4 = m.X[nd[l4]];
  double4 U1 = u[nd[l1]], U2 = u[nd[l2]], U3 = u[nd[l3]];
  // stretch of N1N2 and N2N3: 2 dX.du + |du|^2 > 0  <=>  |x_j - x_i| > |X_j - X_i|
  double d1x = U2.x - U1.x, d1y = U2.y - U1.y, d1z = U2.z - U1.z;
  double e1x = X2.x - X1.x, e1y = X2.y - X1.y, e1z = X2.z - X1.z;
  double s1 = 2.0 * (e1x * d1x + e1y * d1y + e1z * d1z) + (d1x * d1x + d1y * d1y + d1z * d1z);
  if (!(s1 > 0.0)) { d1x = 0; d1y = 0; d1z = 0; }
  double d2x = U3.x - U2.x, d2y = U3.y - U2.y, d2z = U3.z - U2.z;
  double e2x = X3.x - X2.x, e2y = X3.y - X2.y, e2z = X3.z - X2.z;
  double s2 = 2.0 * (e2x * d2x + e2y * d2y + e2z * d2z) + (d2x * d2x + d2y * d2y + d2z * d2z);
  if (!(s2 > 0.0)) { d2x = 0; d2y = 0; d2z = 0; }
  if (d1x == 0 && d1y == 0 && d1z == 0 && d2x == 0 && d2y == 0 && d2z == 0) {
    GI = GII = 0.0;  // neither front edge lengthens
    maskI = (1 << l2) | (1 << l4);
    maskII = (1 << l2);
    return;
  }
  // crack normals: pattern I plane spanned by N1N3 and N2N4, pattern II parallel to N1N3N4
  double ax = X3.x - X1.x, ay = X3.y - X1.y, az = X3.z - X1.z;
  double bx = X4.x - X2.x, by = X4.y - X2.y, bz = X4.z - X2.z;
  double cx = X4.x - X1.x, cy = X4.y - X1.y, cz = X4.z - X1.z;
  double nIx = ay * bz - az * by, nIy = az * bx - ax * bz, nIz = ax * by - ay * bx;
  double nn = sqrt(nIx * nIx + nIy * nIy + nIz * nIz);
  nIx /= nn; nIy /= nn; nIz /= nn;
  double nJx = ay * cz - az * cy, nJy = az * cx - ax * cz, nJz = ax * cy - ay * cx;
  nn = sqrt(nJx * nJx + nJy * nJy + nJz * nJz);
  nJx /= nn; nJy /= nn; nJz /= nn;
  double sg[6];
  load_sig(esig, ed[local_edge(l1, l4)], sg);
  double t3 = stress_term(sg, nIx, nIy, nIz, m.gsig);
  load_sig(esig, ed[local_edge(l3, l4)], sg);
  double t4 = stress_term(sg, nIx, nIy, nIz, m.gsig);
  load_sig(esig, ed[local_edge(l2, l4)], sg);
  double t6 = stress_term(sg, nJx, nJy, nJz, m.gsig);
  GI = 0.5 * (t3 * fabs(d1x * nIx + d1y * nIy + d1z * nIz) +
              t4 * fabs(d2x * nIx + d2y * nIy + d2z * nIz));
  GII = 0.5 * t6 * (fabs(d1x * nJx + d1y * nJy + d1z * nJz) + fabs(d2x * nJx + d2y * nJy + d2z * nJz));
  maskI = (1 << l2) | (1 << l4);
  maskII = (1 << l2);
}

template <class R>
__device__ __forceinline__ void load_tet(const Mesh& m, int t, int* nd, int* ed) {
  int4 q = m.enodes[t];
  nd[0] = q.x & kNodeMask; nd[1] = q.y; nd[2] = q.z; nd[3] = q.w;
  int2 a = m.et2e[3 * t], b = m.et2e[3 * t + 1], cc = m.et2e[3 * t + 2];
  ed[0] = a.x; ed[1] = a.y; ed[2] = b.x; ed[3] = b.y; ed[4] = cc.x; ed[5] = cc.y;
}

// Four lanes per candidate, one per local face: each evaluates its front (if
// any); lane 0 of the group then takes the best (G, face, pattern) in face
// order, ties to the lower face and to pattern I.  The Griffith test
// G >= Gc flags the tet: it is appended to the (unordered) split list.
template <class R>
__device__ void front_block(const Mesh& m, const double4* __restrict__ u,
                            const Six<R>* __restrict__ esig, Counters* __restrict__ c,
                            int flagging, int blk, int nblk, unsigned long long* red) {
  unsigned long long kmax = 0;
  const int nc = c->n_cand;
  const int room = m.S_cap - c->n_split;
  const int f = threadIdx.x & 3;
  constexpr int cpb = kBlock / 4;
  for (int base = blk * cpb; base < nc; base += nblk * cpb) {
    int idx = base + (int)threadIdx.x / 4;
    int t = idx < nc ? m.cand[idx] : -1;
    bool act = t >= 0 && m.smask[t] < 0;
    int lone = act ? ((const int*)m.front)[4 * t + f] : -1;
    double GI = -INFINITY, GII = -INFINITY;
    int mI = 0, mII = 0;
    if (lone >= 0) {
      int nd[4], ed[6];
      load_tet<R>(m, t, nd, ed);
      front_rates<R>(m, u, esig, nd, ed, f, lone, GI, GII, mI, mII);
    }
    double gI[4], gII[4];
    int mi[4], mii[4], has[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      gI[q] = __shfl(GI, q, 4);
      gII[q] = __shfl(GII, q, 4);
      mi[q] = __shfl(mI, q, 4);
      mii[q] = __shfl(mII, q, 4);
      has[q] = __shfl(lone, q, 4) >= 0;
    }
    if (f != 0 || !act) continue;
    double best = -INFINITY;
    int bmask = 0, bpat = 0;
    bool any = false;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if (!has[q]) continue;
      if (!any || gI[q] > best) { best = gI[q]; bmask = mi[q]; bpat = 1; }
      any = true;
      if (gII[q] > best) { best = gII[q]; bmask = mii[q]; bpat = 2; }
    }
    if (!any) continue;
    unsigned long long k = dkey(best);
    kmax = k > kmax ? k : kmax;
    if (m.n_inst) atomicMax(&m.gmax_inst[m.tinst[t]], k);
    if (flagging && best >= m.Gc) {
      m.pmask[t] = (uint8_t)bmask;
      m.ppat[t] = (uint8_t)bpat;
      m.pG[t] = best;
      int slot = atomicAdd(&c->n_flag, 1);
      if (slot < room) m.splitlist[slot] = t;  // unordered; the topology pass sorts
    }
  }
  red[threadIdx.x] = kmax;
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] = red[threadIdx.x] > red[threadIdx.x + w] ? red[threadIdx.x] : red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0 && red[0] != 0) atomicMax(&c->gmax_key, red[0]);
}

// Crack-front pass alone (the tiled force pass writes the state the front
// pass reads, so it cannot ride along with it).
template <class R>
__global__ __launch_bounds__(kBlock) void k_front(Mesh m, const Six<R>* __restrict__ esig,
                                                  const double4* __restrict__ uh,
                                                  Counters* __restrict__ c, int flagging) {
  if (c->err) return;
  __shared__ unsigned long long red[kBlock];
  front_block<R>(m, uh, esig, c, flagging, blockIdx.x, gridDim.x, red);
}

// Terms of element slot e into the tile's LDS when their node-list position
// lies in the tile's range [P0, P1); entries of extra nodes (positions past
// the original lists) go to the global term array, read by the node pass of
// the extra nodes.
template <class R>
__device__ __forceinline__ void tile_elem(const Mesh& m, int e, const Six<R>* __restrict__ esig,
                                          R* lds, int P0, int P1, R* __restrict__ contrib) {
  const int4 nd = m.enodes[e];
  const int code = (unsigned)nd.x >> kNodeBits;
  R out[4][3];
  if (code == FR_ZERO) {
#pragma unroll
    for (int l = 0; l < 4; ++l) out[l][0] = out[l][1] = out[l][2] = 0;
  } else {
    elem_terms(m, e, nd, code, esig, out);
  }
  const int4 pos = m.epos[e];
  const int ps[4] = {pos.x, pos.y, pos.z, pos.w};
  const int ext = 4 * m.T0;
#pragma unroll
  for (int l = 0; l < 4; ++l) {
    const int q = ps[l];
    if (q >= P0 && q < P1) {
      R* o = lds + 3 * (q - P0);
      o[0] = out[l][0];
      o[1] = out[l][1];
      o[2] = out[l][2];
    } else if (q >= ext) {
      put_term(contrib, q, out[l][0], out[l][1], out[l][2]);
    }
  }
}

// Tiled force pass (force and node update in one launch).  A workgroup owns a
// tile: consecutive original nodes (a Hilbert-compact block) whose node-list
// entries fit in its LDS (3,072 float64 or 12,288 float32 terms).  Phase 1 forms the nodal terms of every element
// slot with an entry in the tile (the tile's parent tets and the second copy
// of each split one) into LDS at the entries' list positions; phase 2 sums
// each node's entries from LDS in list order, G lanes per node with the
// butterfly of node_gather, and updates the node.  The terms and their sums
// are those of the term layout, so the results are the same bits; no term
// makes a round trip through memory.  Tiles are dealt to the XCDs in eight
// contiguous ranges.
template <class R, int MODE, int G, bool BC>
__global__ __launch_bounds__(tile_block<R>()) void k_force_tile(Mesh m, State st,
                                                           const Six<R>* __restrict__ esig,
                                                           R* __restrict__ contrib,
                                                           double4* __restrict__ fout,
                                                           Counters* __restrict__ c) {
  if (c->err || over_capacity(m, c)) return;
  constexpr int P = sizeof(R) == 8 ? 0 : 1;
  __shared__ R lds[3 * (P ? kTileEntries32 : kTileEntries64)];
  const int* __restrict__ toff = m.toff[P];
  const int* __restrict__ ttoff = m.ttoff[P];
  const int* __restrict__ ttet = m.ttet[P];
  const int ntile = m.ntile[P];
  const int x = (int)blockIdx.x % 8, j0 = (int)blockIdx.x / 8, stride = (int)gridDim.x / 8;
  const int b_hi = (int)((long long)ntile * (x + 1) / 8);
  const int g = (int)threadIdx.x % G;
  const bool phantom = m.mode == MODE_PHANTOM;
  for (int b = (int)((long long)ntile * x / 8) + j0; b < b_hi; b += stride) {
    const int n0 = toff[b], n1 = toff[b + 1];
    const int P0 = m.noff[n0], P1 = m.noff[n1];
    for (int jj = ttoff[b] + (int)threadIdx.x; jj < ttoff[b + 1]; jj += tile_block<R>()) {
      const int t = ttet[jj];
      tile_elem<R>(m, t, esig, lds, P0, P1, contrib);
      if (phantom) {
        const int code = (unsigned)m.enodes[t].x >> kNodeBits;
        if (code != FR_ONE) tile_elem<R>(m, m.T0 + m.split_of[t], esig, lds, P0, P1, contrib);
      }
    }
    __syncthreads();
    const int items = (n1 - n0) * G;
    for (int base = 0; base < items; base += tile_block<R>()) {
      const int item = base + (int)threadIdx.x;
      const int i = n0 + item / G;
      const bool active = item < items;
      double fx = 0, fy = 0, fz = 0;
      const int p0 = active ? m.noff[i] : 0, p1 = active ? m.noff[i + 1] : 0;
      for (int q = p0 + g; q < p1; q += G) {
        const R* o = lds + 3 * (q - P0);
        fx += (double)o[0];
        fy += (double)o[1];
        fz += (double)o[2];
      }
#pragma unroll
      for (int off = G / 2; off > 0; off >>= 1) {
        fx += __shfl_xor(fx, off, G);
        fy += __shfl_xor(fy, off, G);
        fz += __shfl_xor(fz, off, G);
      }
      if (active && g == 0) node_update<MODE, BC>(m, st, fout, c, i, fx, fy, fz);
    }
    __syncthreads();  // the next tile overwrites the LDS
  }
}

// Terms of element slot e into the 64-bit node sums of the fixed-point tile
// (nodes [n0, n1)): each term rounded to a multiple of 1 / S and added as an
// integer, so the sums do not depend on the order of the additions; terms
// of extra nodes go to the global term array.
template <class R>
__device__ __forceinline__ void fx_elem(const Mesh& m, int e, const Six<R>* __restrict__ esig,
                                        unsigned long long* acc, int n0, int n1, double S,
                                        R* __restrict__ contrib) {
  const int4 nd = m.enodes[e];
  const int code = (unsigned)nd.x >> kNodeBits;
  if (code == FR_ZERO) return;
  R out[4][3];
  elem_terms(m, e, nd, code, esig, out);
  const int ns[4] = {nd.x & kNodeMask, nd.y, nd.z, nd.w};
#pragma unroll
  for (int l = 0; l < 4; ++l) {
    const int i = ns[l];
    if (i >= n0 && i < n1) {
      unsigned long long* a = acc + 3 * (i - n0);
#pragma unroll
      for (int d = 0; d < 3; ++d) atomicAdd(a + d, (unsigned long long)__double2ll_rn((double)out[l][d] * S));
    } else if (i >= m.N0) {  // an extra node of a split copy: its single entry
      const int4 pos = m.epos[e];
      put_term(contrib, l == 0 ? pos.x : l == 1 ? pos.y : l == 2 ? pos.z : pos.w, out[l][0], out[l][1],
               out[l][2]);
    }
  }
}

// Fixed-point tiled force pass: a workgroup owns a tile of up to kFxNodes
// consecutive original nodes and keeps one 64-bit sum per node and component
// in LDS.  Phase 1 adds the terms of every element slot with a node in the
// tile (integer additions: the result does not depend on their order, so
// any assignment of elements to threads gives the same bits); phase 2
// converts each node's sums and updates the node.  The scale S = 2^k is the
// largest power of two with (longest node list) * |term bound| * S < 2^61,
// the bound |G_l|_1 max |sigma| / 6 from the edge pass's max |sigma|: each
// term is kept to 2^-k, far below its own rounding at the bound's scale.
// With no per-entry slots a tile holds more nodes than the term-slot tiles
// (1,536 against 128 or 512), so fewer tets are formed twice on tile borders,
// and its LDS is small enough for several workgroups per CU.
template <class R, int MODE, bool BC>
__global__ __launch_bounds__(kFxBlock) void k_force_fx(Mesh m, State st,
                                                       const Six<R>* __restrict__ esig,
                                                       R* __restrict__ contrib,
                                                       double4* __restrict__ fout,
                                                       Counters* __restrict__ c) {
  if (c->err || over_capacity(m, c)) return;
  __shared__ unsigned long long acc[3 * kFxNodes];
  static_assert(kSigSlots == 64, "one wave reduces the slots");
  unsigned long long key = m.sig_slot[(threadIdx.x & 63) * kSigStride];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const unsigned long long o = __shfl_xor(key, off);
    key = o > key ? o : key;
  }
  const double bound = key ? m.fx_g1 * key_to_double(key) / 6.0 * (double)m.fx_deg : 0.0;
  int ex = 0;
  if (bound > 0.0) (void)frexp(bound, &ex);  // bound < 2^ex
  const double S = ldexp(1.0, 61 - ex), iS = ldexp(1.0, ex - 61);
  const int x = (int)blockIdx.x % 8, j0 = (int)blockIdx.x / 8, stride = (int)gridDim.x / 8;
  const int b_hi = (int)((long long)m.ntile_fx * (x + 1) / 8);
  const bool phantom = m.mode == MODE_PHANTOM;
  for (int b = (int)((long long)m.ntile_fx * x / 8) + j0; b < b_hi; b += stride) {
    const int n0 = m.toff_fx[b], n1 = m.toff_fx[b + 1];
    for (int q = (int)threadIdx.x; q < 3 * (n1 - n0); q += kFxBlock) acc[q] = 0ull;
    __syncthreads();
    for (int jj = m.ttoff_fx[b] + (int)threadIdx.x; jj < m.ttoff_fx[b + 1]; jj += kFxBlock) {
      const int t = m.ttet_fx[jj];
      fx_elem<R>(m, t, esig, acc, n0, n1, S, contrib);
      if (phantom) {
        const int code = (unsigned)m.enodes[t].x >> kNodeBits;
        if (code != FR_ONE) fx_elem<R>(m, m.T0 + m.split_of[t], esig, acc, n0, n1, S, contrib);
      }
    }
    __syncthreads();
    for (int i = n0 + (int)threadIdx.x; i < n1; i += kFxBlock) {
      const unsigned long long* a = acc + 3 * (i - n0);
      node_update<MODE, BC>(m, st, fout, c, i, (double)(long long)a[0] * iS,
                            (double)(long long)a[1] * iS, (double)(long long)a[2] * iS);
    }
    __syncthreads();  // the next tile clears the sums
  }
}

// The element force pass and the crack-front pass in one launch: the first fg
// workgroups (dispatched first, so they run beside the element workgroups
// instead of after them) take the crack-front candidates, the others the
// elements.  Both read the edge stresses and write disjoint data; the
// capacity test on the flags is left to the node pass, which runs after both.
template <class R>
__global__ __launch_bounds__(kBlock, CEM_WPE_ELEM) void k_elem_force_front(
    Mesh m, const Six<R>* __restrict__ esig, R* __restrict__ contrib,
    const double4* __restrict__ uh, Counters* __restrict__ c, int fg, int flagging) {
  if (c->err) return;
  __shared__ unsigned long long red[kBlock];
  if ((int)blockIdx.x < fg) {
    front_block<R>(m, uh, esig, c, flagging, blockIdx.x, fg, red);
    return;
  }
  elem_force_items(m, esig, contrib, c, (int)gridDim.x - fg, fg);
}

// Readback of every front's G_I and G_II (unordered; the host sorts).
template <class R>
__global__ __launch_bounds__(kBlock) void k_front_eval(Mesh m, const double4* __restrict__ u,
                                                       const Six<R>* __restrict__ esig,
                                                       const Counters* __restrict__ c, int* out_tfl,
                                                       double* out_g, int* out_n) {
  int nc = c->n_cand;
  for (int idx = blockIdx.x * kBlock + threadIdx.x; idx < nc; idx += gridDim.x * kBlock) {
    int t = m.cand[idx];
    if (m.smask[t] >= 0) continue;
    int4 fr = m.front[t];
    int frs[4] = {fr.x, fr.y, fr.z, fr.w};
    int nd[4], ed[6];
    load_tet<R>(m, t, nd, ed);
    for (int f = 0; f < 4; ++f) {
      if (frs[f] < 0) continue;
      double GI, GII;
      int mI, mII;
      front_rates<R>(m, u, esig, nd, ed, f, frs[f], GI, GII, mI, mII);
      int o = atomicAdd(out_n, 1);
      out_tfl[3 * o] = t;
      out_tfl[3 * o + 1] = f;
      out_tfl[3 * o + 2] = frs[f];
      out_g[2 * o] = GI;
      out_g[2 * o + 1] = GII;
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_count_fronts(Mesh m, const Counters* __restrict__ c,
                                                         int* out, int want) {
  int nc = c->n_cand;
  int cnt = 0;
  for (int idx = blockIdx.x * kBlock + threadIdx.x; idx < nc; idx += gridDim.x * kBlock) {
    int t = m.cand[idx];
    if (m.smask[t] >= 0) continue;
    if (want >= 0 && m.tinst[t] != want) continue;
    if (m.etype == 8) {
      for (int f = 0; f < 6; ++f) cnt += m.hfront[6 * t + f] >= 0;
      continue;
    }
    int4 fr = m.front[t];
    cnt += (fr.x >= 0) + (fr.y >= 0) + (fr.z >= 0) + (fr.w >= 0);
  }
  if (cnt) atomicAdd(out, cnt);
}

// ---------------------------------------------------------------- forced schedule

// Forced schedule: the entries of the coming step, already sorted by tet.
__global__ void k_replay_select(Mesh m, Counters* __restrict__ c) {
  if (threadIdx.x != 0 || c->err) return;
  int cur = c->replay_cursor;
  int next = (int)(c->step + 1);
  while (cur < c->n_sched && m.sched[3 * cur] < next) cur++;
  int n = 0, prev = -1;
  while (cur < c->n_sched && m.sched[3 * cur] == next) {
    int t = m.sched[3 * cur + 1];
    int mk = m.sched[3 * cur + 2];
    cur++;
    if (t == prev || t < 0 || t >= m.T0 || m.smask[t] >= 0) continue;
    prev = t;
    if (c->n_split + n >= m.S_cap) { c->err = -5; break; }
    m.splitlist[n++] = t;
    m.pmask[t] = (uint8_t)mk;
    m.ppat[t] = __popc(mk) == 2 ? 1 : 2;
    m.pG[t] = 0.0;
  }
  c->replay_cursor = cur;
  c->n_flag = n;
}

__global__ void k_set_presplit(Mesh m, Counters* __restrict__ c, const int* tets,
                               const uint8_t* masks, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    int t = tets[i];
    m.splitlist[i] = t;
    m.pmask[t] = masks[i];
    m.ppat[t] = 0;
    m.pG[t] = 0.0;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) c->n_flag = n;
}

// ---------------------------------------------------------------- topology

__device__ __forceinline__ int code_for_side(int nodes_on_side) {
  return nodes_on_side == 1 ? FR_EIGHTH : nodes_on_side == 3 ? FR_SEVEN8 : FR_HALF;
}

// Element l of four values (select chain: no indexed local array).
template <class T>
__device__ __forceinline__ T pick4(T a, T b, T c, T d, int l) {
  return l == 0 ? a : l == 1 ? b : l == 2 ? c : d;
}

// Area of the midpoint crack surface of a 2|2 cut (Varignon parallelogram) or
// a 1|3 cut (corner triangle).  Corner indices from the mask's bits.
__device__ __forceinline__ double crack_area(const Mesh& m, const int* nd, int mask) {
  const double4 x0 = m.X[nd[0]], x1 = m.X[nd[1]], x2 = m.X[nd[2]], x3 = m.X[nd[3]];
  const int nb = __popc(mask);
  int i0, i1, j0, j1;
  double f;
  if (nb == 2) {
    // edge A0A1 (nodes off the mask) and edge B0B1 (nodes on it)
    const int a = ~mask & 15;
    i0 = __ffs(a) - 1;
    i1 = 31 - __clz(a);
    j0 = __ffs(mask) - 1;
    j1 = 31 - __clz(mask);
    f = 0.25;
  } else {
    // the three corners of the larger side: q0 q1 and q0 q2
    int big = nb == 1 ? (~mask & 15) : mask;
    i0 = __ffs(big) - 1;
    big &= big - 1;
    i1 = __ffs(big) - 1;
    big &= big - 1;
    j1 = __ffs(big) - 1;
    j0 = i0;
    f = 0.125;
  }
  const double4 p0 = pick4(x0, x1, x2, x3, i0), p1 = pick4(x0, x1, x2, x3, i1);
  const double4 r0 = pick4(x0, x1, x2, x3, j0), r1 = pick4(x0, x1, x2, x3, j1);
  const double ax = p1.x - p0.x, ay = p1.y - p0.y, az = p1.z - p0.z;
  const double bx = r1.x - r0.x, by = r1.y - r0.y, bz = r1.z - r0.z;
  const double cx = ay * bz - az * by, cy = az * bx - ax * bz, cz = ax * by - ay * bx;
  return f * sqrt(cx * cx + cy * cy + cz * cz);
}

// Sort of the n tets in list[0, n) by one workgroup, ascending in the
// caller's tet id key[t] (unique): rank sort in LDS up to kSortLds tets, else a
// bitonic sort in global memory over list[0, P) (P = next power of two, padded
// with -1 entries that sort last; the list has room).
constexpr int kSortLds = 2048;

__device__ __forceinline__ int sort_key(const int* key, int t) { return t < 0 ? 0x7fffffff : key[t]; }

__device__ void block_sort(int* list, int n, const int* key, int* shk, int* shv) {
  const int tid = threadIdx.x;
  if (n <= 1) return;
  if (n <= kSortLds) {
    for (int i = tid; i < n; i += kTopoBlock) {
      int t = list[i];
      shv[i] = t;
      shk[i] = key[t];
    }
    __syncthreads();
    for (int i = tid; i < n; i += kTopoBlock) {
      int v = shk[i], r = 0;
      for (int j = 0; j < n; ++j) r += shk[j] < v;
      list[r] = shv[i];
    }
    __threadfence_block();
    __syncthreads();
    return;
  }
  int P = 1;
  while (P < n) P <<= 1;
  for (int i = n + tid; i < P; i += kTopoBlock) list[i] = -1;
  __threadfence_block();
  __syncthreads();
  for (int k = 2; k <= P; k <<= 1)
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = tid; i < P; i += kTopoBlock) {
        int ixj = i ^ j;
        if (ixj > i) {
          int a = list[i], b = list[ixj];
          bool up = (i & k) == 0;
          if ((sort_key(key, a) > sort_key(key, b)) == up) {
            list[i] = b;
            list[ixj] = a;
          }
        }
      }
      __threadfence_block();
      __syncthreads();
    }
}

// Sum over groups of G consecutive lanes by a fixed butterfly (every lane of a
// group must take part).
template <int G>
__device__ __forceinline__ double group_sum(double v) {
#pragma unroll
  for (int off = G / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, G);
  return v;
}

// Phase 2 of a split batch (global split indices base .. base + n): lumped
// masses of the touched nodes (16 lanes per node list) and volumes of the
// touched edges (8 lanes per patch), each a fixed-order group sum, so the
// result does not depend on which threads run it.  Thread gtid of gthreads (a
// multiple of the group width; every lane of a group takes part).
template <class R>
__device__ void topo_masses(const Mesh& m, const int4* __restrict__ snodes, int base, int n,
                            int gtid, int gthreads) {
  if (m.mode != MODE_PHANTOM) return;
  constexpr int GN = 16;
  const int gl = gtid % GN;
  for (int item = gtid / GN; item < 4 * n; item += gthreads / GN) {
    int i = item >> 2, l = item & 3;
    int4 q4 = snodes[i];
    int node = l == 0 ? q4.x : l == 1 ? q4.y : l == 2 ? q4.z : q4.w;
    double part = 0;
    for (int p = m.noff[node] + gl; p < m.noff[node + 1]; p += GN) {
      int e = m.nent[p] >> 2;
      part += m.rho * frac_of((unsigned)m.enodes[e].x >> kNodeBits) * m.vol[e] / 4.0;
    }
    part = group_sum<GN>(part);
    if (gl == 0) m.invm[node] = part > 0 ? 1.0 / part : 0.0;
    if (gl == 1) {
      int t = m.splitlist[i];
      int mask = m.pmask[t];
      int nbB = __popc(mask);
      bool onB = (mask >> l) & 1;
      // the extra node of l belongs to the copy of the other side
      double fo = frac_of(code_for_side(onB ? 4 - nbB : nbB));
      m.invm[m.N0 + 4 * (base + i) + l] = 1.0 / (m.rho * fo * m.vol[t] / 4.0);
    }
  }
}

template <class R>
__device__ void topo_volumes(const Mesh& m, R* __restrict__ einvV, const int* __restrict__ sedges,
                             int n, int gtid, int gthreads) {
  constexpr int GE = 8;
  const int gl = gtid % GE;
  for (int item = gtid / GE; item < 6 * n; item += gthreads / GE) {
    int k = sedges[item];
    double part = 0, partk = 0;
    for (int p = m.poff[k] + gl; p < m.poff[k + 1]; p += GE) {
      int e = m.pent[p];
      if (e < 0) continue;
      double ve = frac_of((unsigned)m.enodes[e].x >> kNodeBits) * m.vol[e];
      part += ve;
      if (m.kap) partk += ve * m.kap[e];
    }
    part = group_sum<GE>(part);
    if (m.kap) partk = group_sum<GE>(partk);
    if (gl == 0)
      einvV[k] = !(part > 0) ? (R)0 : m.kap ? (R)(partk / part / part) : (R)(1.0 / part);
  }
}

// Phase 3: new crack fronts on intact face neighbours, one lane per face.
__device__ void topo_fronts(const Mesh& m, Counters* __restrict__ c,
                            const int4* __restrict__ snodes, int n, int gtid, int gthreads) {
  for (int item = gtid; item < 4 * n; item += gthreads) {
    const int i = item >> 2, f = item & 3;
    int t = m.splitlist[i];
    int mask = m.pmask[t];
    int fl[3], k = 0;
    for (int l = 0; l < 4; ++l)
      if (l != f) fl[k++] = l;
    int b0 = (mask >> fl[0]) & 1, b1 = (mask >> fl[1]) & 1, b2 = (mask >> fl[2]) & 1;
    if (b0 == b1 && b1 == b2) continue;
    int lone = (b1 == b2) ? fl[0] : (b0 == b2) ? fl[1] : fl[2];
    int cn = ((const int*)&m.nbr[t])[f];
    if (cn < 0 || m.smask[cn] >= 0) continue;
    int fc = (m.nbrface[t] >> (8 * f)) & 0xff;
    int4 q4 = snodes[i];
    const int nd[4] = {q4.x, q4.y, q4.z, q4.w};
    ((int*)m.front)[4 * cn + fc] = nd[lone];
    if (atomicCAS(&m.candf[cn], 0, 1) == 0) m.cand[atomicAdd(&c->n_cand, 1)] = cn;
  }
}

// Phase 2 of a large batch, over the whole chip, after k_topology.
template <class R>
__global__ __launch_bounds__(kBlock) void k_topo_sums(Mesh m, Work w, const Counters* __restrict__ c,
                                                      const int4* __restrict__ snodes,
                                                      const int* __restrict__ sedges) {
  const int n = c->batch_n;
  if (n == 0) return;
  const int gtid = (int)(blockIdx.x * blockDim.x + threadIdx.x), gthreads = (int)(gridDim.x * blockDim.x);
  topo_masses<R>(m, snodes, c->batch_base, n, gtid, gthreads);
  topo_volumes<R>(m, (R*)w.einvV, sedges, n, gtid, gthreads);
}

// What a split reads of its parent (phase 0), and writes (phase 1).  Eight
// lanes per split: lane l < 4 copies extra node l and fixes its node-list
// entries, lane q < 6 rewrites edge q's patch entries, lane 0 the records and
// the two copies' element rows.  A workgroup reads every split it holds
// before a barrier and writes after it, so a split never sees its own
// writes; splits of one batch touch disjoint data (their own tet, copy slot,
// extra nodes, new edges and list entries), so any grouping of splits into
// workgroups gives the same result.
struct SplitIn {
  int t, mask, nd[4], ed[6], pp[6];
  int4 op4;
  double V, kp, area, G;
  int ti, pat;
  double4 xr, ur, vr, ar, uhr;  // the real twin's state for extra node sl
  int insr;
};

template <class R>
__device__ __forceinline__ void split_read(const Mesh& m, const State& st, int i, int sl,
                                           int dynamic, int* dead, SplitIn& q) {
  q.t = m.splitlist[i];
  q.mask = m.pmask[q.t];
  load_tet<R>(m, q.t, q.nd, q.ed);
  q.op4 = make_int4(0, 0, 0, 0);
  q.V = 0;
  q.kp = 1.0;
  q.area = 0;
  q.G = 0;
  q.ti = 0;
  q.pat = 0;
#pragma unroll
  for (int r = 0; r < 6; ++r) q.pp[r] = 0;
  if (m.mode == MODE_PHANTOM) {
    q.op4 = m.epos[q.t];
    q.V = m.vol[q.t];
    if (m.kap) q.kp = m.kap[q.t];
    if (m.n_inst) q.ti = m.tinst[q.t];
    const int* p6 = (const int*)&m.patchpos[3 * q.t];
#pragma unroll
    for (int r = 0; r < 6; ++r) q.pp[r] = p6[r];
  }
  if (sl == 0 && dynamic) {
    q.pat = m.ppat[q.t];
    q.G = m.pG[q.t];
    q.area = crack_area(m, q.nd, q.mask);
  }
  // candidates that split now leave dead entries in the candidate list
  if (sl == 0 && m.candf[q.t]) atomicAdd(dead, 1);
  // the real twin's state (real nodes are not written by any split)
  q.xr = make_double4(0, 0, 0, 0);
  q.ur = q.vr = q.ar = q.uhr = q.xr;
  q.insr = 0;
  if (sl < 4 && m.mode == MODE_PHANTOM) {
    const int nr = pick4(q.nd[0], q.nd[1], q.nd[2], q.nd[3], sl);
    q.xr = m.X[nr];
    q.ur = st.u[nr];
    q.vr = st.v[nr];
    q.ar = st.a[nr];
    q.uhr = st.uh[nr];
    if (m.n_inst) q.insr = m.inst[nr];
  }
}

template <class R>
__device__ __forceinline__ void split_write(const Mesh& m, const State& st, R* __restrict__ einvV,
                                            const Counters* __restrict__ c, int base, int i,
                                            int sl, int dynamic, const SplitIn& q,
                                            int4* __restrict__ snodes, int* __restrict__ sedges) {
  const int s = base + i, t = q.t, mask = q.mask;
  if (sl == 0) {
    snodes[i] = make_int4(q.nd[0], q.nd[1], q.nd[2], q.nd[3]);
#pragma unroll
    for (int r = 0; r < 6; ++r) sedges[6 * i + r] = q.ed[r];
    m.smask[t] = mask;
    m.rec_step[s] = dynamic ? (int)(c->step + 1) : (int)c->step;
    m.rec_tet[s] = t;
    m.split_of[t] = s;
    m.rec_mask[s] = mask;
    m.rec_pat[s] = q.pat;
    m.rec_G[s] = q.G;
    m.area[i] = q.area;
    m.rec_area[s] = q.area;
    if (m.mode == MODE_ERODE)
      m.enodes[t] = make_int4(pack0(q.nd[0], FR_ZERO), q.nd[1], q.nd[2], q.nd[3]);
  }
  if (m.mode != MODE_PHANTOM) return;
  const int tb = m.T0 + s;
  const int nb = __popc(mask);
  const int codeA = code_for_side(4 - nb), codeB = code_for_side(nb);
  if (sl < 4) {
    const int l = sl;
    const int opl = pick4(q.op4.x, q.op4.y, q.op4.z, q.op4.w, l);
    const int x = m.N0 + 4 * s + l;
    const int xe = 4 * m.T0 + 4 * s + l;  // the extra node's single list entry
    m.X[x] = q.xr;
    st.u[x] = q.ur;
    st.v[x] = q.vr;
    st.a[x] = q.ar;
    st.uh[x] = q.uhr;
    m.lslot[x] = -1;
    if (m.n_inst) m.inst[x] = q.insr;
    const bool onB = (mask >> l) & 1;
    const int owner = onB ? t : tb;  // the copy that holds the extra node
    m.nent[xe] = (owner << 2) | l;
    if (onB) m.nent[opl] = (tb << 2) | l;
  }
  // a new edge's patch is one copy: kappa_k is the parent's
  const R ivA = (R)(q.kp / (frac_of(codeA) * q.V)), ivB = (R)(q.kp / (frac_of(codeB) * q.V));
  const int ebase = m.E0 + 10 * s, pbase = 6 * m.T0 + 10 * s;
  int eA[6], eB[6];
  int r = 0;  // every edge makes one new edge, a cut edge two
#pragma unroll
  for (int e = 0; e < 6; ++e) {
    const int k = q.ed[e];
    const int ba = (mask >> kEA[e]) & 1, bb = (mask >> kEB[e]) & 1;
    const bool mine = sl == e;
    if (!ba && !bb) {          // both nodes on side A: copy A keeps edge k
      eA[e] = k;
      eB[e] = ebase + r;
      if (mine) { m.pent[pbase + r] = tb; einvV[ebase + r] = ivB; }
      r++;
    } else if (ba && bb) {     // both on side B: copy B takes edge k
      eB[e] = k;
      eA[e] = ebase + r;
      if (mine) { m.pent[q.pp[e]] = tb; m.pent[pbase + r] = t; einvV[ebase + r] = ivA; }
      r++;
    } else {                   // cut edge: each copy gets a new one
      eA[e] = ebase + r;
      eB[e] = ebase + r + 1;
      if (mine) {
        m.pent[q.pp[e]] = -1;
        m.pent[pbase + r] = t; einvV[ebase + r] = ivA;
        m.pent[pbase + r + 1] = tb; einvV[ebase + r + 1] = ivB;
      }
      r += 2;
    }
  }
  if (sl == 6)
    for (int e = r; e < 10; ++e) { m.pent[pbase + e] = -1; einvV[ebase + e] = (R)0; }
  if (sl == 7 && m.n_inst) {
    m.tinst[tb] = q.ti;
    for (int e = 0; e < 10; ++e) m.einst[ebase + e] = q.ti;
  }
  if (sl == 0) {
    const int op[4] = {q.op4.x, q.op4.y, q.op4.z, q.op4.w};
    int na[4], nbn[4], pa[4], pb[4];
#pragma unroll
    for (int l = 0; l < 4; ++l) {
      const int x = m.N0 + 4 * s + l, xe = 4 * m.T0 + 4 * s + l;
      const bool onB = (mask >> l) & 1;
      na[l] = onB ? x : q.nd[l];
      nbn[l] = onB ? q.nd[l] : x;
      pa[l] = onB ? xe : op[l];
      pb[l] = onB ? op[l] : xe;
    }
    m.enodes[t] = make_int4(pack0(na[0], codeA), na[1], na[2], na[3]);
    m.enodes[tb] = make_int4(pack0(nbn[0], codeB), nbn[1], nbn[2], nbn[3]);
    m.epos[t] = make_int4(pa[0], pa[1], pa[2], pa[3]);
    m.epos[tb] = make_int4(pb[0], pb[1], pb[2], pb[3]);
    m.vol[tb] = q.V;
    if (m.kap) m.kap[tb] = q.kp;
    m.et2e[3 * t] = make_int2(eA[0], eA[1]);
    m.et2e[3 * t + 1] = make_int2(eA[2], eA[3]);
    m.et2e[3 * t + 2] = make_int2(eA[4], eA[5]);
    m.et2e[3 * tb] = make_int2(eB[0], eB[1]);
    m.et2e[3 * tb + 1] = make_int2(eB[2], eB[3]);
    m.et2e[3 * tb + 2] = make_int2(eB[4], eB[5]);
    // the copy's corners sit where the parent's do (extra nodes copy their twins)
#pragma unroll
    for (int r = 0; r < 9; ++r) m.gtab[9 * (size_t)tb + r] = m.gtab[9 * (size_t)t + r];
  }
}

// The candidate list drops the tets that have split once they are the
// majority (and at least CEM_CAND_COMPACT_MIN): an order-keeping compaction in
// place by one workgroup of kTopoBlock threads (each chunk is read in full
// before any of it is written, and writes land at or below it).  Its work
// over a run is at most twice the entries ever appended.  new_dead: the
// batch's candidates, the same value in every thread.
__device__ void compact_candidates(const Mesh& m, Counters* __restrict__ c, int new_dead) {
  __shared__ int s_nc, s_nd, s_wtot[kTopoBlock / 64], s_total;
  const int tid = threadIdx.x;
  // one thread reads the counters, so that every thread takes the same branch
  if (tid == 0) {
    s_nc = c->n_cand;
    s_nd = c->n_cand_dead + new_dead;
  }
  __syncthreads();
  const int nc = s_nc, nd_all = s_nd;
  if (nd_all >= CEM_CAND_COMPACT_MIN && 2 * nd_all > nc) {
    const int lane = tid & 63, wv = tid >> 6;
    int out = 0;
    for (int b0 = 0; b0 < nc; b0 += kTopoBlock) {
      const int idx = b0 + tid;
      const int t = idx < nc ? m.cand[idx] : -1;
      const bool alive = t >= 0 && m.smask[t] < 0;
      const unsigned long long bal = __ballot(alive);
      const int pre = __popcll(bal & ((1ull << lane) - 1ull));
      if (lane == 0) s_wtot[wv] = __popcll(bal);
      __syncthreads();
      if (tid == 0) {
        int acc = 0;
        for (int w = 0; w < kTopoBlock / 64; ++w) {
          const int x = s_wtot[w];
          s_wtot[w] = acc;
          acc += x;
        }
        s_total = acc;
      }
      __syncthreads();
      if (alive) m.cand[out + s_wtot[wv] + pre] = t;
      out += s_total;
      __threadfence_block();
      __syncthreads();
    }
    if (tid == 0) {
      c->n_cand = out;
      c->n_cand_dead = 0;
    }
  } else if (tid == 0) {
    c->n_cand_dead = nd_all;
  }
  __threadfence_block();
  __syncthreads();
}

// Counters after a batch of n splits from global index base (thread 0), and
// the per-instance G maxima (all threads).
__device__ void topo_tail(const Mesh& m, Counters* __restrict__ c, int base, int n, int dynamic,
                          int advance) {
  if (threadIdx.x == 0) {
    if (!c->err) {
      if (n > 0 && dynamic) {
        double ud = c->Ud;
        for (int i = 0; i < n; ++i) ud += m.Gc * m.area[i];
        c->Ud = ud;
      }
      c->n_split = base + n;
      if (advance) {
        c->step += 1;
        c->gmax_last = c->gmax_key;
        c->gmax_key = 0;
      }
    }
    c->n_flag = 0;
  }
  if (advance && m.n_inst) {
    for (int i = threadIdx.x; i < m.n_inst; i += blockDim.x) {
      m.gmax_inst[m.n_inst + i] = m.gmax_inst[i];
      m.gmax_inst[i] = 0;
    }
  }
}

// All splits of one step, applied by one workgroup in phases separated by
// barriers.  Split i of this batch gets global index s = n_split + i; its
// copy B takes element slot T0 + s, its extra nodes N0 + 4 s + l and its new
// edges E0 + 10 s + r.  Copy A stays in the parent's slot.  With topo_multi
// (or for a host pre-split), a batch over kTopoInline is only sorted here:
// k_topo_apply, k_topo_sums and k_topo_finish complete it on the whole chip,
// with the same per-split code and sums.
template <class R>
__global__ __launch_bounds__(kTopoBlock) void k_topology(Mesh m, State st, Work w,
                                                         Counters* __restrict__ c, int dynamic,
                                                         int advance, int4* __restrict__ snodes,
                                                         int* __restrict__ sedges) {
  __shared__ int s_n, s_base, s_dead;
  __shared__ int shk[kSortLds], shv[kSortLds];
  const int tid = threadIdx.x;
  if (tid == 0) {
    s_n = c->err ? 0 : c->n_flag;
    s_base = c->n_split;
    s_dead = 0;
  }
  __syncthreads();
  const int n = s_n, base = s_base;
  R* einvV = (R*)w.einvV;
  if (n > 0) {
    if (dynamic) block_sort(m.splitlist, n, m.tet_ext, shk, shv);
    if (m.topo_multi && n > kTopoInline) {
      if (tid == 0) {
        c->batch_base = base;
        c->batch_n = n;
        c->batch_apply_n = n;
        c->dead_pending = 0;
      }
      return;
    }
    // phases 0 + 1, eight lanes per split (split_read, split_write)
    constexpr int GS = 8;
    const int sl = tid % GS;
    for (int i0 = 0; i0 < n; i0 += kTopoBlock / GS) {
      const int i = i0 + tid / GS;
      const bool on = i < n;
      SplitIn q;
      if (on) split_read<R>(m, st, i, sl, dynamic, &s_dead, q);
      __syncthreads();
      if (on) split_write<R>(m, st, einvV, c, base, i, sl, dynamic, q, snodes, sedges);
      __syncthreads();
    }
    __threadfence_block();
    __syncthreads();
    // the compaction comes before phase 3, which appends
    compact_candidates(m, c, s_dead);
    // phases 2 and 3 read what phase 1 wrote and nothing of each other.
    // Phase 2 (masses and edge volumes touched by the batch) and phase 3 (new
    // crack fronts) of a batch not left to the whole chip.  A batch of up to 8
    // splits runs the three item sets side by side on disjoint threads.
    if (n <= 8) {
      if (tid < 64 * n) topo_masses<R>(m, snodes, base, n, tid, 64 * n);
      else if (tid < 112 * n) topo_volumes<R>(m, einvV, sedges, n, tid - 64 * n, 48 * n);
      else if (tid < 116 * n) topo_fronts(m, c, snodes, n, tid - 112 * n, 4 * n);
    } else {
      topo_masses<R>(m, snodes, base, n, tid, kTopoBlock);
      topo_volumes<R>(m, einvV, sedges, n, tid, kTopoBlock);
      topo_fronts(m, c, snodes, n, tid, kTopoBlock);
    }
    __syncthreads();
  }
  if (tid == 0) {
    c->batch_base = base;
    c->batch_n = 0;
    c->batch_apply_n = 0;
  }
  topo_tail(m, c, base, n, dynamic, advance);
}

// Phases 0 + 1 of a deferred batch over the whole chip: 32 splits per
// workgroup pass, the same read / barrier / write as k_topology.
template <class R>
__global__ __launch_bounds__(kBlock) void k_topo_apply(Mesh m, State st, Work w,
                                                       Counters* __restrict__ c, int dynamic,
                                                       int4* __restrict__ snodes,
                                                       int* __restrict__ sedges) {
  const int n = c->batch_apply_n;
  if (n == 0) return;
  const int base = c->batch_base;
  R* einvV = (R*)w.einvV;
  constexpr int GS = 8, PER = kBlock / GS;
  const int sl = threadIdx.x % GS;
  for (int i0 = blockIdx.x * PER; i0 < n; i0 += gridDim.x * PER) {
    const int i = i0 + threadIdx.x / GS;
    const bool on = i < n;
    SplitIn q;
    if (on) split_read<R>(m, st, i, sl, dynamic, &c->dead_pending, q);
    __syncthreads();
    if (on) split_write<R>(m, st, einvV, c, base, i, sl, dynamic, q, snodes, sedges);
    __syncthreads();
  }
}

// The rest of a deferred batch, by one workgroup after k_topo_apply:
// candidate compaction, new crack fronts, counters.
template <class R>
__global__ __launch_bounds__(kTopoBlock) void k_topo_finish(Mesh m, Counters* __restrict__ c,
                                                            int dynamic, int advance,
                                                            const int4* __restrict__ snodes) {
  __shared__ int s_n, s_base, s_dead;
  const int tid = threadIdx.x;
  if (tid == 0) {
    s_n = c->batch_apply_n;
    s_base = c->batch_base;
    s_dead = c->dead_pending;
  }
  __syncthreads();
  const int n = s_n, base = s_base;
  if (n == 0) return;
  compact_candidates(m, c, s_dead);
  topo_fronts(m, c, snodes, n, tid, kTopoBlock);
  __syncthreads();
  if (tid == 0) {
    c->batch_apply_n = 0;
    c->dead_pending = 0;
  }
  topo_tail(m, c, base, n, dynamic, advance);
}

// ---------------------------------------------------------------- hex crack patterns

// Readback of every candidate of every hex front (unordered; the host sorts):
// (hex, face, plane) and (G, pattern).
template <class R>
__global__ __launch_bounds__(kBlock) void k_hex_front_eval(Mesh m, const double4* __restrict__ u,
                                                           const Six<R>* __restrict__ esig,
                                                           const Counters* __restrict__ c, int* out_tfl,
                                                           double* out_g, int* out_n) {
  const int nc = c->n_cand;
  for (int idx = blockIdx.x * kBlock + threadIdx.x; idx < nc; idx += gridDim.x * kBlock) {
    const int t = m.cand[idx];
    if (m.smask[t] >= 0) continue;
    int nd[8], ed[12];
    hx_load(m, t, nd, ed);
    for (int f = 0; f < 6; ++f) {
      const int code = m.hfront[6 * t + f];
      if (code < 0) continue;
      const int qa = code >> 4, qb = code & 15;
      int pl, pt, q3, q4;
      for (int j = 0; hx_candidate(f, qa, qb, j, pl, pt, q3, q4); ++j) {
        const double g = hx_G<R>(m, u, esig, nd, ed, qa, qb, pt, q3, q4);
        const int o = atomicAdd(out_n, 1);
        out_tfl[3 * o] = t;
        out_tfl[3 * o + 1] = f;
        out_tfl[3 * o + 2] = pl;
        out_g[2 * o] = g;
        out_g[2 * o + 1] = (double)pt;
      }
    }
  }
}

// All hex cracks of one step (or a host precrack batch), by one workgroup:
// sort by the caller's id, then per crack its record, its volume fraction,
// the volumes of its twelve edges (the patch sum in patch order, as at
// upload) and the new fronts of its intact face neighbours.
template <class R>
__global__ __launch_bounds__(kTopoBlock) void k_hex_topology(Mesh m, Work w, Counters* __restrict__ c,
                                                             int dynamic, int advance) {
  __shared__ int s_n, s_base;
  __shared__ int shk[kSortLds], shv[kSortLds];
  const int tid = threadIdx.x;
  if (tid == 0) {
    s_n = c->err ? 0 : c->n_flag;
    s_base = c->n_split;
  }
  __syncthreads();
  const int n = s_n, base = s_base;
  R* einvV = (R*)w.einvV;
  if (n > 0) {
    if (dynamic) block_sort(m.splitlist, n, m.tet_ext, shk, shv);
    for (int i = tid; i < n; i += kTopoBlock) {
      const int t = m.splitlist[i], p = m.pmask[t], s = base + i;
      int nd[8], ed[12];
      hx_load(m, t, nd, ed);
      const double area = dynamic ? hx_plane_area(m, nd, p) : 0.0;
      m.smask[t] = p;
      m.rec_step[s] = dynamic ? (int)(c->step + 1) : (int)c->step;
      m.rec_tet[s] = t;
      m.rec_mask[s] = p;
      m.rec_pat[s] = dynamic ? m.ppat[t] : 0;
      m.rec_G[s] = dynamic ? m.pG[t] : 0.0;
      m.area[i] = area;
      m.rec_area[s] = area;
      m.vol[t] *= p < 3 ? 0.0 : 0.5;
    }
    __threadfence_block();
    __syncthreads();
    for (int item = tid; item < 12 * n; item += kTopoBlock) {
      const int t = m.splitlist[item / 12], q = item % 12;
      const int2 e2 = m.he2e[6 * t + (q >> 1)];
      const int k = (q & 1) ? e2.y : e2.x;
      double S = 0;
      for (int pp = m.poff[k]; pp < m.poff[k + 1]; ++pp) S += m.vol[m.pent[pp] / 12];
      einvV[k] = !(S > 0) ? (R)0 : (R)(1.0 / S);
    }
    for (int item = tid; item < 6 * n; item += kTopoBlock) {
      const int t = m.splitlist[item / 6], f = item % 6;
      const int on = hx_plane_mask(m.smask[t]) & hx_face_mask(f);
      if (__popc(on) != 2) continue;
      const int nb8 = m.hnbr[6 * t + f];
      if (nb8 < 0) continue;
      const int nb = nb8 >> 3, fb = nb8 & 7;
      if (m.smask[nb] >= 0) continue;
      int ed[12], nd[8], edn[12], ndn[8];
      hx_load(m, t, nd, ed);
      hx_load(m, nb, ndn, edn);
      int ql[2], r = 0;
      for (int q = 0; q < 12; ++q) {
        if (!((on >> q) & 1)) continue;
        int x = -1;
        for (int qq = 0; qq < 12; ++qq)
          if (edn[qq] == ed[q]) x = qq;
        ql[r++] = x;
      }
      const int lo = ql[0] < ql[1] ? ql[0] : ql[1], hi = ql[0] < ql[1] ? ql[1] : ql[0];
      m.hfront[6 * nb + fb] = 16 * lo + hi;
      if (atomicCAS(&m.candf[nb], 0, 1) == 0) m.cand[atomicAdd(&c->n_cand, 1)] = nb;
    }
    __threadfence_block();
    __syncthreads();
  }
  if (tid == 0) {
    c->batch_base = base;
    c->batch_n = 0;
    c->batch_apply_n = 0;
  }
  topo_tail(m, c, base, n, dynamic, advance);
}

// ---------------------------------------------------------------- prescribed velocities

// Constrained components of u at the current time (before a force evaluation
// that starts the integration).
__global__ __launch_bounds__(kBlock) void k_bc_apply(Mesh m, State st, const Counters* c) {
  int b = blockIdx.x * kBlock + threadIdx.x;
  if (b >= m.n_bc) return;
  int i = m.bnode[b], mk = m.bmask[b];
  double S, V, A;
  bc_history(m.gt0[mk >> 4], (double)c->step * node_dt(m, i), S, V, A);
  double4 u = st.u[i], w = m.bv0[b], ref = m.bref[b];
  if (mk & 1) u.x = ref.x + w.x * S;
  if (mk & 2) u.y = ref.y + w.y * S;
  if (mk & 4) u.z = ref.z + w.z * S;
  st.u[i] = u;
}

// Reaction of each group summed over its slots in a fixed tree order, as one
// history row of the step just taken (the step counter advances after).
__global__ __launch_bounds__(kBlock) void k_reaction(Mesh m, const Counters* __restrict__ c) {
  __shared__ double red[3][kBlock];
  if (c->err) return;
  const long long n = c->step;
  const double t1 = (double)(n + 1) * m.dt;
  for (int g = 0; g < m.n_grp; ++g) {
    double sx = 0, sy = 0, sz = 0;
    for (int b = m.goff[g] + threadIdx.x; b < m.goff[g + 1]; b += kBlock) {
      double4 R = m.breact[b];
      sx += R.x;
      sy += R.y;
      sz += R.z;
    }
    red[0][threadIdx.x] = sx;
    red[1][threadIdx.x] = sy;
    red[2][threadIdx.x] = sz;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
      if (threadIdx.x < w)
        for (int q = 0; q < 3; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + w];
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      double S, V, A;
      bc_history(m.gt0[g], t1, S, V, A);
      double* row = m.ghist + ((size_t)g * m.hist_cap + (size_t)(n % m.hist_cap)) * 6;
      row[0] = (double)(n + 1);
      row[1] = t1;
      row[2] = red[0][0];
      row[3] = red[1][0];
      row[4] = red[2][0];
      row[5] = S;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------- setup

__global__ __launch_bounds__(kBlock) void k_volumes(Mesh m) {
  int e = blockIdx.x * kBlock + threadIdx.x;
  if (e >= m.T0) return;
  m.vol[e] = elem_volume(m, m.enodes[e]);
}

// Corner-normal table rows of every element slot in use, from the coordinates.
__global__ __launch_bounds__(kBlock) void k_normals(Mesh m, const Counters* __restrict__ c) {
  const int e = blockIdx.x * kBlock + threadIdx.x;
  if (e >= elems_now(m, c)) return;
  const int4 nd = m.enodes[e];
  float g[3][3];
  face_normals(m.X[nd.x & kNodeMask], m.X[nd.y], m.X[nd.z], m.X[nd.w], g);
  float* p = m.gtab + 9 * (size_t)e;
#pragma unroll
  for (int l = 0; l < 3; ++l)
#pragma unroll
    for (int d = 0; d < 3; ++d) p[3 * l + d] = g[l][d];
}

// Lumped mass m_i = sum rho V_eff / 4 over the elements holding node i.
__global__ __launch_bounds__(kBlock) void k_masses(Mesh m) {
  int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= m.N0) return;
  double ms = 0;
  for (int p = m.noff[i]; p < m.noff[i + 1]; ++p) {
    if (m.etype == 8) {  // a hex gives rho V / 8 to each of its nodes
      ms += m.rho * m.vol[m.nent[p] >> 3] / 8.0;
      continue;
    }
    int e = m.nent[p] >> 2;
    ms += m.rho * frac_of((unsigned)m.enodes[e].x >> kNodeBits) * m.vol[e] / 4.0;
  }
  m.invm[i] = ms > 0 ? 1.0 / ms : 0.0;
}

// einvV_k = kappa_k / S_k with S_k the patch's effective volume and
// kappa_k = sum_patch V_eff kappa_e / S_k: a per-tet modulus enters the
// smoothing domain as the volume average of the element elasticities, and
// folding it into this factor leaves the stress pass unchanged.
template <class R>
__global__ __launch_bounds__(kBlock) void k_edge_volumes(Mesh m, R* einvV, int count) {
  int k = blockIdx.x * kBlock + threadIdx.x;
  if (k >= count) return;
  double S = 0, SK = 0;
  for (int p = m.poff[k]; p < m.poff[k + 1]; ++p) {
    int e = m.pent[p];
    if (e < 0) continue;
    // a hex mesh's entries name (hex, edge point) as 12 hex + q
    double ve = m.etype == 8 ? m.vol[e / 12] : frac_of((unsigned)m.enodes[e].x >> kNodeBits) * m.vol[e];
    S += ve;
    if (m.kap) SK += ve * m.kap[e];
  }
  einvV[k] = !(S > 0) ? (R)0 : m.kap ? (R)(SK / S / S) : (R)(1.0 / S);
}

__global__ __launch_bounds__(kBlock) void k_kap_copies(Mesh m, int n_split) {
  int s = blockIdx.x * kBlock + threadIdx.x;
  if (s < n_split && m.mode == MODE_PHANTOM) m.kap[m.T0 + s] = m.kap[m.rec_tet[s]];
}

// Nodal loads: each loaded triangle adds t A / 3 to each vertex (gathered per
// loaded node over its triangles).
__global__ __launch_bounds__(kBlock) void k_loads(Mesh m, const int4* ftri, const double4* ftrac,
                                                  const int* lfoff, const int* lfent) {
  int sl = blockIdx.x * kBlock + threadIdx.x;
  if (sl >= m.n_load) return;
  double fx = 0, fy = 0, fz = 0;
  for (int p = lfoff[sl]; p < lfoff[sl + 1]; ++p) {
    int f = lfent[p];
    int4 tr = ftri[f];
    double4 a = m.X[tr.x], b = m.X[tr.y], cc = m.X[tr.z];
    double ux = b.x - a.x, uy = b.y - a.y, uz = b.z - a.z;
    double vx = cc.x - a.x, vy = cc.y - a.y, vz = cc.z - a.z;
    double cx = uy * vz - uz * vy, cy = uz * vx - ux * vz, cz = ux * vy - uy * vx;
    double A = 0.5 * sqrt(cx * cx + cy * cy + cz * cz);
    double4 t = ftrac[f];
    fx += t.x * A / 3.0;
    fy += t.y * A / 3.0;
    fz += t.z * A / 3.0;
  }
  m.Fload[sl] = make_double4(fx, fy, fz, 0.0);
  m.wacc[sl] = 0.0;
}

// Largest eigenvalue of B^T C B per tet: the nonzero spectrum equals that of
// the 6 x 6 matrix (L^T B)(L^T B)^T with C = L L^T (Cholesky), solved by
// cyclic Jacobi rotations.
__global__ __launch_bounds__(kBlock) void k_dtcrit(Mesh m, Counters* __restrict__ c) {
  __shared__ unsigned long long red[kBlock];
  double lmax = 0;
  int t = blockIdx.x * kBlock + threadIdx.x;
  if (t < m.T0) {
    int4 nd = m.enodes[t];
    double4 x0 = m.X[nd.x & kNodeMask], x1 = m.X[nd.y], x2 = m.X[nd.z], x3 = m.X[nd.w];
    double c1[3] = {x1.x - x0.x, x1.y - x0.y, x1.z - x0.z};
    double c2[3] = {x2.x - x0.x, x2.y - x0.y, x2.z - x0.z};
    double c3[3] = {x3.x - x0.x, x3.y - x0.y, x3.z - x0.z};
    double g[4][3];
    g[1][0] = c2[1] * c3[2] - c2[2] * c3[1]; g[1][1] = c2[2] * c3[0] - c2[0] * c3[2]; g[1][2] = c2[0] * c3[1] - c2[1] * c3[0];
    g[2][0] = c3[1] * c1[2] - c3[2] * c1[1]; g[2][1] = c3[2] * c1[0] - c3[0] * c1[2]; g[2][2] = c3[0] * c1[1] - c3[1] * c1[0];
    g[3][0] = c1[1] * c2[2] - c1[2] * c2[1]; g[3][1] = c1[2] * c2[0] - c1[0] * c2[2]; g[3][2] = c1[0] * c2[1] - c1[1] * c2[0];
    double det = c1[0] * g[1][0] + c1[1] * g[1][1] + c1[2] * g[1][2];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      g[1][d] /= det; g[2][d] /= det; g[3][d] /= det;
      g[0][d] = -(g[1][d] + g[2][d] + g[3][d]);
    }
    // B (6 x 12)
    double B[6][12];
#pragma unroll
    for (int r = 0; r < 6; ++r)
#pragma unroll
      for (int q = 0; q < 12; ++q) B[r][q] = 0;
#pragma unroll
    for (int l = 0; l < 4; ++l) {
      B[0][3 * l] = g[l][0];
      B[1][3 * l + 1] = g[l][1];
      B[2][3 * l + 2] = g[l][2];
      B[3][3 * l] = g[l][1]; B[3][3 * l + 1] = g[l][0];
      B[4][3 * l + 1] = g[l][2]; B[4][3 * l + 2] = g[l][1];
      B[5][3 * l] = g[l][2]; B[5][3 * l + 2] = g[l][0];
    }
    // Cholesky of the normal block [[a b b][b a b][b b a]], a = lam + 2 mu, b = lam
    double a = m.lam + 2 * m.mu, b = m.lam;
    double L11 = sqrt(a), L21 = b / L11, L31 = b / L11;
    double L22 = sqrt(a - L21 * L21), L32 = (b - L31 * L21) / L22;
    double L33 = sqrt(a - L31 * L31 - L32 * L32);
    double sm = sqrt(m.mu);
    double Xm[6][12];
#pragma unroll
    for (int q = 0; q < 12; ++q) {
      Xm[0][q] = L11 * B[0][q] + L21 * B[1][q] + L31 * B[2][q];
      Xm[1][q] = L22 * B[1][q] + L32 * B[2][q];
      Xm[2][q] = L33 * B[2][q];
      Xm[3][q] = sm * B[3][q];
      Xm[4][q] = sm * B[4][q];
      Xm[5][q] = sm * B[5][q];
    }
    double A[6][6];
#pragma unroll
    for (int i = 0; i < 6; ++i)
#pragma unroll
      for (int j = 0; j < 6; ++j) {
        double s = 0;
#pragma unroll
        for (int q = 0; q < 12; ++q) s += Xm[i][q] * Xm[j][q];
        A[i][j] = s;
      }
    lmax = jacobi_lmax6(A);
    if (m.kap) lmax *= m.kap[t];  // C_t = kappa_t C scales the spectrum
    if (m.n_inst) atomicMax(&m.lam_inst[m.tinst[t]], dkey(lmax));
  }
  red[threadIdx.x] = dkey(lmax);
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] = red[threadIdx.x] > red[threadIdx.x + w] ? red[threadIdx.x] : red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicMax(&c->lam_key, red[0]);
}

__global__ void k_dtfinish(Mesh m, Counters* c) {
  if (threadIdx.x == 0) {
    double lam = key_to_double(c->lam_key);
    // lumped element mass rho V / n per node (n = 4 tets, 8 hexes)
    c->dt_crit = 2.0 / sqrt((m.etype == 8 ? 8.0 : 4.0) / m.rho * lam);
  }
  for (int i = threadIdx.x; i < m.n_inst; i += blockDim.x)
    m.dtc_inst[i] = 2.0 / sqrt(4.0 / m.rho * key_to_double(m.lam_inst[i]));
}

// Instance of each original edge: that of its first patch element.
__global__ __launch_bounds__(kBlock) void k_edge_instances(Mesh m) {
  int k = blockIdx.x * kBlock + threadIdx.x;
  if (k < m.E0) m.einst[k] = m.tinst[m.pent[m.poff[k]]];
}

// ---------------------------------------------------------------- reductions

__global__ __launch_bounds__(kBlock) void k_kinetic(Mesh m, State st, const Counters* __restrict__ c,
                                                    double* partial, int want) {
  __shared__ double red[kBlock];
  double s = 0;
  int Nn = nodes_now(m, c);
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < Nn; i += gridDim.x * kBlock) {
    if (want >= 0 && m.inst[i] != want) continue;
    double im = m.invm[i];
    if (im > 0) {
      double4 v = st.v[i];
      s += 0.5 * (v.x * v.x + v.y * v.y + v.z * v.z) / im;
    }
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// External work of one instance (or all): fixed-order sum over load slots.
__global__ __launch_bounds__(kBlock) void k_work_sum(Mesh m, double* out, int want) {
  __shared__ double red[kBlock];
  double s = 0;
  for (int i = threadIdx.x; i < m.n_load; i += kBlock)
    if (want < 0 || m.inst[m.lnode[i]] == want) s += m.wacc[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

// Dissipated energy of one instance: Gc x crack area over its splits decided
// by the G test (records with a pattern), fixed-order sum.
__global__ __launch_bounds__(kBlock) void k_dissipated(Mesh m, const Counters* __restrict__ c,
                                                       double* out, int want) {
  __shared__ double red[kBlock];
  __shared__ int cnt[kBlock];
  double s = 0;
  int n = 0;
  for (int i = threadIdx.x; i < c->n_split; i += kBlock) {
    if (want >= 0 && m.tinst[m.rec_tet[i]] != want) continue;
    n++;
    if (m.rec_pat[i] > 0) s += m.Gc * m.rec_area[i];
  }
  red[threadIdx.x] = s;
  cnt[threadIdx.x] = n;
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      red[threadIdx.x] += red[threadIdx.x + w];
      cnt[threadIdx.x] += cnt[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = red[0];
    out[1] = (double)cnt[0];  // splits of the instance
  }
}

// Fixed-order sum (single workgroup).
__global__ __launch_bounds__(kBlock) void k_sum(const double* __restrict__ x, int n, double* out) {
  __shared__ double red[kBlock];
  double s = 0;
  for (int i = threadIdx.x; i < n; i += kBlock) s += x[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

// ---------------------------------------------------------------- launchers

int grid_for(long long n) { return (int)((n + kBlock - 1) / kBlock); }
double key_to_double_host(unsigned long long k) { return key_to_double(k); }

template <class R>
hipError_t Launch<R>::strain(const Mesh& m, const double4* u, const Work& w, Counters* c,
                             hipStream_t s) {
  if (m.etype == 8) return launch_strain_hex<R>(m, u, w.veps, c, s);
  hipLaunchKernelGGL(k_strain<R>, dim3(persistent_grid(m, m.T_cap)), dim3(kBlock), 0, s, m, u,
                     (Six<R>*)w.veps, c);
  return hipGetLastError();
}

template <class R>
hipError_t Launch<R>::edge_stress(const Mesh& m, const Work& w, Counters* c, hipStream_t s) {
  hipLaunchKernelGGL(k_edge_stress<R>, dim3(persistent_grid(m, m.E_cap)), dim3(kBlock), 0, s, m,
                     (const Six<R>*)w.veps, (const R*)w.einvV, (Six<R>*)w.esig, c);
  return hipGetLastError();
}

// The candidate list is short next to the mesh: a small grid-stride grid.
static int front_grid(const Mesh& m) {
  int g = grid_for(m.T0);
  return g < 1 ? 1 : (g > 64 ? 64 : g);
}

template <class R>
hipError_t Launch<R>::front_eval(const Mesh& m, const State& st, const Work& w, Counters* c,
                                 int* out_tfl, double* out_g, int* out_n, hipStream_t s) {
  if (m.etype == 8)
    hipLaunchKernelGGL(k_hex_front_eval<R>, dim3(front_grid(m)), dim3(kBlock), 0, s, m,
                       (const double4*)st.u, (const Six<R>*)w.esig, c, out_tfl, out_g, out_n);
  else
    hipLaunchKernelGGL(k_front_eval<R>, dim3(front_grid(m)), dim3(kBlock), 0, s, m,
                       (const double4*)st.u, (const Six<R>*)w.esig, c, out_tfl, out_g, out_n);
  return hipGetLastError();
}

template <class R, int G, int KIND>
static void launch_node_kind(const Mesh& m, const State& st, const R* ct, Counters* c, int mode,
                             double4* fout, hipStream_t s, int first = 0) {
  dim3 g(persistent_grid(m, (long long)(m.N_cap - first) * G)), b(kBlock);
  // constrained nodes take their own kernel variant, so that a mesh without
  // prescribed velocities pays nothing for them
  if (mode == NODE_FORCE)
    hipLaunchKernelGGL((k_node<R, NODE_FORCE, G, false, KIND>), g, b, 0, s, m, st, ct, fout, c, first);
  else if (mode == NODE_INIT && m.n_bc)
    hipLaunchKernelGGL((k_node<R, NODE_INIT, G, true, KIND>), g, b, 0, s, m, st, ct, fout, c, first);
  else if (mode == NODE_INIT)
    hipLaunchKernelGGL((k_node<R, NODE_INIT, G, false, KIND>), g, b, 0, s, m, st, ct, fout, c, first);
  else if (m.n_bc)
    hipLaunchKernelGGL((k_node<R, NODE_STEP, G, true, KIND>), g, b, 0, s, m, st, ct, fout, c, first);
  else
    hipLaunchKernelGGL((k_node<R, NODE_STEP, G, false, KIND>), g, b, 0, s, m, st, ct, fout, c, first);
}

template <class R, int G>
static void launch_node_lanes(const Mesh& m, const State& st, const R* ct, const Six<R>* sg,
                              Counters* c, int mode, double4* fout, hipStream_t s,
                              int first = 0) {
  // hexes hand over their nodal terms at node-list positions, like the
  // tetrahedra's term layout
  if (m.etype != 8 && m.ssum) launch_node_kind<R, G, 2>(m, st, ct, c, mode, fout, s, first);
  else launch_node_kind<R, G, 0>(m, st, ct, c, mode, fout, s, first);
}

template <class R, int G>
static void launch_tile_lanes(const Mesh& m, const State& st, const Work& w, Counters* c, int mode,
                              double4* fout, hipStream_t s) {
  int grid = (m.ntile[sizeof(R) == 8 ? 0 : 1] + 7) / 8 * 8;
  if (grid > m.grid_cap) grid = m.grid_cap;
  if (grid < 8) grid = 8;
  dim3 g(grid), b(tile_block<R>());
  const Six<R>* sg = (const Six<R>*)w.esig;
  R* ct = (R*)w.contrib;
  if (mode == NODE_FORCE)
    hipLaunchKernelGGL((k_force_tile<R, NODE_FORCE, G, false>), g, b, 0, s, m, st, sg, ct, fout, c);
  else if (mode == NODE_INIT && m.n_bc)
    hipLaunchKernelGGL((k_force_tile<R, NODE_INIT, G, true>), g, b, 0, s, m, st, sg, ct, fout, c);
  else if (mode == NODE_INIT)
    hipLaunchKernelGGL((k_force_tile<R, NODE_INIT, G, false>), g, b, 0, s, m, st, sg, ct, fout, c);
  else if (m.n_bc)
    hipLaunchKernelGGL((k_force_tile<R, NODE_STEP, G, true>), g, b, 0, s, m, st, sg, ct, fout, c);
  else
    hipLaunchKernelGGL((k_force_tile<R, NODE_STEP, G, false>), g, b, 0, s, m, st, sg, ct, fout, c);
  // the extra nodes of split copies: their single terms were written to the
  // global term array by the tiles
  // one lane per extra node: each has a single entry
  if (m.mode == MODE_PHANTOM) launch_node_kind<R, 1, 0>(m, st, ct, c, mode, fout, s, m.N0);
}

template <class R>
static void launch_fx(const Mesh& m, const State& st, const Work& w, Counters* c, int mode,
                      double4* fout, hipStream_t s) {
  int grid = (m.ntile_fx + 7) / 8 * 8;
  if (grid > m.grid_cap) grid = m.grid_cap;
  if (grid < 8) grid = 8;
  dim3 g(grid), b(kFxBlock);
  const Six<R>* sg = (const Six<R>*)w.esig;
  R* ct = (R*)w.contrib;
  if (mode == NODE_FORCE)
    hipLaunchKernelGGL((k_force_fx<R, NODE_FORCE, false>), g, b, 0, s, m, st, sg, ct, fout, c);
  else if (mode == NODE_INIT && m.n_bc)
    hipLaunchKernelGGL((k_force_fx<R, NODE_INIT, true>), g, b, 0, s, m, st, sg, ct, fout, c);
  else if (mode == NODE_INIT)
    hipLaunchKernelGGL((k_force_fx<R, NODE_INIT, false>), g, b, 0, s, m, st, sg, ct, fout, c);
  else if (m.n_bc)
    hipLaunchKernelGGL((k_force_fx<R, NODE_STEP, true>), g, b, 0, s, m, st, sg, ct, fout, c);
  else
    hipLaunchKernelGGL((k_force_fx<R, NODE_STEP, false>), g, b, 0, s, m, st, sg, ct, fout, c);
  // the extra nodes of split copies: one lane each (a single entry)
  if (m.mode == MODE_PHANTOM) launch_node_kind<R, 1, 0>(m, st, ct, c, mode, fout, s, m.N0);
}

template <class R>
hipError_t Launch<R>::node(const Mesh& m, const State& st, const Work& w, Counters* c, int mode,
                           double4* fout, hipStream_t s, hipEvent_t mid, int front) {
  if (m.etype != 8 && m.tiled) {
    if (front >= 0) {
      hipLaunchKernelGGL(k_front<R>, dim3((front_grid(m) + 7) / 8 * 8), dim3(kBlock), 0, s, m,
                         (const Six<R>*)w.esig, (const double4*)st.uh, c, front);
      if (front == 0) {  // forced schedule: select this step's entries
        hipError_t e = launch_replay_select(m, c, s);
        if (e != hipSuccess) return e;
      }
    }
    if (mid) {
      hipError_t e = hipEventRecord(mid, s);
      if (e != hipSuccess) return e;
    }
    if (m.tiled == 2) launch_fx<R>(m, st, w, c, mode, fout, s);
    else if (m.lanes == 4) launch_tile_lanes<R, 4>(m, st, w, c, mode, fout, s);
    else if (m.lanes == 16) launch_tile_lanes<R, 16>(m, st, w, c, mode, fout, s);
    else launch_tile_lanes<R, 8>(m, st, w, c, mode, fout, s);
    return hipGetLastError();
  }
  if (m.etype == 8) {
    // the hex crack pass rides along with the element force launch
    const int fg = front > 0 ? (front_grid(m) + 7) / 8 * 8 : 0;
    hipError_t e = launch_elem_force_hex<R>(m, w.esig, w.contrib, (const double4*)st.uh, c, fg,
                                            front > 0, s);
    if (e != hipSuccess) return e;
  } else if (front >= 0) {
    // crack-front workgroups ride along with the element force launch
    const int fg = (front_grid(m) + 7) / 8 * 8;
    hipLaunchKernelGGL(k_elem_force_front<R>, dim3(fg + persistent_grid(m, m.T_cap)), dim3(kBlock), 0,
                       s, m, (const Six<R>*)w.esig, (R*)w.contrib, (const double4*)st.uh, c, fg, front);
    if (front == 0) {  // forced schedule: select this step's entries
      hipError_t e = launch_replay_select(m, c, s);
      if (e != hipSuccess) return e;
    }
  } else {
    hipLaunchKernelGGL(k_elem_force<R>, dim3(persistent_grid(m, m.T_cap)), dim3(kBlock), 0, s, m,
                       (const Six<R>*)w.esig, (R*)w.contrib, c);
  }
  if (mid) {
    hipError_t e = hipEventRecord(mid, s);
    if (e != hipSuccess) return e;
  }
  const R* ct = (const R*)w.contrib;
  const Six<R>* sg = (const Six<R>*)w.esig;
  if (m.lanes == 4) launch_node_lanes<R, 4>(m, st, ct, sg, c, mode, fout, s);
  else if (m.lanes == 16) launch_node_lanes<R, 16>(m, st, ct, sg, c, mode, fout, s);
  else launch_node_lanes<R, 8>(m, st, ct, sg, c, mode, fout, s);
  return hipGetLastError();
}

template <class R>
hipError_t Launch<R>::edge_volumes(const Mesh& m, const Work& w, int count, hipStream_t s) {
  if (count < 0) count = m.E0;
  if (count == 0) return hipSuccess;
  hipLaunchKernelGGL(k_edge_volumes<R>, dim3(grid_for(count)), dim3(kBlock), 0, s, m, (R*)w.einvV,
                     count);
  return hipGetLastError();
}

hipError_t launch_bc_apply(const Mesh& m, const State& st, const Counters* c, hipStream_t s) {
  if (m.n_bc == 0) return hipSuccess;
  hipLaunchKernelGGL(k_bc_apply, dim3(grid_for(m.n_bc)), dim3(kBlock), 0, s, m, st, c);
  return hipGetLastError();
}

hipError_t launch_reaction(const Mesh& m, const Counters* c, hipStream_t s) {
  if (m.n_grp == 0) return hipSuccess;
  hipLaunchKernelGGL(k_reaction, dim3(1), dim3(kBlock), 0, s, m, c);
  return hipGetLastError();
}

hipError_t launch_kap_copies(const Mesh& m, int n_split, hipStream_t s) {
  if (n_split <= 0 || !m.kap) return hipSuccess;
  hipLaunchKernelGGL(k_kap_copies, dim3(grid_for(n_split)), dim3(kBlock), 0, s, m, n_split);
  return hipGetLastError();
}

template struct Launch<double>;
template struct Launch<float>;

template <class R>
hipError_t launch_strain_energy(const Mesh& m, const Work& w, Counters* c, double* partial,
                                int nparts, int inst, hipStream_t s) {
  hipLaunchKernelGGL(k_strain_energy<R>, dim3(nparts), dim3(kBlock), 0, s, m,
                     (const Six<R>*)w.veps, (const R*)w.einvV, partial, c, inst);
  return hipGetLastError();
}
template hipError_t launch_strain_energy<double>(const Mesh&, const Work&, Counters*, double*, int,
                                                 int, hipStream_t);
template hipError_t launch_strain_energy<float>(const Mesh&, const Work&, Counters*, double*, int,
                                                int, hipStream_t);

template <class R>
hipError_t launch_topology_t(const Mesh& m, const State& st, const Work& w, Counters* c,
                             int dynamic, int advance, int4* snodes, int* sedges, hipStream_t s) {
  // a host pre-split (dynamic 0) always takes the whole-chip path for large batches
  Mesh mm = m;
  if (!dynamic) mm.topo_multi = 1;
  if (mm.etype == 8) {  // hex cracks: one workgroup applies the whole batch
    hipLaunchKernelGGL(k_hex_topology<R>, dim3(1), dim3(kTopoBlock), 0, s, mm, w, c, dynamic, advance);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_topology<R>, dim3(1), dim3(kTopoBlock), 0, s, mm, st, w, c, dynamic, advance,
                     snodes, sedges);
  // one-workgroup mode: everything happened in k_topology
  if (!mm.topo_multi) return hipGetLastError();
  hipLaunchKernelGGL(k_topo_apply<R>, dim3(256), dim3(kBlock), 0, s, mm, st, w, c, dynamic, snodes,
                     sedges);
  hipLaunchKernelGGL(k_topo_sums<R>, dim3(256), dim3(kBlock), 0, s, mm, w, c, snodes, sedges);
  hipLaunchKernelGGL(k_topo_finish<R>, dim3(1), dim3(kTopoBlock), 0, s, mm, c, dynamic, advance,
                     (const int4*)snodes);
  return hipGetLastError();
}
template hipError_t launch_topology_t<double>(const Mesh&, const State&, const Work&, Counters*,
                                              int, int, int4*, int*, hipStream_t);
template hipError_t launch_topology_t<float>(const Mesh&, const State&, const Work&, Counters*, int,
                                             int, int4*, int*, hipStream_t);

hipError_t launch_replay_select(const Mesh& m, Counters* c, hipStream_t s) {
  hipLaunchKernelGGL(k_replay_select, dim3(1), dim3(64), 0, s, m, c);
  return hipGetLastError();
}

hipError_t launch_set_presplit(const Mesh& m, Counters* c, const int* tets, const uint8_t* masks,
                               int n, hipStream_t s) {
  int g = grid_for(n);
  if (g < 1) g = 1;
  if (g > 4096) g = 4096;
  hipLaunchKernelGGL(k_set_presplit, dim3(g), dim3(kBlock), 0, s, m, c, tets, masks, n);
  return hipGetLastError();
}

hipError_t launch_normals(const Mesh& m, const Counters* c, hipStream_t s) {
  if (m.etype == 8 || !m.gtab || m.T_cap == 0) return hipSuccess;
  hipLaunchKernelGGL(k_normals, dim3(grid_for(m.T_cap)), dim3(kBlock), 0, s, m, c);
  return hipGetLastError();
}

hipError_t launch_masses(const Mesh& m, hipStream_t s) {
  if (m.etype == 8) {
    hipError_t e = launch_hex_geometry(m, s);
    if (e != hipSuccess) return e;
  } else {
    hipLaunchKernelGGL(k_volumes, dim3(grid_for(m.T0)), dim3(kBlock), 0, s, m);
  }
  hipLaunchKernelGGL(k_masses, dim3(grid_for(m.N0)), dim3(kBlock), 0, s, m);
  return hipGetLastError();
}

hipError_t launch_loads(const Mesh& m, const int4* ftri, const double4* ftrac, const int* lfoff,
                        const int* lfent, hipStream_t s) {
  if (m.n_load == 0) return hipSuccess;
  hipLaunchKernelGGL(k_loads, dim3(grid_for(m.n_load)), dim3(kBlock), 0, s, m, ftri, ftrac, lfoff,
                     lfent);
  return hipGetLastError();
}

hipError_t launch_dtcrit(const Mesh& m, Counters* c, hipStream_t s) {
  if (m.etype == 8) {
    hipError_t e = launch_dtcrit_hex(m, c, s);
    if (e != hipSuccess) return e;
  } else {
    hipLaunchKernelGGL(k_dtcrit, dim3(grid_for(m.T0)), dim3(kBlock), 0, s, m, c);
  }
  hipLaunchKernelGGL(k_dtfinish, dim3(1), dim3(64), 0, s, m, c);
  return hipGetLastError();
}

hipError_t launch_kinetic(const Mesh& m, const State& st, Counters* c, double* partial, int nparts,
                          int inst, hipStream_t s) {
  hipLaunchKernelGGL(k_kinetic, dim3(nparts), dim3(kBlock), 0, s, m, st, c, partial, inst);
  return hipGetLastError();
}

hipError_t launch_work_sum(const Mesh& m, double* out, int inst, hipStream_t s) {
  hipLaunchKernelGGL(k_work_sum, dim3(1), dim3(kBlock), 0, s, m, out, inst);
  return hipGetLastError();
}

hipError_t launch_edge_instances(const Mesh& m, hipStream_t s) {
  hipLaunchKernelGGL(k_edge_instances, dim3(grid_for(m.E0)), dim3(kBlock), 0, s, m);
  return hipGetLastError();
}

hipError_t launch_dissipated(const Mesh& m, Counters* c, double* out, int inst, hipStream_t s) {
  hipLaunchKernelGGL(k_dissipated, dim3(1), dim3(kBlock), 0, s, m, c, out, inst);
  return hipGetLastError();
}

hipError_t launch_sum(const double* partial, int n, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_sum, dim3(1), dim3(kBlock), 0, s, partial, n, out);
  return hipGetLastError();
}

hipError_t launch_count_fronts(const Mesh& m, Counters* c, int* out, int inst, hipStream_t s) {
  hipLaunchKernelGGL(k_count_fronts, dim3(front_grid(m)), dim3(kBlock), 0, s, m, c, out, inst);
  return hipGetLastError();
}

}  // namespace cem
