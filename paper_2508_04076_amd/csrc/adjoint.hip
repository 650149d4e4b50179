// HIP kernels (gfx950) of the reverse sweep over a fixed-topology window of
// explicit steps: the discrete adjoint of the Newmark update (beta = 0,
// gamma = 1/2, end of Section 2.2) with the edge-smoothed internal force of
// Eq. CSTet_fint_discretization.
//
// Forward, per step: u1 = u + dt v + dt^2/2 a;  a1 = M^-1 (r1 F - K u1);
// v1 = v + dt/2 (a + a1).  With p, q the sensitivities of the objective to u
// and v, and lambda = M^-1 (sensitivity to a), one reverse step is
//   f = K lambda                      (strain, edge and element passes on lambda)
//   gE_e -= (V_eff,e / 6) sum_{k in edges(e)} eps_k(lambda) . Chat eps_k(u1)
//   p <- p - f;  q <- q + dt p;  lambda <- M^-1 (dt/2 q_old + dt^2/2 p + dt/2 q)
// where Chat is the elasticity at unit modulus: a per-tet modulus E_e enters
// edge k as C_k = sum_e w_ek E_e Chat, and w_ek V_k = V_eff,e / 6.  K is
// symmetric, so K lambda reuses the forward passes' arithmetic on lambda.
#include "device_util.h"

namespace cem {

// Element strains of lambda and of the window's displacement u, in one pass
// over the element geometry.
template <class R>
__global__ __launch_bounds__(kBlock) void k_strain2(Mesh m, const double4* __restrict__ lam,
                                                    const double4* __restrict__ u,
                                                    Six<R>* __restrict__ vl,
                                                    Six<R>* __restrict__ vu,
                                                    const Counters* __restrict__ c) {
  if (c->err) return;
  const int Tn = elems_now(m, c);
  Chunks it(Tn);
  for (int e; it.next(e);) {
    if (e >= Tn) continue;
    int4 nd = m.enodes[e];
    int code = (unsigned)nd.x >> kNodeBits;
    int n0 = nd.x & kNodeMask;
    R ol[6] = {0, 0, 0, 0, 0, 0}, ou[6] = {0, 0, 0, 0, 0, 0};
    if (code != FR_ZERO) {
      R g[3][3], d[3][3];
      slot_normals<R>(m, e, nd, g);
      R f = (R)(frac_of(code) / 6.0);
      node_diffs(lam[n0], lam[nd.y], lam[nd.z], lam[nd.w], d);
      sym_grad(g, d, f, ol);
      node_diffs(u[n0], u[nd.y], u[nd.z], u[nd.w], d);
      sym_grad(g, d, f, ou);
    }
    store6(vl + e, ol);
    store6(vu + e, ou);
  }
}

// Per edge: sigma_k(lambda) = C_k eps_k(lambda) (einvV carries kappa_k / S_k),
// and z_k = eps_k(lambda) . Chat eps_k(u) with eps = acc / S_k (einv0 = 1 / S_k).
template <class R>
__global__ __launch_bounds__(kBlock) void k_edge2(Mesh m, const Six<R>* __restrict__ vl,
                                                  const Six<R>* __restrict__ vu,
                                                  const R* __restrict__ einvV,
                                                  const R* __restrict__ einv0,
                                                  Six<R>* __restrict__ esig, R* __restrict__ z,
                                                  R lh, R mh, const Counters* __restrict__ c) {
  if (c->err) return;
  const int En = edges_now(m, c);
  Chunks it(En);
  for (int k; it.next(k);) {
    if (k >= En) continue;
    R al[6], au[6], eps[6], sig[6];
    edge_sum(m, vl, k, al);
    edge_sum(m, vu, k, au);
    R iv = einvV[k], i0 = einv0[k];
#pragma unroll
    for (int i = 0; i < 6; ++i) eps[i] = al[i] * iv;
    hooke((R)m.lam, (R)m.mu, eps, sig);
    store6(esig + k, sig);
#pragma unroll
    for (int i = 0; i < 6; ++i) eps[i] = au[i] * i0;
    hooke(lh, mh, eps, sig);
    R s = 0;
#pragma unroll
    for (int i = 0; i < 6; ++i) s += al[i] * i0 * sig[i];
    z[k] = s;
  }
}

// Nodal terms of K lambda (as in the forward element pass, in the context's
// force layout: terms at node-list positions or per-element stress sums) and
// the modulus sensitivity of the element slot, accumulated over the reverse
// steps.
template <class R>
__global__ __launch_bounds__(kBlock) void k_elem_adj(Mesh m, const Six<R>* __restrict__ esig,
                                                     const R* __restrict__ z,
                                                     R* __restrict__ contrib,
                                                     double* __restrict__ gE,
                                                     const Counters* __restrict__ c) {
  if (c->err) return;
  const int Tn = elems_now(m, c);
  Chunks it(Tn);
  for (int e; it.next(e);) {
    if (e >= Tn) continue;
    int4 nd = m.enodes[e];
    int code = (unsigned)nd.x >> kNodeBits;
    if (code != FR_ZERO) {
      int2 q01 = m.et2e[3 * e], q23 = m.et2e[3 * e + 1], q45 = m.et2e[3 * e + 2];
      double zs = (double)z[q01.x] + (double)z[q01.y] + (double)z[q23.x] + (double)z[q23.y] +
                  (double)z[q45.x] + (double)z[q45.y];
      gE[e] -= frac_of(code) * m.vol[e] / 6.0 * zs;
    }
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

// Node update of one reverse step.  last: only p <- p - f (the initial
// acceleration's term).  half: the new lambda's index is >= 1, so it also
// holds dt/2 q from the step before it.
template <class R, int G, bool SSUM>
__global__ __launch_bounds__(kBlock) void k_node_adj(Mesh m, const R* __restrict__ contrib,
                                                     double4* __restrict__ p,
                                                     double4* __restrict__ q,
                                                     double4* __restrict__ lam, int last,
                                                     int half, const Counters* __restrict__ c) {
  if (c->err) return;
  const int Nn = nodes_now(m, c);
  Chunks it((long long)Nn * G);
  const int g = (int)threadIdx.x % G;
  for (int item; it.next(item);) {
    const int i = item / G;
    const bool active = i < Nn;
    double fx, fy, fz;
    if (SSUM) node_gather_tet<R, G>(m, contrib, i, active, g, fx, fy, fz);
    else node_gather<R, G>(m, contrib, i, active, g, fx, fy, fz);
    if (!active || g != 0) continue;
    double4 p0 = p[i];
    double px = p0.x - fx, py = p0.y - fy, pz = p0.z - fz;
    p[i] = make_double4(px, py, pz, 0.0);
    if (last) continue;
    const double dt = node_dt(m, i), h = 0.5 * dt, h2 = 0.5 * dt * dt;
    const double im = m.invm[i];
    double4 q0 = q[i];
    double qx = q0.x + dt * px, qy = q0.y + dt * py, qz = q0.z + dt * pz;
    q[i] = make_double4(qx, qy, qz, 0.0);
    double ax = h * q0.x + h2 * px, ay = h * q0.y + h2 * py, az = h * q0.z + h2 * pz;
    if (half) {
      ax += h * qx;
      ay += h * qy;
      az += h * qz;
    }
    lam[i] = make_double4(im * ax, im * ay, im * az, 0.0);
  }
}

// lambda of the window's last index: M^-1 (coef dt q) (coef 1/2, or 0 for an
// empty window).
__global__ __launch_bounds__(kBlock) void k_adj_init(Mesh m, const double4* __restrict__ q,
                                                     double4* __restrict__ lam, double coef,
                                                     const Counters* __restrict__ c) {
  const int Nn = nodes_now(m, c);
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < Nn; i += gridDim.x * kBlock) {
    double s = coef * node_dt(m, i) * m.invm[i];
    double4 q0 = q[i];
    lam[i] = make_double4(s * q0.x, s * q0.y, s * q0.z, 0.0);
  }
}

// 1 / S_k (the patch's effective volume) of the first `count` edges.
template <class R>
__global__ __launch_bounds__(kBlock) void k_inv_volumes(Mesh m, R* __restrict__ out, int count) {
  int k = blockIdx.x * kBlock + threadIdx.x;
  if (k >= count) return;
  double S = 0;
  for (int p = m.poff[k]; p < m.poff[k + 1]; ++p) {
    int e = m.pent[p];
    if (e >= 0) S += frac_of((unsigned)m.enodes[e].x >> kNodeBits) * m.vol[e];
  }
  out[k] = S > 0 ? (R)(1.0 / S) : (R)0;
}

// ---------------------------------------------------------------- launchers

template <class R>
hipError_t Adjoint<R>::strain2(const Mesh& m, const double4* lam, const double4* u, void* vl,
                               void* vu, const Counters* c, hipStream_t s) {
  hipLaunchKernelGGL(k_strain2<R>, dim3(persistent_grid(m, m.T_cap)), dim3(kBlock), 0, s, m, lam,
                     u, (Six<R>*)vl, (Six<R>*)vu, c);
  return hipGetLastError();
}

template <class R>
hipError_t Adjoint<R>::edge2(const Mesh& m, const void* vl, const void* vu, const void* einvV,
                             const void* einv0, void* esig, void* z, double lh, double mh,
                             const Counters* c, hipStream_t s) {
  hipLaunchKernelGGL(k_edge2<R>, dim3(persistent_grid(m, m.E_cap)), dim3(kBlock), 0, s, m,
                     (const Six<R>*)vl, (const Six<R>*)vu, (const R*)einvV, (const R*)einv0,
                     (Six<R>*)esig, (R*)z, (R)lh, (R)mh, c);
  return hipGetLastError();
}

template <class R>
hipError_t Adjoint<R>::elem(const Mesh& m, const void* esig, const void* z, void* contrib,
                            double* gE, const Counters* c, hipStream_t s) {
  hipLaunchKernelGGL(k_elem_adj<R>, dim3(persistent_grid(m, m.T_cap)), dim3(kBlock), 0, s, m,
                     (const Six<R>*)esig, (const R*)z, (R*)contrib, gE, c);
  return hipGetLastError();
}

template <class R, int G>
static void launch_node_adj(const Mesh& m, const R* ct, double4* p, double4* q, double4* lam,
                            int last, int half, const Counters* c, hipStream_t s) {
  if (m.ssum)
    hipLaunchKernelGGL((k_node_adj<R, G, true>), dim3(persistent_grid(m, (long long)m.N_cap * G)),
                       dim3(kBlock), 0, s, m, ct, p, q, lam, last, half, c);
  else
    hipLaunchKernelGGL((k_node_adj<R, G, false>), dim3(persistent_grid(m, (long long)m.N_cap * G)),
                       dim3(kBlock), 0, s, m, ct, p, q, lam, last, half, c);
}

template <class R>
hipError_t Adjoint<R>::node(const Mesh& m, const void* contrib, double4* p, double4* q,
                            double4* lam, int last, int half, const Counters* c, hipStream_t s) {
  const R* ct = (const R*)contrib;
  if (m.lanes == 4) launch_node_adj<R, 4>(m, ct, p, q, lam, last, half, c, s);
  else if (m.lanes == 16) launch_node_adj<R, 16>(m, ct, p, q, lam, last, half, c, s);
  else launch_node_adj<R, 8>(m, ct, p, q, lam, last, half, c, s);
  return hipGetLastError();
}

template <class R>
hipError_t Adjoint<R>::inv_volumes(const Mesh& m, void* out, int count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_inv_volumes<R>, dim3(grid_for(count)), dim3(kBlock), 0, s, m, (R*)out,
                     count);
  return hipGetLastError();
}

template struct Adjoint<double>;
template struct Adjoint<float>;

hipError_t launch_adj_init(const Mesh& m, const double4* q, double4* lam, double coef,
                           const Counters* c, hipStream_t s) {
  int g = grid_for(m.N_cap);
  g = g < 1 ? 1 : (g > 4096 ? 4096 : g);
  hipLaunchKernelGGL(k_adj_init, dim3(g), dim3(kBlock), 0, s, m, q, lam, coef, c);
  return hipGetLastError();
}

}  // namespace cem
