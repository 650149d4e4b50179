// Hexahedral crack patterns III-VI (Section 3, the parallelepiped element):
// the local hex tables, the candidates of a crack front, their release rates
// and the crack pass, shared by the element force launch that carries the
// crack pass and by the topology and readback kernels.
#ifndef CEM_HEX_CRACK_H
#define CEM_HEX_CRACK_H

#include "device_util.h"

namespace cem {

// Hexahedral crack patterns III-VI (Section 3, the parallelepiped element).
// Cut planes c . xi = d in the hex's natural coordinates pass through edge
// midpoints: mid-planes (d = 0, index = axis), wedge planes (two nonzero
// coefficients, d = 1, index 3 + 4 pair + 2 [c_a > 0] + [c_b > 0] for the
// axis pairs (0,1), (0,2), (1,2)) and corner planes (d = 2, index
// 15 + 4 [c0 > 0] + 2 [c1 > 0] + [c2 > 0]).  A front on local face f runs
// through the midpoints of two of its edges qa < qb; opposite edges give III
// (the mid-plane, which deactivates the hex) and IV (two wedge planes
// tilted toward either side), neighbouring edges V (the wedge plane along
// the face normal) and VI (the corner plane at their shared corner).  After
// IV-VI the hex carries half its volume.

// sign (+1 / -1) of natural coordinate d of local node l: bottom face 0-1-2-3
// counter-clockwise from (-1, -1, -1), top face 4-7 above it
__device__ __forceinline__ int hx_sign(int l, int d) {
  const int b = d == 0 ? ((l ^ (l >> 1)) & 1) : d == 1 ? ((l >> 1) & 1) : (l >> 2);
  return b ? 1 : -1;
}
// local edge q: 0-3 bottom ring, 4-7 top ring, 8-11 verticals
__device__ __forceinline__ int hx_ea(int q) { return q < 8 ? q : q - 8; }
__device__ __forceinline__ int hx_eb(int q) { return q < 4 ? ((q + 1) & 3) : q < 8 ? 4 + ((q - 3) & 3) : q - 4; }
__device__ __forceinline__ int hx_axis(int q) { return q < 8 ? (q & 1) : 2; }
// natural coordinate d of the midpoint of edge q (-1, 0, 1)
__device__ __forceinline__ int hx_mid(int q, int d) { return (hx_sign(hx_ea(q), d) + hx_sign(hx_eb(q), d)) / 2; }

// the edge along `axis` whose midpoint has coordinates w[d] for d != axis
__device__ inline int hx_edge_at(int axis, int w0, int w1, int w2) {
  const int w[3] = {w0, w1, w2};
  for (int q = 0; q < 12; ++q) {
    if (hx_axis(q) != axis) continue;
    bool ok = true;
#pragma unroll
    for (int d = 0; d < 3; ++d)
      if (d != axis && hx_mid(q, d) != w[d]) ok = false;
    if (ok) return q;
  }
  return 0;
}

__device__ __forceinline__ int hx_plane_wedge(const int* cf) {
  const int a = cf[0] ? 0 : 1, b = cf[2] ? 2 : 1;
  const int k = (a == 0 && b == 1) ? 0 : (a == 0 ? 1 : 2);
  return 3 + 4 * k + 2 * (cf[a] > 0) + (cf[b] > 0);
}

// cut-edge mask of plane p (edges whose midpoints lie on it)
__device__ inline int hx_plane_mask(int p) {
  int cf[3] = {0, 0, 0}, d;
  if (p < 3) {
    cf[p] = 1;
    d = 0;
  } else if (p < 15) {
    const int k = (p - 3) >> 2, r = (p - 3) & 3;
    const int a = k == 2 ? 1 : 0, b = k == 0 ? 1 : 2;
    cf[a] = (r & 2) ? 1 : -1;
    cf[b] = (r & 1) ? 1 : -1;
    d = 1;
  } else {
    const int r = p - 15;
    cf[0] = (r & 4) ? 1 : -1;
    cf[1] = (r & 2) ? 1 : -1;
    cf[2] = (r & 1) ? 1 : -1;
    d = 2;
  }
  int m = 0;
  for (int q = 0; q < 12; ++q)
    if (cf[0] * hx_mid(q, 0) + cf[1] * hx_mid(q, 1) + cf[2] * hx_mid(q, 2) == d) m |= 1 << q;
  return m;
}

// the four edges of local face f = 2 axis + (side > 0)
__device__ inline int hx_face_mask(int f) {
  const int axis = f >> 1, side = (f & 1) ? 1 : -1;
  int m = 0;
  for (int q = 0; q < 12; ++q)
    if (hx_sign(hx_ea(q), axis) == side && hx_sign(hx_eb(q), axis) == side) m |= 1 << q;
  return m;
}

// Candidate j of the front (f, qa, qb): plane, pattern and the local edges
// of G1, G2, G3, G4 (G6 in q3 for VI).  Returns false past the last one.
__device__ inline bool hx_candidate(int f, int qa, int qb, int j, int& plane, int& pat, int& q3, int& q4) {
  const int k = f >> 1, s = (f & 1) ? 1 : -1;
  const int i = hx_axis(qa), i2 = hx_axis(qb);
  int w3[3] = {0, 0, 0}, w4[3] = {0, 0, 0};
  if (i == i2) {  // opposite edges along i: III, IV toward -1, IV toward +1
    if (j > 2) return false;
    const int jj = 3 - i - k;
    if (j == 0) {
      w3[jj] = hx_mid(qa, jj); w3[k] = -s;
      w4[jj] = hx_mid(qb, jj); w4[k] = -s;
      plane = i;
      pat = 3;
      q3 = hx_edge_at(i, w3[0], w3[1], w3[2]);
      q4 = hx_edge_at(i, w4[0], w4[1], w4[2]);
      return true;
    }
    const int sg = j == 1 ? -1 : 1;
    int cf[3] = {0, 0, 0};
    cf[i] = sg;
    cf[k] = s;
    w3[i] = sg; w3[jj] = hx_mid(qa, jj);
    w4[i] = sg; w4[jj] = hx_mid(qb, jj);
    plane = hx_plane_wedge(cf);
    pat = 4;
    q3 = hx_edge_at(k, w3[0], w3[1], w3[2]);
    q4 = hx_edge_at(k, w4[0], w4[1], w4[2]);
    return true;
  }
  if (j > 1) return false;  // neighbouring edges: V, VI
  const int p = hx_mid(qa, i2), r = hx_mid(qb, i);
  int cf[3] = {0, 0, 0};
  cf[i] = r;
  cf[i2] = p;
  if (j == 0) {
    w3[i2] = p; w3[k] = -s;
    w4[i] = r; w4[k] = -s;
    plane = hx_plane_wedge(cf);
    pat = 5;
    q3 = hx_edge_at(i, w3[0], w3[1], w3[2]);
    q4 = hx_edge_at(i2, w4[0], w4[1], w4[2]);
    return true;
  }
  cf[k] = s;
  w3[i] = r; w3[i2] = p;
  plane = 15 + 4 * (cf[0] > 0) + 2 * (cf[1] > 0) + (cf[2] > 0);
  pat = 6;
  q3 = hx_edge_at(k, w3[0], w3[1], w3[2]);
  q4 = -1;
  return true;
}

__device__ __forceinline__ void hx_load(const Mesh& m, int t, int* nd, int* ed) {
  const int4 a = m.hnodes[2 * t], b = m.hnodes[2 * t + 1];
  nd[0] = a.x; nd[1] = a.y; nd[2] = a.z; nd[3] = a.w;
  nd[4] = b.x; nd[5] = b.y; nd[6] = b.z; nd[7] = b.w;
#pragma unroll
  for (int r = 0; r < 6; ++r) {
    const int2 e = m.he2e[6 * t + r];
    ed[2 * r] = e.x;
    ed[2 * r + 1] = e.y;
  }
}

__device__ __forceinline__ double3 hx_point(const Mesh& m, const int* nd, int q) {
  const double4 a = m.X[nd[hx_ea(q)]], b = m.X[nd[hx_eb(q)]];
  return make_double3(0.5 * (a.x + b.x), 0.5 * (a.y + b.y), 0.5 * (a.z + b.z));
}

// Eq. stretch-delta on edge q: its end-to-end displacement difference if the
// edge lengthens, else 0
__device__ __forceinline__ double3 hx_stretch(const Mesh& m, const double4* __restrict__ u,
                                              const int* nd, int q) {
  const int a = nd[hx_ea(q)], b = nd[hx_eb(q)];
  const double4 ua = u[a], ub = u[b], xa = m.X[a], xb = m.X[b];
  const double dx = ub.x - ua.x, dy = ub.y - ua.y, dz = ub.z - ua.z;
  const double ex = xb.x - xa.x, ey = xb.y - xa.y, ez = xb.z - xa.z;
  if (2.0 * (ex * dx + ey * dy + ez * dz) + (dx * dx + dy * dy + dz * dz) > 0.0) return make_double3(dx, dy, dz);
  return make_double3(0, 0, 0);
}

__device__ __forceinline__ double3 hx_cross(double3 a, double3 b) {
  return make_double3(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ double3 hx_sub(double3 a, double3 b) { return make_double3(a.x - b.x, a.y - b.y, a.z - b.z); }

// Release rate of a candidate (Eq. G-I over the quad G1 G2 G4 G3, normal of
// its diagonals; Eq. G-II over the triangle G1 G2 G6 for VI)
template <class R>
__device__ double hx_G(const Mesh& m, const double4* __restrict__ u, const Six<R>* __restrict__ esig,
                       const int* nd, const int* ed, int qa, int qb, int pat, int q3, int q4) {
  const double3 P1 = hx_point(m, nd, qa), P2 = hx_point(m, nd, qb), P3 = hx_point(m, nd, q3);
  double3 n = pat == 6 ? hx_cross(hx_sub(P2, P1), hx_sub(P3, P1))
                       : hx_cross(hx_sub(hx_point(m, nd, q4), P1), hx_sub(P3, P2));
  const double l = sqrt(n.x * n.x + n.y * n.y + n.z * n.z);
  n.x /= l; n.y /= l; n.z /= l;
  const double3 d1 = hx_stretch(m, u, nd, qa), d2 = hx_stretch(m, u, nd, qb);
  const double a1 = fabs(d1.x * n.x + d1.y * n.y + d1.z * n.z);
  const double a2 = fabs(d2.x * n.x + d2.y * n.y + d2.z * n.z);
  double sg[6];
  load_sig(esig, ed[q3], sg);
  const double s3 = stress_term(sg, n.x, n.y, n.z, m.gsig);
  if (pat == 6) return 0.5 * s3 * (a1 + a2);
  load_sig(esig, ed[q4], sg);
  const double s4 = stress_term(sg, n.x, n.y, n.z, m.gsig);
  return 0.5 * (s3 * a1 + s4 * a2);
}

// Area of the crack surface of plane p in hex t: the triangle of its three
// cut-edge midpoints, or the quad of four, whose diagonals join the midpoints
// farthest apart in natural coordinates.
__device__ inline double hx_plane_area(const Mesh& m, const int* nd, int p) {
  const int cut = hx_plane_mask(p);
  int qs[4], n = 0;
  for (int q = 0; q < 12; ++q)
    if ((cut >> q) & 1) qs[n++] = q;
  double3 P[4];
  for (int r = 0; r < n; ++r) P[r] = hx_point(m, nd, qs[r]);
  double3 x;
  if (n == 3) {
    x = hx_cross(hx_sub(P[1], P[0]), hx_sub(P[2], P[0]));
  } else {
    int far = 1, best = -1;
    for (int r = 1; r < 4; ++r) {
      int d2 = 0;
      for (int d = 0; d < 3; ++d) {
        const int v = hx_mid(qs[r], d) - hx_mid(qs[0], d);
        d2 += v * v;
      }
      if (d2 > best) { best = d2; far = r; }
    }
    int o0 = -1, o1 = -1;
    for (int r = 1; r < 4; ++r)
      if (r != far) { if (o0 < 0) o0 = r; else o1 = r; }
    x = hx_cross(hx_sub(P[far], P[0]), hx_sub(P[o1], P[o0]));
  }
  return 0.5 * sqrt(x.x * x.x + x.y * x.y + x.z * x.z);
}

// Crack pass of a hex mesh, run by workgroups blk of nblk: eight lanes per
// candidate hex, lane f < 6 takes its face f (the face's best candidate, ties
// to the earlier one); lane 0 then takes the best face (ties to the lower
// face) and runs the Griffith test G >= Gc, appending the hex to the
// (unordered) split list.
template <class R>
__device__ void hex_front_block(const Mesh& m, const double4* __restrict__ u,
                                const Six<R>* __restrict__ esig, Counters* __restrict__ c,
                                int flagging, int blk, int nblk, unsigned long long* red) {
  unsigned long long kmax = 0;
  const int nc = c->n_cand;
  const int room = m.S_cap - c->n_split;
  const int f = threadIdx.x & 7;
  constexpr int cpb = kBlock / 8;
  for (int base = blk * cpb; base < nc; base += nblk * cpb) {
    const int idx = base + (int)threadIdx.x / 8;
    const int t = idx < nc ? m.cand[idx] : -1;
    const bool act = t >= 0 && m.smask[t] < 0;
    const int code = act && f < 6 ? m.hfront[6 * t + f] : -1;
    double G = -INFINITY;
    int plane = 0, pat = 0;
    if (code >= 0) {
      int nd[8], ed[12];
      hx_load(m, t, nd, ed);
      const int qa = code >> 4, qb = code & 15;
      int pl, pt, q3, q4;
      for (int j = 0; hx_candidate(f, qa, qb, j, pl, pt, q3, q4); ++j) {
        const double g = hx_G<R>(m, u, esig, nd, ed, qa, qb, pt, q3, q4);
        if (j == 0 || g > G) { G = g; plane = pl; pat = pt; }
      }
    }
    double gq[6];
    int pq[6], tq[6], hq[6];
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      gq[q] = __shfl(G, q, 8);
      pq[q] = __shfl(plane, q, 8);
      tq[q] = __shfl(pat, q, 8);
      hq[q] = __shfl(code, q, 8) >= 0;
    }
    if (f != 0 || !act) continue;
    double best = -INFINITY;
    int bplane = 0, bpat = 0;
    bool any = false;
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      if (!hq[q]) continue;
      if (!any || gq[q] > best) { best = gq[q]; bplane = pq[q]; bpat = tq[q]; }
      any = true;
    }
    if (!any) continue;
    const unsigned long long k = dkey(best);
    kmax = k > kmax ? k : kmax;
    if (flagging && best >= m.Gc) {
      m.pmask[t] = (uint8_t)bplane;
      m.ppat[t] = (uint8_t)bpat;
      m.pG[t] = best;
      const int slot = atomicAdd(&c->n_flag, 1);
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

}  // namespace cem

#endif
