// Host runtime of libcem: context, mesh preprocessing, buffers, time-step
// driver (plain launches or captured HIP graphs) and the C-ABI of cem.h.
#include "../../include/cem.h"
#include "cem_device.h"


#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>
#include <string>
#include <mutex>
#include <vector>

using namespace cem;

// events per profiled step: before strain, edge, crack, element force, node
// sum, topology, and after topology
constexpr int kEvents = 7;

namespace {

struct Region {
  void* ptr;
  size_t bytes;
};

}  // namespace

struct cem_ctx {
  cem_options opt{};
  std::string err;
  int stage = 0;  // 0 created, 1 mesh uploaded
  hipStream_t stream = nullptr;
  cem_material mat{};
  int mixed = 0;

  Mesh m{};
  Work w{};
  State st{};
  Counters* d_ctr = nullptr;
  Counters* h_ctr = nullptr;  // pinned mirror
  int4* d_snodes = nullptr;
  int* d_sedges = nullptr;
  double4* d_tmp = nullptr;   // internal_force input / output staging
  double4* d_tmp2 = nullptr;
  double* d_out = nullptr;    // scalar outputs of reductions
  int* d_iout = nullptr;
  int n_partial = 1024;
  bool bound = false;
  bool own_stream = false;
  unsigned char* scratch = nullptr;  // this device's static staging (cem_read_front_G_static)

  // host mirrors (internal numbering)
  std::vector<double> X;       // 3 N0
  std::vector<int> tets;       // 4 T0, oriented
  // the library renumbers nodes and tets for locality; the API keeps the
  // caller's numbering
  std::vector<int> node_new, node_old;  // [N0]
  std::vector<int> inst_nodes, inst_tets;  // original nodes / tets per instance
  std::vector<int> tet_new, tet_old;    // [T0]
  std::vector<char> split_host;
  int n_split_host = 0;
  long long step_host = 0;
  bool dt_set = false;
  bool need_init = true;
  bool traction_set = false;

  // traction staging
  int4* d_ftri = nullptr;
  double4* d_ftrac = nullptr;
  int* d_lfoff = nullptr;
  int* d_lfent = nullptr;
  int n_faces = 0;

  // graph
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  int graph_steps = 0;
  int graph_replay = -1;
  // how the last cem_step call ran: steps, graph launches, steps per graph,
  // steps as plain launches
  int64_t last_run[4] = {0, 0, 0, 0};

  // profiling
  hipEvent_t tev[2] = {nullptr, nullptr};  // whole-call timing (created once)
  int profiling = 0;
  double times[7] = {0, 0, 0, 0, 0, 0, 0};
  std::vector<hipEvent_t> evpool;

  std::vector<void*> allocs;
  std::vector<Region> regions;  // checkpointed device arrays

  // prescribed-velocity groups (host mirror, internal node ids)
  std::vector<int> bc_node, bc_mask;      // mask | group << 4
  std::vector<double4> bc_v0;
  std::vector<double> bc_t0;              // per group
  std::vector<int> bc_goff{0};            // slot range per group

  // per-tet modulus (relative to mat.E); m.kap points at it while on
  double* kap_buf = nullptr;
  bool kap_on = false;

  // any change of state, mesh or launch shape bumps gen (discards a window)
  long long gen = 0;
  int frozen = 0;        // steps skip the crack pass
  int topo_mode = 0;     // 0 auto, 1 one workgroup, 2 whole chip for large split batches
  int graph_frozen = -1;

  // fixed-topology gradient window
  struct Window {
    int n = 0, every = 1, n_ck = 0, nodes = 0, n_split = 0;
    long long gen = -1;
    double4* ck = nullptr;    // [n_ck][4][nodes] u, v, a, predictor
    Counters* ckc = nullptr;  // [n_ck]
    double* ckw = nullptr;    // [n_ck][n_load] external work per loaded node
    double4* tape = nullptr;  // [every + 1][nodes] displacement along a segment
    double4* p = nullptr;     // [nodes] dJ/du
    double4* q = nullptr;     // [nodes] dJ/dv
    double4* lam = nullptr;   // [nodes] M^-1 dJ/da
    double* gE = nullptr;     // [T_cap] dJ/dE per element slot
    void* vu = nullptr;       // [T_cap] Six<R>: V_eff eps(u)
    void* z = nullptr;        // [E_cap] R
    void* einv0 = nullptr;    // [E_cap] R: 1 / patch volume
    size_t ck_bytes = 0, tape_bytes = 0;
    std::vector<void*> fixed;  // buffers sized by the mesh (allocated once)
    double times[6] = {0, 0, 0, 0, 0, 0};
  } win;

  int fail(int code, const std::string& msg) {
    err = msg;
    return code;
  }
};

namespace {

#define HIPCHK(ctx, expr)                                                        \
  do {                                                                           \
    hipError_t e_ = (expr);                                                      \
    if (e_ != hipSuccess)                                                        \
      return (ctx)->fail(CEM_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

template <class T>
int dalloc(cem_ctx* c, T** p, size_t count, bool checkpoint = false) {
  size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
  void* q = nullptr;
  hipError_t e = hipMalloc(&q, bytes);
  if (e != hipSuccess) {
    return c->fail(e == hipErrorOutOfMemory ? CEM_ENOMEM : CEM_EHIP,
                   std::string("hipMalloc: ") + hipGetErrorString(e));
  }
  c->allocs.push_back(q);
  *p = (T*)q;
  if (checkpoint) c->regions.push_back({q, bytes});
  return CEM_OK;
}

// Stable LSD radix sort of (key, value) pairs on the low `bits` bits of key.
void radix_sort(std::vector<uint64_t>& key, std::vector<uint32_t>& val, int bits) {
  size_t n = key.size();
  std::vector<uint64_t> k2(n);
  std::vector<uint32_t> v2(n);
  for (int shift = 0; shift < bits; shift += 16) {
    std::vector<size_t> cnt(65537, 0);
    for (size_t i = 0; i < n; ++i) cnt[((key[i] >> shift) & 0xffff) + 1]++;
    for (int d = 0; d < 65536; ++d) cnt[d + 1] += cnt[d];
    for (size_t i = 0; i < n; ++i) {
      size_t pos = cnt[(key[i] >> shift) & 0xffff]++;
      k2[pos] = key[i];
      v2[pos] = val[i];
    }
    key.swap(k2);
    val.swap(v2);
  }
}

int bits_for(uint64_t maxv) {
  int b = 1;
  while (b < 64 && (maxv >> b)) ++b;
  return b;
}

const int kLE[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};
// hex edges (node order: bottom face 0-1-2-3 counter-clockwise, top face 4-7)
const int kHexLE[12][2] = {{0, 1}, {1, 2}, {2, 3}, {3, 0}, {4, 5}, {5, 6},
                           {6, 7}, {7, 4}, {0, 4}, {1, 5}, {2, 6}, {3, 7}};

int local_edge_h(int a, int b) {
  int lo = std::min(a, b), hi = std::max(a, b);
  for (int q = 0; q < 6; ++q)
    if (kLE[q][0] == lo && kLE[q][1] == hi) return q;
  return -1;
}

struct HostTopo {
  int E0 = 0;
  std::vector<int> et2e;      // 6 T0
  std::vector<int> poff;      // E0 + 1
  std::vector<int> pent;      // 6 T0
  std::vector<int> patchpos;  // 6 T0
  std::vector<int> noff;      // N0 + 1
  std::vector<int> nent;      // 4 T0
  std::vector<int> nodepos;   // 4 T0
  std::vector<int> nbr;       // 4 T0
  std::vector<int> nbrface;   // T0 packed
};

// Orientation fix and degeneracy test (Section 2.2 needs V_j > 0).
int check_orient(cem_ctx* c, int N, const double* X, int T, std::vector<int>& tets) {
  double lsum = 0;
  for (int t = 0; t < T; ++t)
    for (int q = 0; q < 6; ++q) {
      const double* a = X + 3 * tets[4 * t + kLE[q][0]];
      const double* b = X + 3 * tets[4 * t + kLE[q][1]];
      lsum += std::sqrt((a[0] - b[0]) * (a[0] - b[0]) + (a[1] - b[1]) * (a[1] - b[1]) +
                        (a[2] - b[2]) * (a[2] - b[2]));
    }
  double lm = T ? lsum / (6.0 * T) : 0;
  double tol = 1e-12 * lm * lm * lm;
  (void)N;
  for (int t = 0; t < T; ++t) {
    int* n = &tets[4 * t];
    const double *x0 = X + 3 * n[0], *x1 = X + 3 * n[1], *x2 = X + 3 * n[2], *x3 = X + 3 * n[3];
    double ax = x1[0] - x0[0], ay = x1[1] - x0[1], az = x1[2] - x0[2];
    double bx = x2[0] - x0[0], by = x2[1] - x0[1], bz = x2[2] - x0[2];
    double cx = x3[0] - x0[0], cy = x3[1] - x0[1], cz = x3[2] - x0[2];
    double V = (ax * (by * cz - bz * cy) + ay * (bz * cx - bx * cz) + az * (bx * cy - by * cx)) / 6.0;
    if (!(std::fabs(V) > tol))
      return c->fail(CEM_EMESH, "degenerate tetrahedron " + std::to_string(t));
    if (V < 0) std::swap(n[2], n[3]);
  }
  return CEM_OK;
}

// Hilbert-curve node order (3D, 21 bits per axis), one connected component
// after another (components in the order of their first node, each on its own
// bounding box, so a batch of meshes is ordered exactly as its members would
// be alone).  The index is Skilling's transposed-axes construction (J.
// Skilling, "Programming the Hilbert curve", AIP Conf. Proc. 707, 2004) read
// out level by level.  Nearby nodes get nearby ids in all three directions
// with no long jumps, so a block of consecutive elements touches a compact
// region of the mesh however large it is.
void hilbert_order(int N, int T, int K, const std::vector<int>& elems, const double* X,
                   std::vector<int>& new_of_old) {
  const int b = 21;
  // connected components (union-find over the element node lists)
  std::vector<int> par(N);
  for (int i = 0; i < N; ++i) par[i] = i;
  auto find = [&](int x) {
    while (par[x] != x) x = par[x] = par[par[x]];
    return x;
  };
  for (int t = 0; t < T; ++t) {
    int r0 = find(elems[(size_t)K * t]);
    for (int l = 1; l < K; ++l) {
      int r = find(elems[(size_t)K * t + l]);
      if (r != r0) par[std::max(r, r0)] = std::min(r, r0);
      r0 = std::min(r, r0);
    }
  }
  std::vector<int> comp(N), first(N, -1);
  int nc = 0;
  for (int i = 0; i < N; ++i) {
    int r = find(i);
    if (first[r] < 0) first[r] = nc++;
    comp[i] = first[r];
  }
  std::vector<double> lo((size_t)3 * nc, 1e300), hi((size_t)3 * nc, -1e300);
  for (int i = 0; i < N; ++i)
    for (int d = 0; d < 3; ++d) {
      lo[3 * (size_t)comp[i] + d] = std::min(lo[3 * (size_t)comp[i] + d], X[3 * (size_t)i + d]);
      hi[3 * (size_t)comp[i] + d] = std::max(hi[3 * (size_t)comp[i] + d], X[3 * (size_t)i + d]);
    }
  std::vector<uint64_t> key(N);
  std::vector<uint32_t> val(N);
  for (int i = 0; i < N; ++i) {
    const double* cl = &lo[3 * (size_t)comp[i]];
    const double* ch = &hi[3 * (size_t)comp[i]];
    double span = std::max(ch[0] - cl[0], std::max(ch[1] - cl[1], ch[2] - cl[2]));
    double sc = span > 0 ? 2097151.0 / span : 0.0;
    uint32_t x[3];
    for (int d = 0; d < 3; ++d) x[d] = (uint32_t)((X[3 * (size_t)i + d] - cl[d]) * sc);
    // axes -> transposed Hilbert index
    for (uint32_t q = 1u << (b - 1); q > 1; q >>= 1) {
      uint32_t p = q - 1;
      for (int d = 0; d < 3; ++d) {
        if (x[d] & q) {
          x[0] ^= p;
        } else {
          uint32_t t = (x[0] ^ x[d]) & p;
          x[0] ^= t;
          x[d] ^= t;
        }
      }
    }
    for (int d = 1; d < 3; ++d) x[d] ^= x[d - 1];
    uint32_t t = 0;
    for (uint32_t q = 1u << (b - 1); q > 1; q >>= 1)
      if (x[2] & q) t ^= q - 1;
    for (int d = 0; d < 3; ++d) x[d] ^= t;
    uint64_t k = 0;
    for (int lev = b - 1; lev >= 0; --lev)
      for (int d = 0; d < 3; ++d) k = (k << 1) | ((x[d] >> lev) & 1u);
    key[i] = k;
    val[i] = (uint32_t)i;
  }
  radix_sort(key, val, 3 * b);  // by curve index (stable)
  for (int k = 0; k < N; ++k) key[k] = (uint64_t)comp[val[k]];
  radix_sort(key, val, bits_for((uint64_t)std::max(nc - 1, 1)));  // then by component
  new_of_old.assign(N, 0);
  for (int k = 0; k < N; ++k) new_of_old[val[k]] = k;
}

// Node tiles of the tiled force pass: runs of consecutive (Hilbert-ordered)
// node ids whose node-list entries fit in cap, and per tile the
// ascending tets that have an entry there.  Returns false (no tiles) if a
// node alone has more entries than a tile holds.
bool build_tiles(int N, const HostTopo& h, int cap, std::vector<int>& toff, std::vector<int>& ttoff,
                 std::vector<int>& ttet) {
  toff.assign(1, 0);
  for (int i = 0; i < N; ++i) {
    if (h.noff[i + 1] - h.noff[i] > cap) return false;
    if (h.noff[i + 1] - h.noff[toff.back()] > cap) toff.push_back(i);
  }
  toff.push_back(N);
  const int nt = (int)toff.size() - 1;
  ttoff.assign(1, 0);
  ttet.clear();
  std::vector<int> tmp;
  for (int b = 0; b < nt; ++b) {
    tmp.clear();
    for (int p = h.noff[toff[b]]; p < h.noff[toff[b + 1]]; ++p) tmp.push_back(h.nent[p] >> 2);
    std::sort(tmp.begin(), tmp.end());
    tmp.erase(std::unique(tmp.begin(), tmp.end()), tmp.end());
    ttet.insert(ttet.end(), tmp.begin(), tmp.end());
    ttoff.push_back((int)ttet.size());
  }
  return true;
}

// Nodes per tile of the fixed-point tiled pass: kFxNodes, or fewer (a multiple
// of 64, at least kFxMinNodes) when that gives at least kFxTargetTiles tiles.
static int fx_tile_nodes(int N) {
  int t = (int)(((long long)N + kFxTargetTiles - 1) / kFxTargetTiles);
  t = (t + 63) / 64 * 64;
  return std::min(kFxNodes, std::max(kFxMinNodes, t));
}

// Tiles of the fixed-point tiled pass: runs of fx_tile_nodes(N) consecutive
// nodes, each with the parent tets that have an entry in it (ascending).
void build_tiles_fx(int N, const HostTopo& h, std::vector<int>& toff, std::vector<int>& ttoff,
                    std::vector<int>& ttet) {
  const int tn = fx_tile_nodes(N);
  toff.clear();
  for (int i = 0; i < N; i += tn) toff.push_back(i);
  toff.push_back(N);
  const int nt = (int)toff.size() - 1;
  ttoff.assign(1, 0);
  ttet.clear();
  std::vector<int> tmp;
  for (int b = 0; b < nt; ++b) {
    tmp.clear();
    for (int p = h.noff[toff[b]]; p < h.noff[toff[b + 1]]; ++p) tmp.push_back(h.nent[p] >> 2);
    std::sort(tmp.begin(), tmp.end());
    tmp.erase(std::unique(tmp.begin(), tmp.end()), tmp.end());
    ttet.insert(ttet.end(), tmp.begin(), tmp.end());
    ttoff.push_back((int)ttet.size());
  }
}

// Largest |G_l|_1 over the tets and their local nodes (G_l = 6 V grad N_l:
// G_1 = c2 x c3, G_2 = c3 x c1, G_3 = c1 x c2, G_0 = -(G_1 + G_2 + G_3)).
double max_face_normal_l1(int T, const std::vector<int>& tets, const double* X) {
  double g1 = 0.0;
  for (int t = 0; t < T; ++t) {
    const double* x0 = X + 3 * (size_t)tets[4 * t];
    double cc[3][3];
    for (int l = 0; l < 3; ++l)
      for (int d = 0; d < 3; ++d) cc[l][d] = X[3 * (size_t)tets[4 * t + 1 + l] + d] - x0[d];
    double G[4][3];
    for (int l = 0; l < 3; ++l) {
      const double* a = cc[(l + 1) % 3];
      const double* b = cc[(l + 2) % 3];
      G[l + 1][0] = a[1] * b[2] - a[2] * b[1];
      G[l + 1][1] = a[2] * b[0] - a[0] * b[2];
      G[l + 1][2] = a[0] * b[1] - a[1] * b[0];
    }
    for (int d = 0; d < 3; ++d) G[0][d] = -(G[1][d] + G[2][d] + G[3][d]);
    for (int l = 0; l < 4; ++l)
      g1 = std::max(g1, std::fabs(G[l][0]) + std::fabs(G[l][1]) + std::fabs(G[l][2]));
  }
  return g1;
}

int build_topology(cem_ctx* c, int N, int T, const std::vector<int>& tets, HostTopo& h) {
  // edges: sort (min, max) node-pair keys of every (tet, local edge)
  size_t M = (size_t)6 * T;
  std::vector<uint64_t> key(M);
  std::vector<uint32_t> val(M);
  for (int t = 0; t < T; ++t)
    for (int q = 0; q < 6; ++q) {
      uint64_t a = (uint32_t)tets[4 * t + kLE[q][0]], b = (uint32_t)tets[4 * t + kLE[q][1]];
      if (a > b) std::swap(a, b);
      key[(size_t)6 * t + q] = (a << 32) | b;
      val[(size_t)6 * t + q] = (uint32_t)(6 * t + q);
    }
  int nb = bits_for((uint64_t)std::max(N - 1, 1));
  // sort on b (low word) then a (high word)
  {
    std::vector<uint64_t> k2(M);
    for (size_t i = 0; i < M; ++i) k2[i] = (key[i] >> 32 << nb) | (key[i] & 0xffffffffull);
    radix_sort(k2, val, 2 * nb);
    for (size_t i = 0; i < M; ++i) key[i] = k2[i];
  }
  h.et2e.assign(M, -1);
  h.patchpos.assign(M, -1);
  h.pent.assign(M, -1);
  h.poff.clear();
  int E = 0;
  for (size_t i = 0; i < M; ++i) {
    if (i == 0 || key[i] != key[i - 1]) {
      h.poff.push_back((int)i);
      E++;
    }
    uint32_t tq = val[i];
    h.et2e[tq] = E - 1;
    h.patchpos[tq] = (int)i;
    h.pent[i] = (int)(tq / 6);
  }
  h.poff.push_back((int)M);
  h.E0 = E;
  // node lists: counting sort of (node, tet, local) in tet order
  h.noff.assign(N + 1, 0);
  for (int t = 0; t < T; ++t)
    for (int l = 0; l < 4; ++l) h.noff[tets[4 * t + l] + 1]++;
  for (int i = 0; i < N; ++i) h.noff[i + 1] += h.noff[i];
  std::vector<int> fill(h.noff.begin(), h.noff.end() - 1);
  h.nent.assign((size_t)4 * T, 0);
  h.nodepos.assign((size_t)4 * T, 0);
  for (int t = 0; t < T; ++t)
    for (int l = 0; l < 4; ++l) {
      int p = fill[tets[4 * t + l]]++;
      h.nent[p] = (t << 2) | l;
      h.nodepos[(size_t)4 * t + l] = p;
    }
  // faces: key (edge id of the two smallest nodes, largest node)
  size_t F = (size_t)4 * T;
  std::vector<uint64_t> fk(F);
  std::vector<uint32_t> fv(F);
  for (int t = 0; t < T; ++t)
    for (int f = 0; f < 4; ++f) {
      int ln[3], k = 0;
      for (int l = 0; l < 4; ++l)
        if (l != f) ln[k++] = l;
      std::sort(ln, ln + 3, [&](int x, int y) { return tets[4 * t + x] < tets[4 * t + y]; });
      int eid = h.et2e[(size_t)6 * t + local_edge_h(ln[0], ln[1])];
      fk[(size_t)4 * t + f] = ((uint64_t)eid << nb) | (uint32_t)tets[4 * t + ln[2]];
      fv[(size_t)4 * t + f] = (uint32_t)(4 * t + f);
    }
  radix_sort(fk, fv, nb + bits_for((uint64_t)std::max(E - 1, 1)));
  h.nbr.assign(F, -1);
  h.nbrface.assign(T, 0);
  for (size_t i = 0; i < F;) {
    size_t j = i;
    while (j < F && fk[j] == fk[i]) ++j;
    if (j - i > 2) return c->fail(CEM_EMESH, "face shared by more than two tetrahedra");
    if (j - i == 2) {
      uint32_t p = fv[i], q = fv[i + 1];
      int tp = p / 4, fp = p % 4, tq = q / 4, fq = q % 4;
      if (tp == tq) return c->fail(CEM_EMESH, "tetrahedron with a repeated face");
      h.nbr[p] = tq;
      h.nbr[q] = tp;
      h.nbrface[tp] |= fq << (8 * fp);
      h.nbrface[tq] |= fp << (8 * fq);
    }
    i = j;
  }
  for (int t = 0; t < T; ++t)
    for (int f = 0; f < 4; ++f)
      for (int g = f + 1; g < 4; ++g)
        if (h.nbr[4 * t + f] >= 0 && h.nbr[4 * t + f] == h.nbr[4 * t + g])
          return c->fail(CEM_EMESH, "duplicated tetrahedron " + std::to_string(t));
  return CEM_OK;
}

// Hex mesh topology: edges (12 per hex) with their patches, node lists with
// eight entries per hex and each (hex, local) entry's position.
struct HexTopo {
  int E0 = 0;
  std::vector<int> he2e;     // 12 H
  std::vector<int> poff;     // E0 + 1
  std::vector<int> pent;     // 12 H: 12 hex + local edge (the hex's record at that edge's point)
  std::vector<int> noff;     // N + 1
  std::vector<int> nent;     // 8 H: hex << 3 | local
  std::vector<int> nodepos;  // 8 H: position of entry (hex, local) in the node lists
};

void build_hex_topology(int N, int H, const std::vector<int>& hx, HexTopo& h) {
  size_t M = (size_t)12 * H;
  std::vector<uint64_t> key(M);
  std::vector<uint32_t> val(M);
  int nb = bits_for((uint64_t)std::max(N - 1, 1));
  for (int t = 0; t < H; ++t)
    for (int q = 0; q < 12; ++q) {
      uint64_t a = (uint32_t)hx[8 * (size_t)t + kHexLE[q][0]], b = (uint32_t)hx[8 * (size_t)t + kHexLE[q][1]];
      if (a > b) std::swap(a, b);
      key[(size_t)12 * t + q] = (a << nb) | b;
      val[(size_t)12 * t + q] = (uint32_t)(12 * t + q);
    }
  radix_sort(key, val, 2 * nb);
  h.he2e.assign(M, -1);
  h.pent.assign(M, -1);
  h.poff.clear();
  int E = 0;
  for (size_t i = 0; i < M; ++i) {
    if (i == 0 || key[i] != key[i - 1]) {
      h.poff.push_back((int)i);
      E++;
    }
    h.he2e[val[i]] = E - 1;
    h.pent[i] = (int)val[i];
  }
  h.poff.push_back((int)M);
  h.E0 = E;
  h.noff.assign(N + 1, 0);
  for (size_t i = 0; i < (size_t)8 * H; ++i) h.noff[hx[i] + 1]++;
  for (int i = 0; i < N; ++i) h.noff[i + 1] += h.noff[i];
  std::vector<int> fill(h.noff.begin(), h.noff.end() - 1);
  h.nent.assign((size_t)8 * H, 0);
  h.nodepos.assign((size_t)8 * H, 0);
  for (int t = 0; t < H; ++t)
    for (int l = 0; l < 8; ++l) {
      int p = fill[hx[8 * (size_t)t + l]]++;
      h.nent[p] = (t << 3) | l;
      h.nodepos[8 * (size_t)t + l] = p;
    }
}

// Face neighbours of a hex mesh: out[6 t + f] = 8 u + g when local face f of
// hex t (f = 2 axis + (side > 0); bottom face 0-1-2-3, top 4-7) is local face
// g of hex u, else -1.  Faces are matched by their sorted node ids.
bool hex_face_neighbours(int H, const std::vector<int>& hx, std::vector<int>& out) {
  static const int kFace[6][4] = {{0, 3, 4, 7}, {1, 2, 5, 6}, {0, 1, 4, 5},
                                  {2, 3, 6, 7}, {0, 1, 2, 3}, {4, 5, 6, 7}};
  struct Rec {
    unsigned long long k0, k1;
    int id;
  };
  std::vector<Rec> rec((size_t)6 * H);
  for (int t = 0; t < H; ++t)
    for (int f = 0; f < 6; ++f) {
      int a[4];
      for (int j = 0; j < 4; ++j) a[j] = hx[8 * (size_t)t + kFace[f][j]];
      std::sort(a, a + 4);
      rec[6 * (size_t)t + f] = {((unsigned long long)a[0] << 32) | (unsigned)a[1],
                                ((unsigned long long)a[2] << 32) | (unsigned)a[3], 8 * t + f};
    }
  std::sort(rec.begin(), rec.end(), [](const Rec& x, const Rec& y) {
    return x.k0 != y.k0 ? x.k0 < y.k0 : x.k1 != y.k1 ? x.k1 < y.k1 : x.id < y.id;
  });
  out.assign((size_t)6 * H, -1);
  for (size_t i = 0; i + 1 < rec.size(); ++i)
    if (rec[i].k0 == rec[i + 1].k0 && rec[i].k1 == rec[i + 1].k1) {
      if (i + 2 < rec.size() && rec[i + 2].k0 == rec[i].k0 && rec[i + 2].k1 == rec[i].k1) return false;
      const int a = rec[i].id, b = rec[i + 1].id;
      out[6 * (size_t)(a >> 3) + (a & 7)] = b;
      out[6 * (size_t)(b >> 3) + (b & 7)] = a;
      ++i;
    }
  return true;
}

// Jacobian determinants of a trilinear hex at its 2 x 2 x 2 Gauss points:
// returns their minimum and maximum.
void hex_det_range(const double* X, const int* nd, double* dmin, double* dmax) {
  static const int sg[8][3] = {{-1, -1, -1}, {1, -1, -1}, {1, 1, -1}, {-1, 1, -1},
                               {-1, -1, 1},  {1, -1, 1},  {1, 1, 1},  {-1, 1, 1}};
  const double a = 1.0 / std::sqrt(3.0);
  *dmin = INFINITY;
  *dmax = -INFINITY;
  // the eight Gauss points, then the twelve edge midpoints
  for (int pt = 0; pt < 20; ++pt) {
    double xi[3];
    for (int d = 0; d < 3; ++d)
      xi[d] = pt < 8 ? a * sg[pt][d] : 0.5 * (sg[kHexLE[pt - 8][0]][d] + sg[kHexLE[pt - 8][1]][d]);
    double J[3][3] = {};
    for (int i = 0; i < 8; ++i) {
      double f[3];
      for (int d = 0; d < 3; ++d) f[d] = 1.0 + xi[d] * sg[i][d];
      double dN[3] = {0.125 * sg[i][0] * f[1] * f[2], 0.125 * f[0] * sg[i][1] * f[2],
                      0.125 * f[0] * f[1] * sg[i][2]};
      const double* x = X + 3 * (size_t)nd[i];
      for (int r = 0; r < 3; ++r)
        for (int cc = 0; cc < 3; ++cc) J[r][cc] += x[r] * dN[cc];
    }
    double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                 J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                 J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
    *dmin = std::min(*dmin, det);
    *dmax = std::max(*dmax, det);
  }
}

template <class T>
int upload(cem_ctx* c, T* d, const T* h, size_t n) {
  if (n == 0) return CEM_OK;
  HIPCHK(c, hipMemcpyAsync(d, h, n * sizeof(T), hipMemcpyHostToDevice, c->stream));
  return CEM_OK;
}

int sync(cem_ctx* c) {
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return CEM_OK;
}

int read_counters(cem_ctx* c) {
  HIPCHK(c, hipMemcpyAsync(c->h_ctr, c->d_ctr, sizeof(Counters), hipMemcpyDeviceToHost, c->stream));
  return sync(c);
}

int check_device_error(cem_ctx* c) {
  int r = read_counters(c);
  if (r) return r;
  c->n_split_host = c->h_ctr->n_split;
  c->step_host = c->h_ctr->step;
  int e = c->h_ctr->err;
  if (e) {
    int zero = 0;
    HIPCHK(c, hipMemcpyAsync(&c->d_ctr->err, &zero, sizeof(int), hipMemcpyHostToDevice, c->stream));
    int r2 = sync(c);
    if (r2) return r2;
    if (e == CEM_ECAPACITY)
      return c->fail(e, "split capacity exhausted at step " + std::to_string(c->h_ctr->step + 1) +
                            " (state left at the start of that step)");
    if (e == CEM_EUNSTABLE)
      return c->fail(e, "non-finite or runaway state near step " + std::to_string(c->h_ctr->step + 1));
    return c->fail(e, "device error");
  }
  c->n_split_host = c->h_ctr->n_split;
  c->step_host = c->h_ctr->step;
  return CEM_OK;
}

template <class R>
int launch_strain_stress(cem_ctx* c, const double4* u) {
  HIPCHK(c, Launch<R>::strain(c->m, u, c->w, c->d_ctr, c->stream));
  HIPCHK(c, Launch<R>::edge_stress(c->m, c->w, c->d_ctr, c->stream));
  return CEM_OK;
}

int strain_stress(cem_ctx* c, const double4* u) {
  return c->mixed ? launch_strain_stress<float>(c, u) : launch_strain_stress<double>(c, u);
}

int node_pass(cem_ctx* c, int mode, double4* fout, hipEvent_t mid = nullptr, int front = -1) {
  hipError_t e = c->mixed ? Launch<float>::node(c->m, c->st, c->w, c->d_ctr, mode, fout, c->stream, mid, front)
                          : Launch<double>::node(c->m, c->st, c->w, c->d_ctr, mode, fout, c->stream, mid, front);
  HIPCHK(c, e);
  return CEM_OK;
}

int initialize(cem_ctx* c) {
  HIPCHK(c, launch_bc_apply(c->m, c->st, c->d_ctr, c->stream));
  int r = strain_stress(c, c->st.u);
  if (r) return r;
  r = node_pass(c, NODE_INIT, nullptr);
  if (r) return r;
  c->need_init = false;
  return CEM_OK;
}

// Kernels of one step, in order; ev (if not null) brackets the passes.
int enqueue_step(cem_ctx* c, hipEvent_t* ev) {
  hipStream_t s = c->stream;
  bool replay = c->h_ctr->n_sched > 0;
  if (ev) HIPCHK(c, hipEventRecord(ev[0], s));
  if (c->mixed) HIPCHK(c, Launch<float>::strain(c->m, c->st.uh, c->w, c->d_ctr, s));
  else HIPCHK(c, Launch<double>::strain(c->m, c->st.uh, c->w, c->d_ctr, s));
  if (ev) HIPCHK(c, hipEventRecord(ev[1], s));
  if (c->mixed) HIPCHK(c, Launch<float>::edge_stress(c->m, c->w, c->d_ctr, s));
  else HIPCHK(c, Launch<double>::edge_stress(c->m, c->w, c->d_ctr, s));
  if (ev) HIPCHK(c, hipEventRecord(ev[2], s));
  bool fracture = (std::isfinite(c->mat.Gc) || replay) && !c->frozen;
  // the crack pass runs inside the element force launch (its own workgroups)
  if (ev) HIPCHK(c, hipEventRecord(ev[3], s));
  int r = node_pass(c, NODE_STEP, nullptr, ev ? ev[4] : nullptr, fracture ? (replay ? 0 : 1) : -1);
  if (r) return r;
  if (ev) HIPCHK(c, hipEventRecord(ev[5], s));
  HIPCHK(c, launch_reaction(c->m, c->d_ctr, s));
  if (c->mixed)
    HIPCHK(c, launch_topology_t<float>(c->m, c->st, c->w, c->d_ctr, 1, 1, c->d_snodes, c->d_sedges, s));
  else
    HIPCHK(c, launch_topology_t<double>(c->m, c->st, c->w, c->d_ctr, 1, 1, c->d_snodes, c->d_sedges, s));
  if (ev) HIPCHK(c, hipEventRecord(ev[6], s));
  return CEM_OK;
}

void drop_graph(cem_ctx* c) {
  if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
  if (c->graph) (void)hipGraphDestroy(c->graph);
  c->gexec = nullptr;
  c->graph = nullptr;
  c->graph_steps = 0;
}

int ensure_events(cem_ctx* c, size_t n) {
  for (size_t i = c->evpool.size(); i < n; ++i) {
    hipEvent_t e;
    HIPCHK(c, hipEventCreate(&e));
    c->evpool.push_back(e);
  }
  return CEM_OK;
}

// The two events that time a whole call (created on first use, destroyed
// with the context).
int timing_events(cem_ctx* c) {
  for (int q = 0; q < 2; ++q)
    if (!c->tev[q]) HIPCHK(c, hipEventCreate(&c->tev[q]));
  return CEM_OK;
}

// Sum the per-pass intervals of k recorded steps (kEvents events per step).
int accumulate_times(cem_ctx* c, int k) {
  for (int i = 0; i < k; ++i)
    for (int q = 1; q < kEvents; ++q) {
      float ms = 0;
      HIPCHK(c, hipEventElapsedTime(&ms, c->evpool[kEvents * i + q - 1], c->evpool[kEvents * i + q]));
      c->times[q] += ms;
    }
  return CEM_OK;
}

// Capture k steps into a graph.
int build_graph(cem_ctx* c, int k) {
  drop_graph(c);
  int r = CEM_OK;
  HIPCHK(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeRelaxed));
  for (int i = 0; i < k && r == CEM_OK; ++i) r = enqueue_step(c, nullptr);
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(c->stream, &g);
  if (r) {
    if (g) (void)hipGraphDestroy(g);
    return r;
  }
  if (e != hipSuccess) return c->fail(CEM_EHIP, std::string("graph capture: ") + hipGetErrorString(e));
  c->graph = g;
  HIPCHK(c, hipGraphInstantiate(&c->gexec, g, nullptr, nullptr, 0));
  c->graph_steps = k;
  c->graph_replay = c->h_ctr->n_sched > 0;
  c->graph_frozen = c->frozen;
  return CEM_OK;
}

int ensure_ready(cem_ctx* c, bool need_dt) {
  if (c->stage < 1) return c->fail(CEM_ESTATE, "no mesh uploaded");
  if (need_dt && !c->dt_set) return c->fail(CEM_ESTATE, "time step not set (cem_set_dt)");
  return CEM_OK;
}

// Host [n][3] arrays in the caller's node numbering <-> padded device rows
// in the internal numbering (extra nodes N0 + 4 s + l keep their ids).
int node_int(const cem_ctx* c, int i) { return i < c->m.N0 ? c->node_new[i] : i; }

void pad3(const cem_ctx* c, const double* src, std::vector<double4>& dst, int n) {
  dst.resize(n);
  for (int i = 0; i < n; ++i)
    dst[node_int(c, i)] = make_double4(src[3 * i], src[3 * i + 1], src[3 * i + 2], 0.0);
}

void unpad3(const cem_ctx* c, const std::vector<double4>& src, double* dst, int n) {
  for (int i = 0; i < n; ++i) {
    const double4& q = src[node_int(c, i)];
    dst[3 * i] = q.x;
    dst[3 * i + 1] = q.y;
    dst[3 * i + 2] = q.z;
  }
}

int nodes_now_host(cem_ctx* c) {
  // the device counters are authoritative (splits happen inside cem_step)
  if (read_counters(c) == CEM_OK) {
    c->n_split_host = c->h_ctr->n_split;
    c->step_host = c->h_ctr->step;
  }
  return c->m.N0 + (c->m.mode == MODE_PHANTOM ? 4 * c->n_split_host : 0);
}

// n steps on the context stream (graphs of K steps where possible); checks
// the device error word at the end.
int run_steps(cem_ctx* c, int32_t n_steps) {
  int r;
  if (n_steps == 0) return CEM_OK;
  if ((r = timing_events(c))) return r;
  hipEvent_t e0 = c->tev[0], e1 = c->tev[1];
  HIPCHK(c, hipEventRecord(e0, c->stream));
  if (c->need_init && (r = initialize(c))) return r;
  for (int q = 0; q < 7; ++q) c->times[q] = 0;
  const int splits0 = c->h_ctr->n_split;
  int K = c->opt.graph_steps;
  int done = 0;
  c->last_run[0] = n_steps;
  c->last_run[1] = c->last_run[2] = c->last_run[3] = 0;
  // HIP cannot time events recorded inside a graph: profiling uses plain launches
  if (!c->profiling && K > 0 && n_steps >= K) {
    int replay = c->h_ctr->n_sched > 0;
    if (!c->gexec || c->graph_steps != K || c->graph_replay != replay ||
        c->graph_frozen != c->frozen) {
      if ((r = build_graph(c, K))) return r;
    }
    while (n_steps - done >= K) {
      HIPCHK(c, hipGraphLaunch(c->gexec, c->stream));
      done += K;
      c->last_run[1]++;
    }
    c->last_run[2] = K;
  }
  if (c->profiling) {
    const int chunk = 64;
    if ((r = ensure_events(c, kEvents * chunk))) return r;
    while (done < n_steps) {
      int k = std::min(chunk, n_steps - done);
      for (int i = 0; i < k; ++i)
        if ((r = enqueue_step(c, &c->evpool[kEvents * i]))) return r;
      if ((r = sync(c))) return r;
      if ((r = accumulate_times(c, k))) return r;
      done += k;
    }
  }
  c->last_run[3] = n_steps - (int64_t)c->last_run[1] * c->last_run[2];
  for (; done < n_steps; ++done)
    if ((r = enqueue_step(c, nullptr))) return r;
  HIPCHK(c, hipEventRecord(e1, c->stream));
  r = check_device_error(c);
  float ms = 0;
  (void)hipEventElapsedTime(&ms, e0, e1);
  c->times[0] = ms;
  if (r == CEM_OK && c->topo_mode == 0) {
    // automatic topology mode: large split batches over the whole chip while
    // the run splits more than 64 tets per step, one workgroup again below 16
    // (the same results either way; only the launches differ)
    const double rate = (double)(c->h_ctr->n_split - splits0) / n_steps;
    const int want = c->m.topo_multi ? (rate >= 16.0) : (rate > 64.0);
    if (want != c->m.topo_multi) {
      c->m.topo_multi = want;
      drop_graph(c);
    }
  }
  return r;
}


// ---- gradient windows

int win_alloc(cem_ctx* c, void** p, size_t bytes) {
  hipError_t e = hipMalloc(p, std::max<size_t>(bytes, 16));
  if (e != hipSuccess)
    return c->fail(e == hipErrorOutOfMemory ? CEM_ENOMEM : CEM_EHIP,
                   std::string("hipMalloc: ") + hipGetErrorString(e));
  return CEM_OK;
}

// Buffers sized by the mesh capacity, allocated on the first window.
int win_fixed(cem_ctx* c) {
  auto& W = c->win;
  if (W.p) return CEM_OK;
  const Mesh& m = c->m;
  // float64-sized whatever the precision (cem_set_precision can change it)
  const size_t RS = sizeof(double);
  void* b[7] = {};
  size_t sz[7] = {sizeof(double4) * m.N_cap, sizeof(double4) * m.N_cap, sizeof(double4) * m.N_cap,
                  sizeof(double) * m.T_cap, RS * 6 * (size_t)m.T_cap, RS * (size_t)m.E_cap,
                  RS * (size_t)m.E_cap};
  for (int i = 0; i < 7; ++i) {
    int r = win_alloc(c, &b[i], sz[i]);
    if (r) return r;
    W.fixed.push_back(b[i]);
  }
  W.p = (double4*)b[0];
  W.q = (double4*)b[1];
  W.lam = (double4*)b[2];
  W.gE = (double*)b[3];
  W.vu = b[4];
  W.z = b[5];
  W.einv0 = b[6];
  return CEM_OK;
}

int win_grow(cem_ctx* c, void** p, size_t* have, size_t bytes) {
  if (*have >= bytes && *p) return CEM_OK;
  if (*p) (void)hipFree(*p);
  *p = nullptr;
  *have = 0;
  int r = win_alloc(c, p, bytes);
  if (r) return r;
  *have = bytes;
  return CEM_OK;
}

// Checkpoint j of the window: node state, counters and external work.
int win_save(cem_ctx* c, int j) {
  auto& W = c->win;
  const size_t nb = sizeof(double4) * W.nodes;
  double4* src[4] = {c->st.u, c->st.v, c->st.a, c->st.uh};
  for (int q = 0; q < 4; ++q)
    HIPCHK(c, hipMemcpyAsync(W.ck + ((size_t)4 * j + q) * W.nodes, src[q], nb,
                             hipMemcpyDeviceToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(W.ckc + j, c->d_ctr, sizeof(Counters), hipMemcpyDeviceToDevice, c->stream));
  if (c->m.n_load)
    HIPCHK(c, hipMemcpyAsync(W.ckw + (size_t)j * c->m.n_load, c->m.wacc, sizeof(double) * c->m.n_load,
                             hipMemcpyDeviceToDevice, c->stream));
  return CEM_OK;
}

int win_load(cem_ctx* c, int j) {
  auto& W = c->win;
  const size_t nb = sizeof(double4) * W.nodes;
  double4* dst[4] = {c->st.u, c->st.v, c->st.a, c->st.uh};
  for (int q = 0; q < 4; ++q)
    HIPCHK(c, hipMemcpyAsync(dst[q], W.ck + ((size_t)4 * j + q) * W.nodes, nb,
                             hipMemcpyDeviceToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(c->d_ctr, W.ckc + j, sizeof(Counters), hipMemcpyDeviceToDevice, c->stream));
  if (c->m.n_load)
    HIPCHK(c, hipMemcpyAsync(c->m.wacc, W.ckw + (size_t)j * c->m.n_load, sizeof(double) * c->m.n_load,
                             hipMemcpyDeviceToDevice, c->stream));
  c->need_init = false;
  return CEM_OK;
}

int edges_now_host(const cem_ctx* c) {
  return c->m.E0 + (c->m.mode == MODE_PHANTOM ? 10 * c->n_split_host : 0);
}

// One reverse step: index s + 1 -> s (last: the initial acceleration's term).
template <class R>
int reverse_step(cem_ctx* c, const double4* u1, int last, int half, double lh, double mh,
                 hipEvent_t* ev) {
  auto& W = c->win;
  hipStream_t s = c->stream;
  if (ev) HIPCHK(c, hipEventRecord(ev[0], s));
  HIPCHK(c, Adjoint<R>::strain2(c->m, W.lam, u1, c->w.veps, W.vu, c->d_ctr, s));
  if (ev) HIPCHK(c, hipEventRecord(ev[1], s));
  HIPCHK(c, Adjoint<R>::edge2(c->m, c->w.veps, W.vu, c->w.einvV, W.einv0, c->w.esig, W.z, lh, mh,
                              c->d_ctr, s));
  if (ev) HIPCHK(c, hipEventRecord(ev[2], s));
  HIPCHK(c, Adjoint<R>::elem(c->m, c->w.esig, W.z, c->w.contrib, W.gE, c->d_ctr, s));
  if (ev) HIPCHK(c, hipEventRecord(ev[3], s));
  HIPCHK(c, Adjoint<R>::node(c->m, c->w.contrib, W.p, W.q, W.lam, last, half, c->d_ctr, s));
  if (ev) HIPCHK(c, hipEventRecord(ev[4], s));
  return CEM_OK;
}

// The reverse sweep proper (state and adjoint buffers set up by the caller).
template <class R>
int reverse_window(cem_ctx* c) {
  auto& W = c->win;
  double lh, mh;
  {
    const double nu = c->mat.nu;
    lh = nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
    mh = 1.0 / (2.0 * (1.0 + nu));
  }
  const bool prof = c->profiling != 0;
  int r;
  hipEvent_t* ev = nullptr;
  if (prof) {
    if ((r = ensure_events(c, (size_t)5 * (W.every + 1) + 2))) return r;
    ev = c->evpool.data();
  }
  const size_t nb = sizeof(double4) * W.nodes;
  for (int j = W.n_ck - 2; j >= 0; --j) {
    const int s0 = j * W.every;
    const int len = std::min(W.every, W.n - s0);
    if ((r = win_load(c, j))) return r;
    if (prof) HIPCHK(c, hipEventRecord(ev[5 * W.every], c->stream));
    HIPCHK(c, hipMemcpyAsync(W.tape, c->st.u, nb, hipMemcpyDeviceToDevice, c->stream));
    for (int i = 0; i < len; ++i) {
      if ((r = enqueue_step(c, nullptr))) return r;
      HIPCHK(c, hipMemcpyAsync(W.tape + (size_t)(i + 1) * W.nodes, c->st.u, nb,
                               hipMemcpyDeviceToDevice, c->stream));
    }
    if (prof) HIPCHK(c, hipEventRecord(ev[5 * W.every + 1], c->stream));
    for (int i = len - 1; i >= 0; --i) {
      const int s = s0 + i;  // this reverse step takes index s + 1 to s
      r = reverse_step<R>(c, W.tape + (size_t)(i + 1) * W.nodes, 0, s >= 1 ? 1 : 0, lh, mh,
                          prof ? ev + 5 * i : nullptr);
      if (r) return r;
    }
    if (prof) {
      if ((r = sync(c))) return r;
      float ms = 0;
      HIPCHK(c, hipEventElapsedTime(&ms, ev[5 * W.every], ev[5 * W.every + 1]));
      W.times[1] += ms;
      for (int i = 0; i < len; ++i)
        for (int q = 0; q < 4; ++q) {
          HIPCHK(c, hipEventElapsedTime(&ms, ev[5 * i + q], ev[5 * i + q + 1]));
          W.times[2 + q] += ms;
        }
    }
  }
  if (W.n == 0) {
    if ((r = win_load(c, 0))) return r;
    HIPCHK(c, hipMemcpyAsync(W.tape, c->st.u, nb, hipMemcpyDeviceToDevice, c->stream));
  }
  // a_0 = M^-1 (r_0 F - K u_0): the tape's first row holds u_0 now
  return reverse_step<R>(c, W.tape, 1, 0, lh, mh, nullptr);
}

// ---- allocation-free read of the crack-front release rates
//
// cem_read_front_G_static stages its device results in one file-scope device
// array instead of buffers it allocates: room for kStaticFronts front slots
// (four per crack-front candidate tet) as packed records, the raw
// (tet, face, lone) and (G_I, G_II) arrays the front kernel writes, and the
// record count.  Every GPU holds its own copy until the process ends; host
// code reaches it only through the address hipGetSymbolAddress returns for
// that device (the array's name is a host-side stand-in).
constexpr int kStaticFronts = 65536;
constexpr size_t kStaticRecBytes = (size_t)kStaticFronts * sizeof(cem_front_g);
constexpr size_t kStaticTflBytes = (size_t)kStaticFronts * 3 * sizeof(int);
constexpr size_t kStaticGBytes = (size_t)kStaticFronts * 2 * sizeof(double);
constexpr size_t kStaticBytes = kStaticRecBytes + kStaticTflBytes + kStaticGBytes + 256;
static_assert(sizeof(cem_front_g) == 32, "front record layout");
static_assert((kStaticRecBytes + kStaticTflBytes) % 8 == 0, "G array alignment");

static __device__ __align__(256) unsigned char scratch[kStaticBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned char* g_scratch_dev[kMaxDevices] = {};

// The device address of `scratch` on the context's device, looked up once per
// device with that device current.
int static_scratch(cem_ctx* c, unsigned char** out) {
  const int dev = c->opt.device;
  if (dev >= kMaxDevices) return c->fail(CEM_EINVAL, "device ordinal above 63");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    HIPCHK(c, hipSetDevice(dev));
    void* ptr = nullptr;
    hipError_t e = hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return c->fail(CEM_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_dev[dev] = (unsigned char*)ptr;
  }
  *out = g_scratch_dev[dev];
  return CEM_OK;
}

__global__ void k_zero_count(int* n) {
  if (blockIdx.x == 0 && threadIdx.x == 0) *n = 0;
}

// (tet, face, lone) and (G_I, G_II) of front o -> one packed record.
__global__ void k_pack_fronts(const int* __restrict__ tfl, const double* __restrict__ g,
                              const int* __restrict__ n, cem_front_g* __restrict__ rec) {
  int o = blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= *n) return;
  cem_front_g r;
  r.tet = tfl[3 * o];
  r.face = tfl[3 * o + 1];
  r.lone = tfl[3 * o + 2];
  r.pad = 0;
  r.G_I = g[2 * o];
  r.G_II = g[2 * o + 1];
  rec[o] = r;
}

}  // namespace

extern "C" {

int cem_create(const cem_options* opt, cem_ctx** out) {
  if (!opt || !out) return CEM_EINVAL;
  *out = nullptr;
  if (opt->precision != CEM_FP64 && opt->precision != CEM_MIXED) return CEM_EINVAL;
  if (opt->split_mode != CEM_PHANTOM && opt->split_mode != CEM_ERODE) return CEM_EINVAL;
  if (opt->gsig != CEM_GSIG_PRINCIPAL && opt->gsig != CEM_GSIG_NORMAL) return CEM_EINVAL;
  if (opt->max_splits < 0 || opt->graph_steps < 0 || opt->device < 0) return CEM_EINVAL;
  cem_ctx* c = new cem_ctx();
  c->opt = *opt;
  c->stream = (hipStream_t)opt->stream;
  c->mixed = opt->precision == CEM_MIXED;
  *out = c;
  return CEM_OK;
}

void cem_destroy(cem_ctx* c) {
  if (!c) return;
  if (c->stage >= 1) {
    (void)hipSetDevice(c->opt.device);
    (void)hipStreamSynchronize(c->stream);
    drop_graph(c);
    for (auto e : c->evpool) (void)hipEventDestroy(e);
    for (auto e : c->tev)
      if (e) (void)hipEventDestroy(e);
    for (void* p : c->allocs) (void)hipFree(p);
    for (void* p : c->win.fixed) (void)hipFree(p);
    (void)hipFree(c->win.ck);
    (void)hipFree(c->win.tape);
    if (c->h_ctr) (void)hipHostFree(c->h_ctr);
    if (c->own_stream) (void)hipStreamDestroy(c->stream);
  }
  delete c;
}

const char* cem_last_error(const cem_ctx* c) { return c ? c->err.c_str() : "null context"; }

int cem_upload_mesh(cem_ctx* c, int32_t N, const double* X, int32_t T, const int32_t* tets,
                    const cem_material* mat) {
  if (!c) return CEM_EINVAL;
  if (c->stage != 0) return c->fail(CEM_ESTATE, "mesh already uploaded");
  if (!X || !tets || !mat || N < 4 || T < 1) return c->fail(CEM_EINVAL, "empty mesh");
  if (N > kNodeMask / 2 || (long long)T * 6 > (1LL << 30))
    return c->fail(CEM_EINVAL, "mesh too large for 32-bit indexing");
  if (!(mat->E > 0) || !(mat->rho > 0) || !(mat->nu > -1.0 && mat->nu < 0.5) || !(mat->Gc > 0))
    return c->fail(CEM_EINVAL, "invalid material");
  for (long long i = 0; i < (long long)T * 4; ++i)
    if (tets[i] < 0 || tets[i] >= N) return c->fail(CEM_EMESH, "node id out of range");
  for (long long i = 0; i < (long long)N * 3; ++i)
    if (!std::isfinite(X[i])) return c->fail(CEM_EINVAL, "non-finite coordinate");
  std::vector<int> ext(tets, tets + (size_t)4 * T);
  int r = check_orient(c, N, X, T, ext);
  if (r) return r;
  // internal numbering: nodes along a Hilbert curve per component, tets by their
  // smallest new node id (stable in the caller's order)
  hilbert_order(N, T, 4, ext, X, c->node_new);
  c->node_old.assign(N, 0);
  for (int i = 0; i < N; ++i) c->node_old[c->node_new[i]] = i;
  {
    std::vector<int> cnt(N + 1, 0), key(T);
    for (int t = 0; t < T; ++t) {
      int mn = N;
      for (int l = 0; l < 4; ++l) mn = std::min(mn, c->node_new[ext[4 * t + l]]);
      key[t] = mn;
      cnt[mn + 1]++;
    }
    for (int i = 0; i < N; ++i) cnt[i + 1] += cnt[i];
    c->tet_new.assign(T, 0);
    c->tet_old.assign(T, 0);
    for (int t = 0; t < T; ++t) {
      int nt = cnt[key[t]]++;
      c->tet_new[t] = nt;
      c->tet_old[nt] = t;
    }
  }
  c->tets.assign((size_t)4 * T, 0);
  for (int t = 0; t < T; ++t)
    for (int l = 0; l < 4; ++l) c->tets[4 * (size_t)c->tet_new[t] + l] = c->node_new[ext[4 * t + l]];
  c->X.assign((size_t)3 * N, 0.0);
  for (int i = 0; i < N; ++i)
    for (int d = 0; d < 3; ++d) c->X[3 * (size_t)c->node_new[i] + d] = X[3 * (size_t)i + d];
  X = c->X.data();
  HostTopo h;
  r = build_topology(c, N, T, c->tets, h);
  if (r) return r;

  // ---- device side
  HIPCHK(c, hipSetDevice(c->opt.device));
  {
    int rs = static_scratch(c, &c->scratch);  // set-up of the static staging, once per device
    if (rs) return rs;
  }
  if (!c->stream) {
    // graphs cannot capture the legacy null stream: use a stream of our own
    HIPCHK(c, hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
    c->own_stream = true;
  }
  c->mat = *mat;
  Mesh& m = c->m;
  const int S = c->opt.max_splits;
  const bool ph = c->opt.split_mode == CEM_PHANTOM;
  m.T0 = T;
  m.N0 = N;
  m.E0 = h.E0;
  m.S_cap = S;
  m.T_cap = T + (ph ? S : 0);
  m.N_cap = N + (ph ? 4 * S : 0);
  m.E_cap = h.E0 + (ph ? 10 * S : 0);
  m.mode = c->opt.split_mode;
  m.gsig = c->opt.gsig;
  m.lam = mat->E * mat->nu / ((1 + mat->nu) * (1 - 2 * mat->nu));
  m.mu = mat->E / (2 * (1 + mat->nu));
  m.rho = mat->rho;
  m.Gc = mat->Gc;
  m.ramp_t0 = 0;
  m.dt = 0;
  m.grid_cap = kDefaultGridCap;
  m.lanes = kDefaultLanes;
  m.ssum = 0;
  m.tiled = 0;
  m.ntile[0] = m.ntile[1] = 0;
  m.topo_multi = 0;
  m.n_inst = 0;
  m.etype = 4;
  m.inst = m.tinst = m.einst = nullptr;
  m.dti = m.dtc_inst = nullptr;
  m.gmax_inst = m.lam_inst = nullptr;
  {
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int i = 0; i < N; ++i)
      for (int d = 0; d < 3; ++d) {
        lo[d] = std::min(lo[d], X[3 * i + d]);
        hi[d] = std::max(hi[d], X[3 * i + d]);
      }
    double diag = std::sqrt((hi[0] - lo[0]) * (hi[0] - lo[0]) + (hi[1] - lo[1]) * (hi[1] - lo[1]) +
                            (hi[2] - lo[2]) * (hi[2] - lo[2]));
    m.umax = diag;  // a small-strain displacement as large as the body is a blow-up
  }
  HIPCHK(c, hipHostMalloc((void**)&c->h_ctr, sizeof(Counters), hipHostMallocDefault));
  std::memset(c->h_ctr, 0, sizeof(Counters));
  c->stage = 1;  // allocations from here are released by cem_destroy

  // the float-typed work arrays are sized for float64 in either precision, so
  // that cem_set_precision can switch the arithmetic without reallocating
  const size_t RS = sizeof(double);
  size_t nsplit_list = 1;  // a power of two >= S (room for the bitonic sort)
  while (nsplit_list < (size_t)std::max(S, 1)) nsplit_list <<= 1;
#define ALLOC(ptr, n, ck) \
  if ((r = dalloc(c, &(ptr), (n), (ck)))) return r
  ALLOC(c->d_ctr, 1, true);
  ALLOC(m.enodes, m.T_cap, true);
  ALLOC(m.et2e, (size_t)3 * m.T_cap, true);
  ALLOC(m.X, m.N_cap, true);
  ALLOC(m.poff, (size_t)m.E_cap + 1, false);
  ALLOC(m.pent, (size_t)6 * T + 10 * (ph ? S : 0), true);
  ALLOC(m.noff, (size_t)m.N_cap + 1, false);
  ALLOC(m.nent, (size_t)4 * T + 4 * (ph ? S : 0), true);
  ALLOC(m.invm, m.N_cap, true);
  ALLOC(m.lslot, m.N_cap, true);
  ALLOC(m.nbr, T, false);
  ALLOC(m.nbrface, T, false);
  ALLOC(m.epos, m.T_cap, true);
  ALLOC(m.tet_ext, T, false);
  ALLOC(m.vol, m.T_cap, true);
  ALLOC(m.patchpos, (size_t)3 * T, false);
  ALLOC(m.front, T, true);
  ALLOC(m.smask, T, true);
  ALLOC(m.pmask, T, true);
  ALLOC(m.ppat, T, true);
  ALLOC(m.pG, T, true);
  ALLOC(m.cand, T, true);
  ALLOC(m.candf, T, true);
  ALLOC(m.splitlist, nsplit_list, false);
  ALLOC(m.area, std::max(S, 1), false);
  ALLOC(m.rec_step, std::max(S, 1), true);
  ALLOC(m.rec_tet, std::max(S, 1), true);
  ALLOC(m.rec_mask, std::max(S, 1), true);
  ALLOC(m.rec_pat, std::max(S, 1), true);
  ALLOC(m.rec_G, std::max(S, 1), true);
  ALLOC(m.rec_area, std::max(S, 1), true);
  ALLOC(m.split_of, T, true);
  for (int p = 0; p < 2; ++p) {
    std::vector<int> toff, ttoff, ttet;
    m.toff[p] = m.ttoff[p] = m.ttet[p] = nullptr;
    if (build_tiles(N, h, p ? kTileEntries32 : kTileEntries64, toff, ttoff, ttet)) {
      m.ntile[p] = (int)toff.size() - 1;
      ALLOC(m.toff[p], toff.size(), false);
      ALLOC(m.ttoff[p], ttoff.size(), false);
      ALLOC(m.ttet[p], ttet.size(), false);
      if ((r = upload(c, m.toff[p], toff.data(), toff.size()))) return r;
      if ((r = upload(c, m.ttoff[p], ttoff.data(), ttoff.size()))) return r;
      if ((r = upload(c, m.ttet[p], ttet.data(), ttet.size()))) return r;
    }
  }
  {
    std::vector<int> toff, ttoff, ttet;
    build_tiles_fx(N, h, toff, ttoff, ttet);
    m.ntile_fx = (int)toff.size() - 1;
    ALLOC(m.toff_fx, toff.size(), false);
    ALLOC(m.ttoff_fx, ttoff.size(), false);
    ALLOC(m.ttet_fx, std::max<size_t>(ttet.size(), 1), false);
    if ((r = upload(c, m.toff_fx, toff.data(), toff.size()))) return r;
    if ((r = upload(c, m.ttoff_fx, ttoff.data(), ttoff.size()))) return r;
    if (!ttet.empty() && (r = upload(c, m.ttet_fx, ttet.data(), ttet.size()))) return r;
    ALLOC(m.sig_slot, (size_t)kSigSlots * kSigStride, false);
    ALLOC(m.gtab, (size_t)9 * m.T_cap, false);
    m.fx_g1 = max_face_normal_l1(T, c->tets, c->X.data());
    m.fx_deg = 0;
    for (int i = 0; i < N; ++i) m.fx_deg = std::max(m.fx_deg, h.noff[i + 1] - h.noff[i]);
  }
  ALLOC(c->d_snodes, std::max(S, 1), false);
  ALLOC(c->d_sedges, (size_t)6 * std::max(S, 1), false);
  char* vb;
  ALLOC(vb, RS * 6 * (size_t)m.T_cap, false);
  c->w.veps = vb;
  ALLOC(vb, RS * 6 * (size_t)m.E_cap, false);
  c->w.esig = vb;
  ALLOC(vb, RS * (size_t)m.E_cap, true);
  c->w.einvV = vb;
  // three values per node-list entry, four entries per element slot (the
  // stress sums take six per slot)
  ALLOC(vb, RS * 12 * (size_t)m.T_cap, false);
  c->w.contrib = vb;
  ALLOC(c->w.partial, c->n_partial, false);
  ALLOC(c->d_out, 8, false);
  ALLOC(c->d_iout, 8, false);
  ALLOC(c->st.u, m.N_cap, true);
  ALLOC(c->st.v, m.N_cap, true);
  ALLOC(c->st.a, m.N_cap, true);
  ALLOC(c->st.uh, m.N_cap, true);
  ALLOC(c->d_tmp, m.N_cap, false);
  ALLOC(c->d_tmp2, m.N_cap, false);
  m.sched = nullptr;
  m.Fload = nullptr;
  m.wacc = nullptr;
  m.lnode = nullptr;
  m.n_load = 0;

  // host images of the initial device arrays
  std::vector<int4> en(m.T_cap, make_int4(0, 0, 0, 0));
  for (int t = 0; t < T; ++t)
    en[t] = make_int4(c->tets[4 * t] | (FR_ONE << kNodeBits), c->tets[4 * t + 1], c->tets[4 * t + 2],
                      c->tets[4 * t + 3]);
  if ((r = upload(c, m.enodes, en.data(), en.size()))) return r;
  std::vector<int2> t2e((size_t)3 * m.T_cap, make_int2(0, 0));
  for (size_t i = 0; i < (size_t)3 * T; ++i) t2e[i] = make_int2(h.et2e[2 * i], h.et2e[2 * i + 1]);
  if ((r = upload(c, m.et2e, t2e.data(), t2e.size()))) return r;
  std::vector<double4> Xp(m.N_cap, make_double4(0, 0, 0, 0));
  for (int i = 0; i < N; ++i) Xp[i] = make_double4(X[3 * i], X[3 * i + 1], X[3 * i + 2], 0.0);
  if ((r = upload(c, m.X, Xp.data(), Xp.size()))) return r;
  std::vector<int> poff(m.E_cap + 1);
  for (int k = 0; k <= h.E0; ++k) poff[k] = h.poff[k];
  for (int k = h.E0 + 1; k <= m.E_cap; ++k) poff[k] = 6 * T + (k - h.E0);
  if ((r = upload(c, m.poff, poff.data(), poff.size()))) return r;
  std::vector<int> pent((size_t)6 * T + 10 * (ph ? S : 0), -1);
  std::copy(h.pent.begin(), h.pent.end(), pent.begin());
  if ((r = upload(c, m.pent, pent.data(), pent.size()))) return r;
  std::vector<int> noff(m.N_cap + 1);
  for (int i = 0; i <= N; ++i) noff[i] = h.noff[i];
  for (int i = N + 1; i <= m.N_cap; ++i) noff[i] = 4 * T + (i - N);
  if ((r = upload(c, m.noff, noff.data(), noff.size()))) return r;
  std::vector<int> nent((size_t)4 * T + 4 * (ph ? S : 0), 0);
  std::copy(h.nent.begin(), h.nent.end(), nent.begin());
  if ((r = upload(c, m.nent, nent.data(), nent.size()))) return r;
  std::vector<int> lsl(m.N_cap, -1);
  if ((r = upload(c, m.lslot, lsl.data(), lsl.size()))) return r;
  if ((r = upload(c, (int*)m.nbr, h.nbr.data(), h.nbr.size()))) return r;
  if ((r = upload(c, m.nbrface, h.nbrface.data(), h.nbrface.size()))) return r;
  if ((r = upload(c, m.tet_ext, c->tet_old.data(), (size_t)T))) return r;
  std::vector<int> ep((size_t)4 * m.T_cap, 0);
  std::copy(h.nodepos.begin(), h.nodepos.end(), ep.begin());
  if ((r = upload(c, (int*)m.epos, ep.data(), ep.size()))) return r;
  if ((r = upload(c, (int*)m.patchpos, h.patchpos.data(), h.patchpos.size()))) return r;
  std::vector<int> neg((size_t)4 * T, -1);
  if ((r = upload(c, (int*)m.front, neg.data(), (size_t)4 * T))) return r;
  if ((r = upload(c, m.smask, neg.data(), (size_t)T))) return r;
  HIPCHK(c, hipMemsetAsync(m.candf, 0, sizeof(int) * T, c->stream));
  HIPCHK(c, hipMemsetAsync(c->d_ctr, 0, sizeof(Counters), c->stream));
  HIPCHK(c, hipMemsetAsync(c->st.u, 0, sizeof(double4) * m.N_cap, c->stream));
  HIPCHK(c, hipMemsetAsync(c->st.v, 0, sizeof(double4) * m.N_cap, c->stream));
  HIPCHK(c, hipMemsetAsync(c->st.a, 0, sizeof(double4) * m.N_cap, c->stream));
  HIPCHK(c, hipMemsetAsync(c->st.uh, 0, sizeof(double4) * m.N_cap, c->stream));
  HIPCHK(c, hipMemsetAsync(c->w.veps, 0, RS * 6 * (size_t)m.T_cap, c->stream));
  HIPCHK(c, hipMemsetAsync(c->w.esig, 0, RS * 6 * (size_t)m.E_cap, c->stream));
  HIPCHK(c, hipMemsetAsync(c->w.einvV, 0, RS * (size_t)m.E_cap, c->stream));
  HIPCHK(c, hipMemsetAsync(c->w.contrib, 0, RS * 12 * (size_t)m.T_cap, c->stream));
  HIPCHK(c, hipMemsetAsync(m.vol, 0, sizeof(double) * m.T_cap, c->stream));
  HIPCHK(c, hipMemsetAsync(m.invm, 0, sizeof(double) * m.N_cap, c->stream));
  HIPCHK(c, launch_masses(m, c->stream));
  HIPCHK(c, launch_normals(m, c->d_ctr, c->stream));
  if (c->mixed) HIPCHK(c, Launch<float>::edge_volumes(m, c->w, -1, c->stream));
  else HIPCHK(c, Launch<double>::edge_volumes(m, c->w, -1, c->stream));
  if ((r = sync(c))) return r;
  c->split_host.assign(T, 0);
  c->need_init = true;
  return CEM_OK;
}

int cem_upload_hex_mesh(cem_ctx* c, int32_t N, const double* X, int32_t H, const int32_t* hexes,
                        const cem_material* mat) {
  if (!c) return CEM_EINVAL;
  if (c->stage != 0) return c->fail(CEM_ESTATE, "mesh already uploaded");
  if (!X || !hexes || !mat || N < 8 || H < 1) return c->fail(CEM_EINVAL, "empty mesh");
  if (N > kNodeMask / 2 || (long long)H * 12 > (1LL << 30))
    return c->fail(CEM_EINVAL, "mesh too large for 32-bit indexing");
  if (!(mat->E > 0) || !(mat->rho > 0) || !(mat->nu > -1.0 && mat->nu < 0.5) || !(mat->Gc > 0))
    return c->fail(CEM_EINVAL, "invalid material");
  for (long long i = 0; i < (long long)H * 8; ++i)
    if (hexes[i] < 0 || hexes[i] >= N) return c->fail(CEM_EMESH, "node id out of range");
  for (long long i = 0; i < (long long)N * 3; ++i)
    if (!std::isfinite(X[i])) return c->fail(CEM_EINVAL, "non-finite coordinate");
  // orientation: mirror a hex that is inverted throughout (1 <-> 3, 5 <-> 7)
  std::vector<int> ext(hexes, hexes + (size_t)8 * H);
  for (int t = 0; t < H; ++t) {
    int* nd = &ext[8 * (size_t)t];
    double lo, hi;
    hex_det_range(X, nd, &lo, &hi);
    if (hi < 0) {
      std::swap(nd[1], nd[3]);
      std::swap(nd[5], nd[7]);
      hex_det_range(X, nd, &lo, &hi);
    }
    if (!(lo > 0)) return c->fail(CEM_EMESH, "degenerate or inverted hexahedron " + std::to_string(t));
  }
  hilbert_order(N, H, 8, ext, X, c->node_new);
  c->node_old.assign(N, 0);
  for (int i = 0; i < N; ++i) c->node_old[c->node_new[i]] = i;
  {
    std::vector<int> cnt(N + 1, 0), key(H);
    for (int t = 0; t < H; ++t) {
      int mn = N;
      for (int l = 0; l < 8; ++l) mn = std::min(mn, c->node_new[ext[8 * (size_t)t + l]]);
      key[t] = mn;
      cnt[mn + 1]++;
    }
    for (int i = 0; i < N; ++i) cnt[i + 1] += cnt[i];
    c->tet_new.assign(H, 0);
    c->tet_old.assign(H, 0);
    for (int t = 0; t < H; ++t) {
      int nt = cnt[key[t]]++;
      c->tet_new[t] = nt;
      c->tet_old[nt] = t;
    }
  }
  std::vector<int> hx((size_t)8 * H);
  for (int t = 0; t < H; ++t)
    for (int l = 0; l < 8; ++l) hx[8 * (size_t)c->tet_new[t] + l] = c->node_new[ext[8 * (size_t)t + l]];
  c->X.assign((size_t)3 * N, 0.0);
  for (int i = 0; i < N; ++i)
    for (int d = 0; d < 3; ++d) c->X[3 * (size_t)c->node_new[i] + d] = X[3 * (size_t)i + d];
  HexTopo h;
  build_hex_topology(N, H, hx, h);

  HIPCHK(c, hipSetDevice(c->opt.device));
  {
    int rs = static_scratch(c, &c->scratch);  // set-up of the static staging, once per device
    if (rs) return rs;
  }
  if (!c->stream) {
    HIPCHK(c, hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
    c->own_stream = true;
  }
  c->mat = *mat;
  Mesh& m = c->m;
  // a hex cracks once, in its own slot: no copies, extra nodes or new edges
  const int S = std::min(c->opt.max_splits, H);
  m.T0 = m.T_cap = H;
  m.N0 = m.N_cap = N;
  m.E0 = m.E_cap = h.E0;
  m.S_cap = S;
  m.mode = CEM_ERODE;
  m.gsig = c->opt.gsig;
  m.lam = mat->E * mat->nu / ((1 + mat->nu) * (1 - 2 * mat->nu));
  m.mu = mat->E / (2 * (1 + mat->nu));
  m.rho = mat->rho;
  m.Gc = mat->Gc;
  m.grid_cap = kDefaultGridCap;
  m.lanes = kDefaultLanes;
  m.ssum = 0;
  m.tiled = 0;
  m.ntile[0] = m.ntile[1] = 0;
  m.split_of = nullptr;
  for (int p = 0; p < 2; ++p) m.toff[p] = m.ttoff[p] = m.ttet[p] = nullptr;
  m.ntile_fx = 0;
  m.toff_fx = m.ttoff_fx = m.ttet_fx = nullptr;
  m.fx_g1 = 0.0;
  m.fx_deg = 0;
  m.sig_slot = nullptr;
  m.gtab = nullptr;
  m.topo_multi = 0;
  m.n_inst = 0;
  m.etype = 8;
  {
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int i = 0; i < N; ++i)
      for (int d = 0; d < 3; ++d) {
        lo[d] = std::min(lo[d], c->X[3 * (size_t)i + d]);
        hi[d] = std::max(hi[d], c->X[3 * (size_t)i + d]);
      }
    m.umax = std::sqrt((hi[0] - lo[0]) * (hi[0] - lo[0]) + (hi[1] - lo[1]) * (hi[1] - lo[1]) +
                       (hi[2] - lo[2]) * (hi[2] - lo[2]));
  }
  HIPCHK(c, hipHostMalloc((void**)&c->h_ctr, sizeof(Counters), hipHostMallocDefault));
  std::memset(c->h_ctr, 0, sizeof(Counters));
  c->stage = 1;
  const size_t RS = sizeof(double);  // either precision (cem_set_precision)
  int r;
  ALLOC(c->d_ctr, 1, true);
  ALLOC(m.hnodes, (size_t)2 * H, false);
  ALLOC(m.he2e, (size_t)6 * H, false);
  ALLOC(m.epos, (size_t)2 * H, false);  // node-list positions of the eight (hex, local) entries
  ALLOC(m.X, m.N_cap, true);
  ALLOC(m.poff, (size_t)m.E0 + 1, false);
  ALLOC(m.pent, (size_t)12 * H, false);
  ALLOC(m.noff, (size_t)N + 1, false);
  ALLOC(m.nent, (size_t)8 * H, false);
  ALLOC(m.invm, m.N_cap, true);
  ALLOC(m.lslot, m.N_cap, true);
  ALLOC(m.vol, m.T_cap, true);
  // crack state: plane per hex, pending crack, candidates, fronts, records
  size_t nsplit_list = 1;  // a power of two >= S (room for the bitonic sort)
  while (nsplit_list < (size_t)std::max(S, 1)) nsplit_list <<= 1;
  ALLOC(m.tet_ext, H, false);
  ALLOC(m.hnbr, (size_t)6 * H, false);
  ALLOC(m.hfront, (size_t)6 * H, true);
  ALLOC(m.smask, H, true);
  ALLOC(m.pmask, H, true);
  ALLOC(m.ppat, H, true);
  ALLOC(m.pG, H, true);
  ALLOC(m.cand, H, true);
  ALLOC(m.candf, H, true);
  ALLOC(m.splitlist, nsplit_list, false);
  ALLOC(m.area, std::max(S, 1), false);
  ALLOC(m.rec_step, std::max(S, 1), true);
  ALLOC(m.rec_tet, std::max(S, 1), true);
  ALLOC(m.rec_mask, std::max(S, 1), true);
  ALLOC(m.rec_pat, std::max(S, 1), true);
  ALLOC(m.rec_G, std::max(S, 1), true);
  ALLOC(m.rec_area, std::max(S, 1), true);
  char* vb;
  ALLOC(vb, RS * 6 * 12 * (size_t)H, false);  // one V eps record per (hex, edge point)
  c->w.veps = vb;
  ALLOC(vb, RS * 6 * (size_t)m.E0, false);
  c->w.esig = vb;
  ALLOC(vb, RS * (size_t)m.E0, true);
  c->w.einvV = vb;
  ALLOC(vb, RS * 3 * 8 * (size_t)H, false);  // the nodal terms at node-list positions
  c->w.contrib = vb;
  ALLOC(c->w.partial, c->n_partial, false);
  ALLOC(c->d_out, 8, false);
  ALLOC(c->d_iout, 8, false);
  ALLOC(c->st.u, m.N_cap, true);
  ALLOC(c->st.v, m.N_cap, true);
  ALLOC(c->st.a, m.N_cap, true);
  ALLOC(c->st.uh, m.N_cap, true);
  ALLOC(c->d_tmp, m.N_cap, false);
  ALLOC(c->d_tmp2, m.N_cap, false);
  std::vector<int4> hn((size_t)2 * H);
  for (size_t t = 0; t < (size_t)H; ++t) {
    const int* q = &hx[8 * t];
    hn[2 * t] = make_int4(q[0], q[1], q[2], q[3]);
    hn[2 * t + 1] = make_int4(q[4], q[5], q[6], q[7]);
  }
  if ((r = upload(c, m.hnodes, hn.data(), hn.size()))) return r;
  std::vector<int2> e2((size_t)6 * H);
  for (size_t i = 0; i < e2.size(); ++i) e2[i] = make_int2(h.he2e[2 * i], h.he2e[2 * i + 1]);
  if ((r = upload(c, m.he2e, e2.data(), e2.size()))) return r;
  std::vector<double4> Xp(N);
  for (int i = 0; i < N; ++i) Xp[i] = make_double4(c->X[3 * (size_t)i], c->X[3 * (size_t)i + 1], c->X[3 * (size_t)i + 2], 0.0);
  if ((r = upload(c, m.X, Xp.data(), Xp.size()))) return r;
  if ((r = upload(c, m.poff, h.poff.data(), h.poff.size()))) return r;
  if ((r = upload(c, m.pent, h.pent.data(), h.pent.size()))) return r;
  if ((r = upload(c, m.noff, h.noff.data(), h.noff.size()))) return r;
  if ((r = upload(c, m.nent, h.nent.data(), h.nent.size()))) return r;
  if ((r = upload(c, (int*)m.epos, h.nodepos.data(), h.nodepos.size()))) return r;
  std::vector<int> lsl(N, -1);
  if ((r = upload(c, m.lslot, lsl.data(), lsl.size()))) return r;
  {
    std::vector<int> ext_id(H), nbr6, minus((size_t)6 * H, -1), zero(H, 0);
    for (int t = 0; t < H; ++t) ext_id[t] = c->tet_old[t];
    if (!hex_face_neighbours(H, hx, nbr6)) return c->fail(CEM_EMESH, "face shared by more than two hexahedra");
    if ((r = upload(c, m.tet_ext, ext_id.data(), ext_id.size()))) return r;
    if ((r = upload(c, m.hnbr, nbr6.data(), nbr6.size()))) return r;
    if ((r = upload(c, m.hfront, minus.data(), minus.size()))) return r;
    if ((r = upload(c, m.smask, minus.data(), (size_t)H))) return r;
    if ((r = upload(c, m.candf, zero.data(), zero.size()))) return r;
  }
  HIPCHK(c, hipMemsetAsync(c->d_ctr, 0, sizeof(Counters), c->stream));
  for (double4* p : {c->st.u, c->st.v, c->st.a, c->st.uh})
    HIPCHK(c, hipMemsetAsync(p, 0, sizeof(double4) * N, c->stream));
  HIPCHK(c, hipMemsetAsync(c->w.contrib, 0, RS * 3 * 8 * (size_t)H, c->stream));
  HIPCHK(c, launch_masses(m, c->stream));  // hex geometry (G_i, V), then lumped masses
  if (c->mixed) HIPCHK(c, Launch<float>::edge_volumes(m, c->w, -1, c->stream));
  else HIPCHK(c, Launch<double>::edge_volumes(m, c->w, -1, c->stream));
  if ((r = sync(c))) return r;
  c->split_host.assign(H, 0);
  c->need_init = true;
  return CEM_OK;
}

int cem_set_traction(cem_ctx* c, int32_t n_faces, const int32_t* tri, const double* t,
                     double ramp_t0) {
  if (!c) return CEM_EINVAL;
  int r = ensure_ready(c, false);
  if (r) return r;
  c->gen++;
  if (n_faces < 0 || (n_faces > 0 && (!tri || !t)) || !(ramp_t0 >= 0))
    return c->fail(CEM_EINVAL, "bad traction arguments");
  Mesh& m = c->m;
  for (long long i = 0; i < 3LL * n_faces; ++i) {
    if (tri[i] < 0 || tri[i] >= m.N0) return c->fail(CEM_EINVAL, "traction face node out of range");
    if (!std::isfinite(t[i])) return c->fail(CEM_EINVAL, "non-finite traction");
  }
  // loaded nodes -> slots; per slot the list of its faces
  std::vector<int> tri_int((size_t)3 * n_faces);
  for (long long i = 0; i < 3LL * n_faces; ++i) tri_int[i] = c->node_new[tri[i]];
  tri = tri_int.data();
  std::vector<int> slot(m.N0, -1), lnode;
  for (long long i = 0; i < 3LL * n_faces; ++i) slot[tri[i]] = 0;
  for (int i = 0; i < m.N0; ++i)
    if (slot[i] == 0) {
      slot[i] = (int)lnode.size();
      lnode.push_back(i);
    }
  int L = (int)lnode.size();
  std::vector<int> lfoff(L + 1, 0), lfent;
  for (long long i = 0; i < 3LL * n_faces; ++i) lfoff[slot[tri[i]] + 1]++;
  for (int s = 0; s < L; ++s) lfoff[s + 1] += lfoff[s];
  lfent.assign(lfoff[L], 0);
  std::vector<int> fill(lfoff.begin(), lfoff.end() - 1);
  for (int f = 0; f < n_faces; ++f)
    for (int q = 0; q < 3; ++q) lfent[fill[slot[tri[3 * f + q]]]++] = f;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  // (re)allocate the load arrays
  auto release = [&](void* p) {
    if (!p) return;
    (void)hipFree(p);
    c->allocs.erase(std::remove(c->allocs.begin(), c->allocs.end(), p), c->allocs.end());
    c->regions.erase(std::remove_if(c->regions.begin(), c->regions.end(),
                                    [&](const Region& g) { return g.ptr == p; }),
                     c->regions.end());
  };
  release(m.Fload); release(m.wacc); release(m.lnode);
  release(c->d_ftri); release(c->d_ftrac); release(c->d_lfoff); release(c->d_lfent);
  m.Fload = nullptr; m.wacc = nullptr; m.lnode = nullptr;
  ALLOC(m.Fload, L, false);
  ALLOC(m.wacc, L, true);
  ALLOC(m.lnode, L, false);
  ALLOC(c->d_ftri, n_faces, false);
  ALLOC(c->d_ftrac, n_faces, false);
  ALLOC(c->d_lfoff, L + 1, false);
  ALLOC(c->d_lfent, lfent.size(), false);
  std::vector<int4> ft(n_faces);
  std::vector<double4> fr(n_faces);
  for (int f = 0; f < n_faces; ++f) {
    ft[f] = make_int4(tri[3 * f], tri[3 * f + 1], tri[3 * f + 2], 0);
    fr[f] = make_double4(t[3 * f], t[3 * f + 1], t[3 * f + 2], 0);
  }
  if ((r = upload(c, c->d_ftri, ft.data(), ft.size()))) return r;
  if ((r = upload(c, c->d_ftrac, fr.data(), fr.size()))) return r;
  if ((r = upload(c, c->d_lfoff, lfoff.data(), lfoff.size()))) return r;
  if ((r = upload(c, c->d_lfent, lfent.data(), lfent.size()))) return r;
  if ((r = upload(c, m.lnode, lnode.data(), lnode.size()))) return r;
  std::vector<int> lsl(m.N0, -1);
  for (int s = 0; s < L; ++s) lsl[lnode[s]] = s;
  if ((r = upload(c, m.lslot, lsl.data(), lsl.size()))) return r;
  m.n_load = L;
  m.ramp_t0 = ramp_t0;
  HIPCHK(c, launch_loads(m, c->d_ftri, c->d_ftrac, c->d_lfoff, c->d_lfent, c->stream));
  if ((r = sync(c))) return r;
  c->traction_set = true;
  c->need_init = true;
  drop_graph(c);
  return CEM_OK;
}

int cem_presplit(cem_ctx* c, int32_t n, const int32_t* tet, const uint8_t* side_mask) {
  if (!c) return CEM_EINVAL;
  int r = ensure_ready(c, false);
  if (r) return r;
  c->gen++;
  if (c->step_host != 0) return c->fail(CEM_ESTATE, "pre-splits must precede the first step");
  if (n < 0 || (n > 0 && (!tet || !side_mask))) return c->fail(CEM_EINVAL, "bad presplit arguments");
  std::vector<std::pair<int, int>> lst;
  for (int i = 0; i < n; ++i) {
    int mk = side_mask[i];
    int nb = __builtin_popcount(mk & 15);
    if (tet[i] < 0 || tet[i] >= c->m.T0) return c->fail(CEM_EINVAL, "presplit element out of range");
    if (c->m.etype == 8) {  // hexes: a crack plane index
      if (mk >= 23) return c->fail(CEM_EINVAL, "crack plane index out of range");
    } else if ((mk & ~15) || nb == 0 || nb == 4) {
      return c->fail(CEM_EINVAL, "presplit mask is not a partition");
    }
    lst.push_back({tet[i], mk});
  }
  std::sort(lst.begin(), lst.end());
  std::vector<int> tt, text;
  std::vector<uint8_t> mm;
  for (size_t i = 0; i < lst.size(); ++i) {
    if (i > 0 && lst[i].first == lst[i - 1].first) continue;
    if (c->split_host[lst[i].first]) continue;
    text.push_back(lst[i].first);
    tt.push_back(c->tet_new[lst[i].first]);  // ascending caller ids, internal slots
    mm.push_back((uint8_t)lst[i].second);
  }
  if ((long long)c->n_split_host + (long long)tt.size() > c->m.S_cap)
    return c->fail(CEM_ECAPACITY, "presplit exceeds the split capacity");
  if (tt.empty()) return CEM_OK;
  int* d_t = nullptr;
  uint8_t* d_m = nullptr;
  HIPCHK(c, hipMalloc(&d_t, sizeof(int) * tt.size()));
  HIPCHK(c, hipMalloc(&d_m, mm.size()));
  HIPCHK(c, hipMemcpyAsync(d_t, tt.data(), sizeof(int) * tt.size(), hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(d_m, mm.data(), mm.size(), hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, launch_set_presplit(c->m, c->d_ctr, d_t, d_m, (int)tt.size(), c->stream));
  if (c->mixed)
    HIPCHK(c, launch_topology_t<float>(c->m, c->st, c->w, c->d_ctr, 0, 0, c->d_snodes, c->d_sedges, c->stream));
  else
    HIPCHK(c, launch_topology_t<double>(c->m, c->st, c->w, c->d_ctr, 0, 0, c->d_snodes, c->d_sedges, c->stream));
  r = sync(c);
  (void)hipFree(d_t);
  (void)hipFree(d_m);
  if (r) return r;
  for (int t : text) c->split_host[t] = 1;
  r = check_device_error(c);
  if (r) return r;
  c->need_init = true;
  return CEM_OK;
}

int cem_critical_dt(cem_ctx* c, double* dt_crit) {
  if (!c || !dt_crit) return CEM_EINVAL;
  int r = ensure_ready(c, false);
  if (r) return r;
  unsigned long long zero = 0;
  HIPCHK(c, hipMemcpyAsync(&c->d_ctr->lam_key, &zero, sizeof(zero), hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, launch_dtcrit(c->m, c->d_ctr, c->stream));
  if ((r = read_counters(c))) return r;
  *dt_crit = c->h_ctr->dt_crit;
  return CEM_OK;
}

int cem_set_dt(cem_ctx* c, double dt) {
  if (!c) return CEM_EINVAL;
  int r = ensure_ready(c, false);
  if (r) return r;
  c->gen++;
  if (!(dt > 0) || !std::isfinite(dt)) return c->fail(CEM_EINVAL, "dt must be positive");
  c->m.dt = dt;
  c->dt_set = true;
  c->need_init = true;
  drop_graph(c);
  return CEM_OK;
}

int cem_set_precision(cem_ctx* c, int32_t precision) {
  if (!c) return CEM_EINVAL;
  int r = ensure_ready(c, false);
  if (r) return r;
  if (precision != CEM_FP64 && precision != CEM_MIXED) return c->fail(CEM_EINVAL, "unknown precision");
  const int mixed = precision == CEM_MIXED;
  if (mixed == c->mixed) return CEM_OK;
  c->mixed = mixed;
  c->opt.precision = precision;
  c->gen++;
  drop_graph(c);
  // 1 / patch volume in the new arithmetic, from the current element volumes,
  // for every edge now (split copies add ten each)
  nodes_now_host(c);
  const int En = edges_now_host(c);
  if (c->mixed) HIPCHK(c, Launch<float>::edge_volumes(c->m, c->w, En, c->stream));
  else HIPCHK(c, Launch<double>::edge_volumes(c->m, c->w, En, c->stream));
  // the state (u, v, a and the predictor) carries over as it is: a
  // recomputed here would see a topology changed by the last step's splits
  return sync(c);
}

int cem_set_graph_steps(cem_ctx* c, int32_t k) {
  if (!c) return CEM_EINVAL;
  if (k < 0) return c->fail(CEM_EINVAL, "graph_steps must be >= 0");
  c->opt.graph_steps = k;
  drop_graph(c);
  return CEM_OK;
}

int cem_last_run(cem_ctx* c, int64_t* out) {
  if (!c || !out) return CEM_EINVAL;
  for (int q = 0; q < 4; ++q) out[q] = c->last_run[q];
  return CEM_OK;
}

int cem_bind_state(cem_ctx* c, double* d_u, double* d_v, int64_t cap) {
  if (!c) return CEM_EINVAL;
  int r = ensure_ready(c, false);
  if (r) return r;
  c->gen++;
  if (!d_u || !d_v || cap < c->m.N_cap) return c->fail(CEM_EINVAL, "bound buffers too small");
  HIPCHK(c, hipMemcpyAsync(d_u, c->st.u, sizeof(double4) * c->m.N_cap, hipMemcpyDeviceToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(d_v, c->st.v, sizeof(double4) * c->m.N_cap, hipMemcpyDeviceToDevice, c->stream));
  if ((r = sync(c))) return r;
  for (auto& g : c->regions) {
    if (g.ptr == c->st.u) g.ptr = d_u;
    else if (g.ptr == c->st.v) g.ptr = d_v;
  }
  c->st.u = (double4*)d_u;
  c->st.v = (double4*)d_v;
  c->bound = true;
  drop_graph(c);
  return CEM_OK;
}

int cem_node_rows(cem_ctx* c, int32_t n, int32_t* row) {
  if (!c || (n > 0 && !row)) return CEM_EINVAL;
  int r = ensure_ready(c, false);
  if (r) return r;
  const int now = nodes_now_host(c);
  if (n < 0 || n > now) return c->fail(CEM_EINVAL, "more rows asked than nodes now");
  for (int i = 0; i < n; ++i) row[i] = node_int(c, i);
  return CEM_OK;
}

int cem_set_state(cem_ctx* c, const double* u, const double* v) {
  if (!c) return CEM_EINVAL;
  int r = ensure_ready(c, false);
  if (r) return r;
  c->gen++;
  int n = nodes_now_host(c);
  std::vector<double4> tmp;
  if (u) {
    pad3(c, u, tmp, n);
    if ((r = upload(c, c->st.u, tmp.data(), n))) return r;
  }
  if (v) {
    pad3(c, v, tmp, n);
    if ((r = upload(c, c->st.v, tmp.data(), n))) return r;
  }
  if ((r = sync(c))) return r;
  c->need_init = true;
  return CEM_OK;
}

int cem_get_state(cem_ctx* c, double* u, double* v, double* a, int32_t* n_now) {
  if (!c) return CEM_EINVAL;
  int r = ensure_ready(c, false);
  if (r) return r;
  if (c->need_init && c->dt_set) {
    if ((r = initialize(c))) return r;
  }
  int n = nodes_now_host(c);
  if (n_now) *n_now = n;
  std::vector<double4> tmp(n);
  double4* src[3] = {c->st.u, c->st.v, c->st.a};
  double* dst[3] = {u, v, a};
  for (int q = 0; q < 3; ++q) {
    if (!dst[q]) continue;
    HIPCHK(c, hipMemcpyAsync(tmp.data(), src[q], sizeof(double4) * n, hipMemcpyDeviceToHost, c->stream));
    if ((r = sync(c))) return r;
    unpad3(c, tmp, dst[q], n);
  }
  return CEM_OK;
}

int cem_internal_force(cem_ctx* c, const double* u, double* f) {
  if (!c || !u || !f) return CEM_EINVAL;
  int r = ensure_ready(c, false);
  if (r) return r;
  int n = nodes_now_host(c);
  std::vector<double4> tmp;
  pad3(c, u, tmp, n);
  if ((r = upload(c, c->d_tmp, tmp.data(), n))) return r;
  if ((r = strain_stress(c, c->d_tmp))) return r;
  if ((r = node_pass(c, NODE_FORCE, c->d_tmp2))) return r;
  tmp.resize(n);
  HIPCHK(c, hipMemcpyAsync(tmp.data(), c->d_tmp2, sizeof(double4) * n, hipMemcpyDeviceToHost, c->stream));
  if ((r = sync(c))) return r;
  unpad3(c, tmp, f, n);
  return CEM_OK;
}

int cem_step(cem_ctx* c, int32_t n_steps) {
  if (!c) return CEM_EINVAL;
  int r = ensure_ready(c, true);
  if (r) return r;
  if (n_steps < 0) return c->fail(CEM_EINVAL, "negative step count");
  c->gen++;
  return run_steps(c, n_steps);
}

int cem_replay_splits(cem_ctx* c, int32_t n, const cem_split_event* ev) {
  if (!c) return CEM_EINVAL;
  int r = ensure_ready(c, false);
  if (r) return r;
  if (c->m.etype == 8) return c->fail(CEM_ESTATE, "a forced schedule is for tetrahedral meshes");
  c->gen++;
  if (n < 0 || (n > 0 && !ev)) return c->fail(CEM_EINVAL, "bad schedule");
  std::vector<std::array<int, 3>> s;
  for (int i = 0; i < n; ++i) {
    int nb = __builtin_popcount(ev[i].side_mask & 15);
    if (ev[i].tet < 0 || ev[i].tet >= c->m.T0 || (ev[i].side_mask & ~15) || nb == 0 || nb == 4)
      return c->fail(CEM_EINVAL, "bad schedule entry");
    s.push_back({ev[i].step, ev[i].tet, ev[i].side_mask});
  }
  std::stable_sort(s.begin(), s.end(), [](const std::array<int, 3>& x, const std::array<int, 3>& y) {
    return x[0] != y[0] ? x[0] < y[0] : x[1] < y[1];
  });
  for (auto& e3 : s) e3[1] = c->tet_new[e3[1]];
  if (c->m.sched) {
    (void)hipFree(c->m.sched);
    c->allocs.erase(std::remove(c->allocs.begin(), c->allocs.end(), (void*)c->m.sched), c->allocs.end());
    c->m.sched = nullptr;
  }
  ALLOC(c->m.sched, (size_t)3 * std::max(n, 1), false);
  if ((r = upload(c, c->m.sched, (const int*)s.data(), (size_t)3 * n))) return r;
  if ((r = read_counters(c))) return r;
  c->h_ctr->n_sched = n;
  c->h_ctr->replay_cursor = 0;
  HIPCHK(c, hipMemcpyAsync(&c->d_ctr->replay_cursor, &c->h_ctr->replay_cursor, 2 * sizeof(int) + sizeof(int),
                           hipMemcpyHostToDevice, c->stream));
  if ((r = sync(c))) return r;
  drop_graph(c);
  return CEM_OK;
}

// Energies of the whole run (inst < 0) or of one instance of a batch.
int read_energy(cem_ctx* c, int inst, cem_energy* e) {
  int r;
  if (c->need_init && c->dt_set && (r = initialize(c))) return r;
  Mesh& m = c->m;
  int np = c->n_partial;
  HIPCHK(c, launch_kinetic(m, c->st, c->d_ctr, c->w.partial, np, inst, c->stream));
  HIPCHK(c, launch_sum(c->w.partial, np, c->d_out, c->stream));
  if (c->mixed) {
    HIPCHK(c, Launch<float>::strain(m, c->st.u, c->w, c->d_ctr, c->stream));
    HIPCHK(c, launch_strain_energy<float>(m, c->w, c->d_ctr, c->w.partial, np, inst, c->stream));
  } else {
    HIPCHK(c, Launch<double>::strain(m, c->st.u, c->w, c->d_ctr, c->stream));
    HIPCHK(c, launch_strain_energy<double>(m, c->w, c->d_ctr, c->w.partial, np, inst, c->stream));
  }
  HIPCHK(c, launch_sum(c->w.partial, np, c->d_out + 1, c->stream));
  if (m.n_load > 0) HIPCHK(c, launch_work_sum(m, c->d_out + 2, inst, c->stream));
  else HIPCHK(c, hipMemsetAsync(c->d_out + 2, 0, sizeof(double), c->stream));
  HIPCHK(c, launch_dissipated(m, c->d_ctr, c->d_out + 3, inst, c->stream));
  HIPCHK(c, hipMemsetAsync(c->d_iout, 0, sizeof(int), c->stream));
  HIPCHK(c, launch_count_fronts(m, c->d_ctr, c->d_iout, inst, c->stream));
  double out[5];
  int nf = 0;
  HIPCHK(c, hipMemcpyAsync(out, c->d_out, sizeof(out), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipMemcpyAsync(&nf, c->d_iout, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  unsigned long long gk[2] = {0, 0};
  if (inst >= 0)
    HIPCHK(c, hipMemcpyAsync(gk, m.gmax_inst + m.n_inst + inst, sizeof(gk[0]), hipMemcpyDeviceToHost,
                             c->stream));
  double dti = m.dt;
  if (inst >= 0)
    HIPCHK(c, hipMemcpyAsync(&dti, m.dti + inst, sizeof(double), hipMemcpyDeviceToHost, c->stream));
  if ((r = read_counters(c))) return r;
  const Counters& k = *c->h_ctr;
  int ns = inst >= 0 ? (int)out[4] : k.n_split;
  int n0 = inst >= 0 ? c->inst_nodes[inst] : m.N0, t0 = inst >= 0 ? c->inst_tets[inst] : m.T0;
  unsigned long long g = inst >= 0 ? gk[0] : k.gmax_last;
  e->step = k.step;
  e->t = (double)k.step * dti;
  e->KE = out[0];
  e->SE = out[1];
  e->Wext = out[2];
  e->Ud = inst >= 0 ? out[3] : k.Ud;
  e->Gmax = g ? key_to_double_host(g) : 0.0;
  e->n_split = ns;
  e->n_front = nf;
  e->n_nodes = n0 + (m.mode == MODE_PHANTOM ? 4 * ns : 0);
  e->n_elems = t0 + (m.mode == MODE_PHANTOM ? ns : 0);
  return CEM_OK;
}

int cem_read_energy(cem_ctx* c, cem_energy* e) {
  if (!c || !e) return CEM_EINVAL;
  int r = ensure_ready(c, false);
  if (r) return r;
  return read_energy(c, -1, e);
}

int cem_read_energy_instances(cem_ctx* c, int32_t n, cem_energy* out) {
  if (!c || !out) return CEM_EINVAL;
  int r = ensure_ready(c, false);
  if (r) return r;
  if (c->m.n_inst == 0 || n != c->m.n_inst) return c->fail(CEM_EINVAL, "no batch of that size");
  for (int i = 0; i < n; ++i)
    if ((r = read_energy(c, i, out + i))) return r;
  return CEM_OK;
}

int cem_set_instances(cem_ctx* c, int32_t n, const int32_t* node_off, const int32_t* tet_off) {
  if (!c) return CEM_EINVAL;
  int r = ensure_ready(c, false);
  if (r) return r;
  if (c->m.etype == 8) return c->fail(CEM_ESTATE, "batches are built from tetrahedral meshes");
  c->gen++;
  Mesh& m = c->m;
  if (c->m.n_inst) return c->fail(CEM_ESTATE, "instances already declared");
  if (c->m.n_grp) return c->fail(CEM_ESTATE, "prescribed velocities are not supported in batches");
  if (c->step_host != 0 || c->n_split_host != 0)
    return c->fail(CEM_ESTATE, "instances must be declared before pre-splits and steps");
  if (n < 1 || !node_off || !tet_off) return c->fail(CEM_EINVAL, "bad instance arguments");
  if (node_off[0] != 0 || tet_off[0] != 0 || node_off[n] != m.N0 || tet_off[n] != m.T0)
    return c->fail(CEM_EINVAL, "instance ranges must cover the mesh");
  for (int i = 0; i < n; ++i)
    if (node_off[i + 1] <= node_off[i] || tet_off[i + 1] <= tet_off[i])
      return c->fail(CEM_EINVAL, "empty or decreasing instance range");
  std::vector<int> ninst(m.N0), tinst(m.T0);
  for (int i = 0; i < n; ++i) {
    for (int q = node_off[i]; q < node_off[i + 1]; ++q) ninst[c->node_new[q]] = i;
    for (int t = tet_off[i]; t < tet_off[i + 1]; ++t) tinst[c->tet_new[t]] = i;
  }
  for (int t = 0; t < m.T0; ++t)
    for (int l = 0; l < 4; ++l)
      if (ninst[c->tets[4 * (size_t)t + l]] != tinst[t])
        return c->fail(CEM_EINVAL, "a tet joins nodes of two instances");
  ALLOC(m.inst, m.N_cap, true);
  ALLOC(m.tinst, m.T_cap, true);
  ALLOC(m.einst, m.E_cap, true);
  ALLOC(m.dti, n, true);
  ALLOC(m.dtc_inst, n, false);
  ALLOC(m.gmax_inst, 2 * n, true);
  ALLOC(m.lam_inst, n, false);
  if ((r = upload(c, m.inst, ninst.data(), ninst.size()))) return r;
  if ((r = upload(c, m.tinst, tinst.data(), tinst.size()))) return r;
  std::vector<double> dts(n, m.dt);
  if ((r = upload(c, m.dti, dts.data(), dts.size()))) return r;
  HIPCHK(c, hipMemsetAsync(m.gmax_inst, 0, sizeof(unsigned long long) * 2 * n, c->stream));
  m.n_inst = n;
  HIPCHK(c, launch_edge_instances(m, c->stream));
  if ((r = sync(c))) return r;
  c->inst_nodes.assign(n, 0);
  c->inst_tets.assign(n, 0);
  for (int i = 0; i < n; ++i) {
    c->inst_nodes[i] = node_off[i + 1] - node_off[i];
    c->inst_tets[i] = tet_off[i + 1] - tet_off[i];
  }
  drop_graph(c);
  return CEM_OK;
}

int cem_set_dt_instances(cem_ctx* c, const double* dt) {
  if (!c || !dt) return CEM_EINVAL;
  int r = ensure_ready(c, false);
  if (r) return r;
  c->gen++;
  if (!c->m.n_inst) return c->fail(CEM_ESTATE, "no instances declared");
  for (int i = 0; i < c->m.n_inst; ++i)
    if (!(dt[i] > 0) || !std::isfinite(dt[i])) return c->fail(CEM_EINVAL, "dt must be positive");
  if ((r = upload(c, c->m.dti, dt, (size_t)c->m.n_inst))) return r;
  if ((r = sync(c))) return r;
  c->m.dt = dt[0];
  c->dt_set = true;
  c->need_init = true;
  drop_graph(c);
  return CEM_OK;
}

int cem_critical_dt_instances(cem_ctx* c, double* out) {
  if (!c || !out) return CEM_EINVAL;
  int r = ensure_ready(c, false);
  if (r) return r;
  if (!c->m.n_inst) return c->fail(CEM_ESTATE, "no instances declared");
  HIPCHK(c, hipMemsetAsync(c->m.lam_inst, 0, sizeof(unsigned long long) * c->m.n_inst, c->stream));
  unsigned long long zero = 0;
  HIPCHK(c, hipMemcpyAsync(&c->d_ctr->lam_key, &zero, sizeof(zero), hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, launch_dtcrit(c->m, c->d_ctr, c->stream));
  HIPCHK(c, hipMemcpyAsync(out, c->m.dtc_inst, sizeof(double) * c->m.n_inst, hipMemcpyDeviceToHost,
                           c->stream));
  return sync(c);
}

int cem_set_launch(cem_ctx* c, int32_t grid_cap, int32_t lanes, int32_t layout) {
  if (!c) return CEM_EINVAL;
  int r = ensure_ready(c, false);
  if (r) return r;
  c->gen++;
  if (grid_cap < 8 || grid_cap % 8 || (lanes != 4 && lanes != 8 && lanes != 16))
    return c->fail(CEM_EINVAL, "grid_cap must be a positive multiple of 8, lanes 4, 8 or 16");
  if (layout < CEM_LAYOUT_TERMS || layout > CEM_LAYOUT_TILES_FX)
    return c->fail(CEM_EINVAL, "layout must be CEM_LAYOUT_TERMS, CEM_LAYOUT_STRESS_SUMS, "
                               "CEM_LAYOUT_TILES or CEM_LAYOUT_TILES_FX");
  if (layout == CEM_LAYOUT_TILES && (c->m.etype == 8 || c->m.ntile[0] == 0 || c->m.ntile[1] == 0))
    return c->fail(CEM_EINVAL, "no node tiles for this mesh");
  if (layout == CEM_LAYOUT_TILES_FX && (c->m.etype == 8 || c->m.ntile_fx == 0))
    return c->fail(CEM_EINVAL, "no node tiles for this mesh");
  c->m.grid_cap = grid_cap;
  c->m.lanes = lanes;
  c->m.ssum = c->m.etype == 8 ? 0 : layout == CEM_LAYOUT_STRESS_SUMS;
  c->m.tiled = layout == CEM_LAYOUT_TILES ? 1 : layout == CEM_LAYOUT_TILES_FX ? 2 : 0;
  drop_graph(c);
  return CEM_OK;
}

// Launch-shape autotuner: times trial_steps steps of the live simulation for
// each candidate (force layout x persistent grid size x lanes per node),
// restoring the state after every trial, and keeps the fastest.  Lanes and
// layout change the order of the node sums, hence the rounding of the results.
int cem_autotune(cem_ctx* c, int32_t trial_steps, int32_t* best_grid, int32_t* best_lanes,
                 int32_t* best_layout, double* best_ms) {
  if (!c) return CEM_EINVAL;
  int r = ensure_ready(c, true);
  if (r) return r;
  if (trial_steps < 1) return c->fail(CEM_EINVAL, "trial_steps must be positive");
  int64_t used = 0;
  if ((r = cem_save_state(c, nullptr, 0, &used))) return r;
  std::vector<char> buf(used);
  if ((r = cem_save_state(c, buf.data(), used, &used))) return r;
  const int grids[4] = {1024, 2048, 4096, 8192};
  const int lanes[3] = {4, 8, 16};
  // hexes have one layout; tets the term and stress-sum layouts, the tiled
  // pass when the mesh has tiles and the fixed-point tiled pass
  const bool have_tiles = c->m.ntile[0] > 0 && c->m.ntile[1] > 0;
  int lays[4], nlay = 0;
  lays[nlay++] = CEM_LAYOUT_TERMS;
  if (c->m.etype != 8) {
    lays[nlay++] = CEM_LAYOUT_STRESS_SUMS;
    if (have_tiles) lays[nlay++] = CEM_LAYOUT_TILES;
    if (c->m.ntile_fx > 0) lays[nlay++] = CEM_LAYOUT_TILES_FX;
  }
  int g0 = c->m.grid_cap, l0 = c->m.lanes;
  int s0 = c->m.ssum ? CEM_LAYOUT_STRESS_SUMS
                     : c->m.tiled == 1 ? CEM_LAYOUT_TILES : c->m.tiled == 2 ? CEM_LAYOUT_TILES_FX : CEM_LAYOUT_TERMS;
  double best = 1e300;
  int bg = g0, bl = l0, bs = s0;
  int saved_prof = c->profiling;
  c->profiling = 0;
  // one warm-up trial, then every candidate
  if ((r = cem_step(c, trial_steps)) == CEM_OK) r = cem_load_state(c, buf.data(), used);
  for (int k = 0; k < nlay && r == CEM_OK; ++k)
    for (int gi = 0; gi < 4 && r == CEM_OK; ++gi)
      for (int li = 0; li < 3 && r == CEM_OK; ++li) {
        const int si = lays[k];
        // the fixed-point tiles have one lane per node: a single lane count
        if (si == CEM_LAYOUT_TILES_FX && li > 0) continue;
        c->m.grid_cap = grids[gi];
        c->m.lanes = lanes[li];
        c->m.ssum = si == CEM_LAYOUT_STRESS_SUMS;
        c->m.tiled = si == CEM_LAYOUT_TILES ? 1 : si == CEM_LAYOUT_TILES_FX ? 2 : 0;
        drop_graph(c);
        if ((r = cem_step(c, trial_steps))) break;
        double ms = c->times[0] / trial_steps;
        if (ms < best) {
          best = ms;
          bg = grids[gi];
          bl = lanes[li];
          bs = si;
        }
        r = cem_load_state(c, buf.data(), used);
      }
  c->profiling = saved_prof;
  const int sf = r ? s0 : bs;
  c->m.grid_cap = r ? g0 : bg;
  c->m.lanes = r ? l0 : bl;
  c->m.ssum = sf == CEM_LAYOUT_STRESS_SUMS;
  c->m.tiled = sf == CEM_LAYOUT_TILES ? 1 : sf == CEM_LAYOUT_TILES_FX ? 2 : 0;
  drop_graph(c);
  if (r) return r;
  if (best_grid) *best_grid = bg;
  if (best_lanes) *best_lanes = bl;
  if (best_layout) *best_layout = bs;
  if (best_ms) *best_ms = best;
  return CEM_OK;
}

int cem_read_splits(cem_ctx* c, int32_t cap, cem_split_event* out, int32_t* n) {
  if (!c || !n) return CEM_EINVAL;
  int r = ensure_ready(c, false);
  if (r) return r;
  if ((r = read_counters(c))) return r;
  int ns = c->h_ctr->n_split;
  *n = ns;
  int k = std::min(ns, std::max(cap, 0));
  if (k == 0 || !out) return CEM_OK;
  std::vector<int> st(k), tt(k), mk(k), pt(k);
  std::vector<double> G(k);
  HIPCHK(c, hipMemcpyAsync(st.data(), c->m.rec_step, sizeof(int) * k, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipMemcpyAsync(tt.data(), c->m.rec_tet, sizeof(int) * k, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipMemcpyAsync(mk.data(), c->m.rec_mask, sizeof(int) * k, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipMemcpyAsync(pt.data(), c->m.rec_pat, sizeof(int) * k, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipMemcpyAsync(G.data(), c->m.rec_G, sizeof(double) * k, hipMemcpyDeviceToHost, c->stream));
  if ((r = sync(c))) return r;
  for (int i = 0; i < k; ++i) out[i] = cem_split_event{st[i], c->tet_old[tt[i]], mk[i], pt[i], G[i]};
  return CEM_OK;
}

// ---- allocation-free read of the crack-front release rates (staging above)

int cem_read_front_G_static(cem_ctx* c, int32_t cap, cem_front_g* out, int32_t* n) {
  if (!c || !n || cap < 0 || (cap > 0 && !out)) return CEM_EINVAL;
  int r = ensure_ready(c, false);
  if (r) return r;
  if (c->m.etype == 8) return c->fail(CEM_ESTATE, "the static readback covers tetrahedral meshes");
  if (!c->scratch) return c->fail(CEM_ESTATE, "static staging not set up");
  if (c->need_init && c->dt_set && (r = initialize(c))) return r;
  if ((r = read_counters(c))) return r;
  const long long slots = 4LL * std::max(c->h_ctr->n_cand, 1);
  if (slots > kStaticFronts)
    return c->fail(CEM_ECAPACITY, "crack-front candidates need " + std::to_string(slots) +
                                      " front slots; the static staging holds 65536");
  unsigned char* base = c->scratch;
  cem_front_g* d_rec = (cem_front_g*)base;
  int* d_tfl = (int*)(base + kStaticRecBytes);
  double* d_g = (double*)(base + kStaticRecBytes + kStaticTflBytes);
  int* d_n = (int*)(base + kStaticRecBytes + kStaticTflBytes + kStaticGBytes);
  if ((r = strain_stress(c, c->st.u))) return r;
  hipLaunchKernelGGL(k_zero_count, dim3(1), dim3(64), 0, c->stream, d_n);
  HIPCHK(c, hipGetLastError());
  hipError_t e = c->mixed ? Launch<float>::front_eval(c->m, c->st, c->w, c->d_ctr, d_tfl, d_g, d_n, c->stream)
                          : Launch<double>::front_eval(c->m, c->st, c->w, c->d_ctr, d_tfl, d_g, d_n, c->stream);
  HIPCHK(c, e);
  hipLaunchKernelGGL(k_pack_fronts, dim3((unsigned)((slots + 255) / 256)), dim3(256), 0, c->stream,
                     d_tfl, d_g, d_n, d_rec);
  HIPCHK(c, hipGetLastError());
  int nf = 0;
  HIPCHK(c, hipMemcpyAsync(&nf, d_n, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  if ((r = sync(c))) return r;
  *n = nf;
  if (cap == 0) return CEM_OK;
  if (cap < nf)
    return c->fail(CEM_EINVAL, "output holds " + std::to_string(cap) + " records for " +
                                   std::to_string(nf) + " crack-front faces");
  if (nf > 0) HIPCHK(c, hipMemcpyAsync(out, d_rec, sizeof(cem_front_g) * nf, hipMemcpyDeviceToHost, c->stream));
  if ((r = sync(c))) return r;
  for (int i = 0; i < nf; ++i) {
    out[i].tet = c->tet_old[out[i].tet];
    out[i].lone = c->node_old[out[i].lone];
  }
  std::sort(out, out + nf, [](const cem_front_g& x, const cem_front_g& y) {
    return x.tet != y.tet ? x.tet < y.tet : x.face < y.face;
  });
  return CEM_OK;
}

int cem_read_front_G(cem_ctx* c, int32_t cap, cem_front_g* out, int32_t* n) {
  if (!c || !n) return CEM_EINVAL;
  int r = ensure_ready(c, false);
  if (r) return r;
  const bool hex = c->m.etype == 8;  // hexes: one row per candidate, up to 18 per hex
  if (c->need_init && c->dt_set && (r = initialize(c))) return r;
  if ((r = read_counters(c))) return r;
  int nc = c->h_ctr->n_cand;
  size_t capf = (size_t)(hex ? 18 : 4) * std::max(nc, 1);
  int* d_tfl = nullptr;
  double* d_g = nullptr;
  HIPCHK(c, hipMalloc(&d_tfl, sizeof(int) * 3 * capf));
  HIPCHK(c, hipMalloc(&d_g, sizeof(double) * 2 * capf));
  if ((r = strain_stress(c, c->st.u))) return r;
  HIPCHK(c, hipMemsetAsync(c->d_iout, 0, sizeof(int), c->stream));
  hipError_t e = c->mixed ? Launch<float>::front_eval(c->m, c->st, c->w, c->d_ctr, d_tfl, d_g, c->d_iout, c->stream)
                          : Launch<double>::front_eval(c->m, c->st, c->w, c->d_ctr, d_tfl, d_g, c->d_iout, c->stream);
  HIPCHK(c, e);
  int nf = 0;
  HIPCHK(c, hipMemcpyAsync(&nf, c->d_iout, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  if ((r = sync(c))) return r;
  std::vector<int> tfl((size_t)3 * nf);
  std::vector<double> g((size_t)2 * nf);
  if (nf > 0) {
    HIPCHK(c, hipMemcpyAsync(tfl.data(), d_tfl, sizeof(int) * 3 * nf, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(g.data(), d_g, sizeof(double) * 2 * nf, hipMemcpyDeviceToHost, c->stream));
  }
  r = sync(c);
  (void)hipFree(d_tfl);
  (void)hipFree(d_g);
  if (r) return r;
  for (int i = 0; i < nf; ++i) {
    tfl[3 * i] = c->tet_old[tfl[3 * i]];
    if (!hex) tfl[3 * i + 2] = c->node_old[tfl[3 * i + 2]];
  }
  std::vector<int> ord(nf);
  for (int i = 0; i < nf; ++i) ord[i] = i;
  // (element, face) order; a hex face's candidates in plane order, which is
  // their tie order (III, IV toward -1, IV toward +1; V, VI)
  std::sort(ord.begin(), ord.end(), [&](int x, int y) {
    if (tfl[3 * x] != tfl[3 * y]) return tfl[3 * x] < tfl[3 * y];
    if (tfl[3 * x + 1] != tfl[3 * y + 1]) return tfl[3 * x + 1] < tfl[3 * y + 1];
    return tfl[3 * x + 2] < tfl[3 * y + 2];
  });
  *n = nf;
  for (int i = 0; i < nf && i < cap && out; ++i) {
    int o = ord[i];
    out[i] = cem_front_g{tfl[3 * o], tfl[3 * o + 1], tfl[3 * o + 2], 0, g[2 * o], g[2 * o + 1]};
  }
  return CEM_OK;
}

// Checkpoint layout: magic, version, T0, N0, E0, S_cap, mixed, mode,
// need_init, step_host, then every checkpointed device region in allocation
// order, then the split mirror.
int cem_save_state(cem_ctx* c, void* buf, int64_t cap, int64_t* used) {
  if (!c || !used) return CEM_EINVAL;
  int r = ensure_ready(c, false);
  if (r) return r;
  const int hdr = 16;
  int64_t total = hdr * 8;
  for (auto& g : c->regions) total += (int64_t)g.bytes;
  total += c->m.T0;
  *used = total;
  if (!buf) return CEM_OK;
  if (cap < total) return c->fail(CEM_EINVAL, "checkpoint buffer too small");
  int64_t h[hdr] = {0x43454d31, 2, c->m.T0, c->m.N0, c->m.E0, c->m.S_cap, c->mixed, c->m.mode,
                    c->need_init ? 1 : 0, c->step_host, c->n_split_host, c->dt_set ? 1 : 0, 0,
                    c->kap_on ? 1 : 0, (int64_t)c->regions.size(), 0};
  for (auto& g : c->regions) h[15] += (int64_t)g.bytes;
  double dtv = c->m.dt;
  std::memcpy(&h[12], &dtv, 8);
  char* p = (char*)buf;
  std::memcpy(p, h, sizeof(h));
  p += sizeof(h);
  for (auto& g : c->regions) {
    HIPCHK(c, hipMemcpyAsync(p, g.ptr, g.bytes, hipMemcpyDeviceToHost, c->stream));
    p += g.bytes;
  }
  if ((r = sync(c))) return r;
  std::memcpy(p, c->split_host.data(), c->m.T0);
  return CEM_OK;
}

int cem_load_state(cem_ctx* c, const void* buf, int64_t size) {
  if (!c || !buf) return CEM_EINVAL;
  int r = ensure_ready(c, false);
  if (r) return r;
  c->gen++;
  const int hdr = 16;
  int64_t h[hdr];
  if (size < (int64_t)sizeof(h)) return c->fail(CEM_EINVAL, "checkpoint too short");
  std::memcpy(h, buf, sizeof(h));
  if (h[0] != 0x43454d31 || h[1] != 2 || h[2] != c->m.T0 || h[3] != c->m.N0 || h[4] != c->m.E0 ||
      h[5] != c->m.S_cap || h[6] != c->mixed || h[7] != c->m.mode ||
      h[14] != (int64_t)c->regions.size())
    return c->fail(CEM_EINVAL, "checkpoint does not match this context");
  {
    int64_t rb = 0;
    for (auto& g : c->regions) rb += (int64_t)g.bytes;
    if (rb != h[15]) return c->fail(CEM_EINVAL, "checkpoint does not match this context");
  }
  int64_t total = sizeof(h);
  for (auto& g : c->regions) total += (int64_t)g.bytes;
  total += c->m.T0;
  if (size < total) return c->fail(CEM_EINVAL, "checkpoint too short");
  const char* p = (const char*)buf + sizeof(h);
  for (auto& g : c->regions) {
    HIPCHK(c, hipMemcpyAsync(g.ptr, p, g.bytes, hipMemcpyHostToDevice, c->stream));
    p += g.bytes;
  }
  // the corner-normal rows of the restored split copies
  HIPCHK(c, launch_normals(c->m, c->d_ctr, c->stream));
  if ((r = sync(c))) return r;
  std::memcpy(c->split_host.data(), p, c->m.T0);
  c->need_init = h[8] != 0;
  c->step_host = h[9];
  c->n_split_host = (int)h[10];
  c->dt_set = h[11] != 0;
  std::memcpy(&c->m.dt, &h[12], 8);
  c->kap_on = h[13] != 0 && c->kap_buf;
  c->m.kap = c->kap_on ? c->kap_buf : nullptr;
  drop_graph(c);
  return read_counters(c);
}

int cem_counts(cem_ctx* c, int32_t* out) {
  if (!c || !out) return CEM_EINVAL;
  int r = ensure_ready(c, false);
  if (r) return r;
  if ((r = read_counters(c))) return r;
  const Counters& k = *c->h_ctr;
  const Mesh& m = c->m;
  bool ph = m.mode == MODE_PHANTOM;
  HIPCHK(c, hipMemsetAsync(c->d_iout, 0, sizeof(int), c->stream));
  HIPCHK(c, launch_count_fronts(m, c->d_ctr, c->d_iout, -1, c->stream));
  int nf = 0;
  HIPCHK(c, hipMemcpyAsync(&nf, c->d_iout, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  if ((r = sync(c))) return r;
  out[0] = m.N0 + (ph ? 4 * k.n_split : 0);
  out[1] = m.T0 + (ph ? k.n_split : 0);
  out[2] = m.E0 + (ph ? 10 * k.n_split : 0);
  out[3] = k.n_split;
  out[4] = nf;
  out[5] = m.E0;
  return CEM_OK;
}

int cem_set_modulus(cem_ctx* c, int32_t n_tets, const double* E) {
  if (!c) return CEM_EINVAL;
  int r = ensure_ready(c, false);
  if (r) return r;
  if (c->m.etype == 8) return c->fail(CEM_ESTATE, "a per-element modulus is for tetrahedral meshes");
  c->gen++;
  Mesh& m = c->m;
  if (E) {
    if (n_tets != m.T0) return c->fail(CEM_EINVAL, "one modulus per tet");
    std::vector<double> k(m.T0);
    for (int t = 0; t < m.T0; ++t) {
      if (!(E[t] > 0) || !std::isfinite(E[t])) return c->fail(CEM_EINVAL, "modulus must be finite and positive");
      k[c->tet_new[t]] = E[t] / c->mat.E;
    }
    if (!c->kap_buf) ALLOC(c->kap_buf, m.T_cap, true);
    if ((r = upload(c, c->kap_buf, k.data(), (size_t)m.T0))) return r;
    c->kap_on = true;
    m.kap = c->kap_buf;
  } else {
    c->kap_on = false;
    m.kap = nullptr;
  }
  if ((r = read_counters(c))) return r;
  c->n_split_host = c->h_ctr->n_split;
  HIPCHK(c, launch_kap_copies(m, c->n_split_host, c->stream));
  int En = edges_now_host(c);
  if (c->mixed) HIPCHK(c, Launch<float>::edge_volumes(m, c->w, En, c->stream));
  else HIPCHK(c, Launch<double>::edge_volumes(m, c->w, En, c->stream));
  if ((r = sync(c))) return r;
  c->need_init = true;
  drop_graph(c);
  return CEM_OK;
}

int cem_add_velocity_bc(cem_ctx* c, int32_t n, const int32_t* node, const int32_t* dof_mask,
                        const double* v0, double t0, int32_t* group) {
  if (!c) return CEM_EINVAL;
  int r = ensure_ready(c, false);
  if (r) return r;
  if ((r = read_counters(c))) return r;
  if (c->h_ctr->step != 0) return c->fail(CEM_ESTATE, "prescribed velocities must precede the first step");
  if (c->m.n_inst) return c->fail(CEM_ESTATE, "prescribed velocities are not supported in batches");
  if (n < 0 || (n > 0 && (!node || !dof_mask || !v0))) return c->fail(CEM_EINVAL, "bad arguments");
  if (!(t0 >= 0) || !std::isfinite(t0)) return c->fail(CEM_EINVAL, "ramp time must be finite and >= 0");
  if ((int)c->bc_t0.size() >= 64) return c->fail(CEM_EINVAL, "at most 64 groups");
  Mesh& m = c->m;
  std::vector<char> seen(m.N0, 0);
  for (int i : c->bc_node) seen[i] = 1;
  for (int b = 0; b < n; ++b) {
    if (node[b] < 0 || node[b] >= m.N0) return c->fail(CEM_EINVAL, "constrained node out of range");
    if (dof_mask[b] < 1 || dof_mask[b] > 7) return c->fail(CEM_EINVAL, "dof mask must be 1..7");
    for (int d = 0; d < 3; ++d)
      if (!std::isfinite(v0[3 * b + d])) return c->fail(CEM_EINVAL, "non-finite velocity");
    int in = c->node_new[node[b]];
    if (seen[in]) return c->fail(CEM_EINVAL, "node constrained twice");
    seen[in] = 1;
  }
  c->gen++;
  const int g = (int)c->bc_t0.size();
  for (int b = 0; b < n; ++b) {
    c->bc_node.push_back(c->node_new[node[b]]);
    c->bc_mask.push_back(dof_mask[b] | (g << 4));
    c->bc_v0.push_back(make_double4(v0[3 * b], v0[3 * b + 1], v0[3 * b + 2], 0.0));
  }
  c->bc_t0.push_back(t0);
  c->bc_goff.push_back((int)c->bc_node.size());
  const int nb = (int)c->bc_node.size(), ng = (int)c->bc_t0.size();
  const int H = 65536;
  // displacement reference: the nodes' current u
  std::vector<double4> uall(m.N0);
  HIPCHK(c, hipMemcpyAsync(uall.data(), c->st.u, sizeof(double4) * m.N0, hipMemcpyDeviceToHost, c->stream));
  if ((r = sync(c))) return r;
  // previous groups keep their reference, reaction, work and history rows
  std::vector<double4> ref(nb), react(nb, make_double4(0, 0, 0, 0));
  std::vector<double> work(nb, 0.0), hist((size_t)ng * H * 6, 0.0);
  const int nb_old = c->bc_goff[ng - 1];
  if (nb_old) {
    HIPCHK(c, hipMemcpyAsync(ref.data(), m.bref, sizeof(double4) * nb_old, hipMemcpyDeviceToHost, c->stream));
    if ((r = sync(c))) return r;
  }
  for (int b = nb_old; b < nb; ++b) ref[b] = uall[c->bc_node[b]];
  auto release = [&](void* p) {
    if (!p) return;
    (void)hipFree(p);
    c->allocs.erase(std::remove(c->allocs.begin(), c->allocs.end(), p), c->allocs.end());
    c->regions.erase(std::remove_if(c->regions.begin(), c->regions.end(),
                                    [&](const Region& q) { return q.ptr == p; }),
                     c->regions.end());
  };
  release(m.bnode); release(m.bmask); release(m.bv0); release(m.bref); release(m.breact);
  release(m.bwork); release(m.gt0); release(m.goff); release(m.ghist);
  if (!m.bslot) ALLOC(m.bslot, m.N_cap, false);
  ALLOC(m.bnode, nb, false);
  ALLOC(m.bmask, nb, false);
  ALLOC(m.bv0, nb, false);
  ALLOC(m.bref, nb, false);
  ALLOC(m.breact, nb, true);
  ALLOC(m.bwork, nb, true);
  ALLOC(m.gt0, ng, false);
  ALLOC(m.goff, ng + 1, false);
  ALLOC(m.ghist, (size_t)ng * H * 6, true);
  std::vector<int> slot(m.N_cap, -1);
  for (int b = 0; b < nb; ++b) slot[c->bc_node[b]] = b;
  if ((r = upload(c, m.bslot, slot.data(), slot.size()))) return r;
  if ((r = upload(c, m.bnode, c->bc_node.data(), (size_t)nb))) return r;
  if ((r = upload(c, m.bmask, c->bc_mask.data(), (size_t)nb))) return r;
  if ((r = upload(c, m.bv0, c->bc_v0.data(), (size_t)nb))) return r;
  if ((r = upload(c, m.bref, ref.data(), (size_t)nb))) return r;
  if ((r = upload(c, m.breact, react.data(), (size_t)nb))) return r;
  if ((r = upload(c, m.bwork, work.data(), (size_t)nb))) return r;
  if ((r = upload(c, m.gt0, c->bc_t0.data(), (size_t)ng))) return r;
  if ((r = upload(c, m.goff, c->bc_goff.data(), (size_t)ng + 1))) return r;
  if ((r = upload(c, m.ghist, hist.data(), hist.size()))) return r;
  if ((r = sync(c))) return r;
  m.n_bc = nb;
  m.n_grp = ng;
  m.hist_cap = H;
  c->need_init = true;
  drop_graph(c);
  if (group) *group = g;
  return CEM_OK;
}

int cem_read_reactions(cem_ctx* c, int32_t group, int32_t cap, double* rows, int32_t* n,
                       double* work) {
  if (!c || !n) return CEM_EINVAL;
  int r = ensure_ready(c, false);
  if (r) return r;
  Mesh& m = c->m;
  if (group < 0 || group >= m.n_grp) return c->fail(CEM_EINVAL, "no such group");
  if ((r = read_counters(c))) return r;
  const long long S = c->h_ctr->step;
  const long long cnt = std::min<long long>(S, m.hist_cap);
  *n = (int32_t)cnt;
  if (rows && cap > 0) {
    std::vector<double> h((size_t)m.hist_cap * 6);
    HIPCHK(c, hipMemcpyAsync(h.data(), m.ghist + (size_t)group * m.hist_cap * 6,
                             sizeof(double) * h.size(), hipMemcpyDeviceToHost, c->stream));
    if ((r = sync(c))) return r;
    long long first = S - cnt;
    for (long long k = 0; k < cnt && k < cap; ++k) {
      long long idx = (first + k) % m.hist_cap;
      for (int q = 0; q < 6; ++q) rows[6 * k + q] = h[6 * idx + q];
    }
  }
  if (work) {
    const int b0 = c->bc_goff[group], b1 = c->bc_goff[group + 1];
    std::vector<double> w(std::max(b1 - b0, 1));
    if (b1 > b0) {
      HIPCHK(c, hipMemcpyAsync(w.data(), m.bwork + b0, sizeof(double) * (b1 - b0),
                               hipMemcpyDeviceToHost, c->stream));
      if ((r = sync(c))) return r;
    }
    double s = 0;
    for (int b = 0; b < b1 - b0; ++b) s += w[b];
    *work = s;
  }
  return CEM_OK;
}

int cem_set_step(cem_ctx* c, int64_t step) {
  if (!c) return CEM_EINVAL;
  int r = ensure_ready(c, false);
  if (r) return r;
  if (step < 0) return c->fail(CEM_EINVAL, "negative step");
  c->gen++;
  long long s = step;
  HIPCHK(c, hipMemcpyAsync(&c->d_ctr->step, &s, sizeof(s), hipMemcpyHostToDevice, c->stream));
  if ((r = sync(c))) return r;
  c->step_host = step;
  c->h_ctr->step = step;
  c->need_init = true;
  return CEM_OK;
}

int cem_window_forward(cem_ctx* c, int32_t n, int32_t every) {
  if (!c) return CEM_EINVAL;
  int r = ensure_ready(c, true);
  if (r) return r;
  if (c->m.etype == 8) return c->fail(CEM_ESTATE, "gradient windows are for tetrahedral meshes");
  if (n < 0 || every < 1) return c->fail(CEM_EINVAL, "window needs n_steps >= 0 and every >= 1");
  if (c->m.n_bc || c->m.n_grp)
    return c->fail(CEM_ESTATE, "gradient windows with prescribed velocities are not supported");
  c->gen++;
  auto& W = c->win;
  W.gen = -1;
  if ((r = win_fixed(c))) return r;
  if (c->need_init && (r = initialize(c))) return r;
  W.nodes = nodes_now_host(c);
  W.n = n;
  W.every = every;
  W.n_ck = (n + every - 1) / every + 1;
  const size_t nl = std::max(c->m.n_load, 1);
  const size_t per = sizeof(double4) * 4 * W.nodes + sizeof(Counters) + sizeof(double) * nl + 256;
  size_t bytes = per * W.n_ck;
  if ((r = win_grow(c, (void**)&W.ck, &W.ck_bytes, bytes))) return r;
  W.ckc = (Counters*)((char*)W.ck + sizeof(double4) * 4 * W.nodes * W.n_ck);
  W.ckw = (double*)((char*)W.ckc + ((sizeof(Counters) * W.n_ck + 255) / 256) * 256);
  if ((r = win_grow(c, (void**)&W.tape, &W.tape_bytes, sizeof(double4) * W.nodes * (every + 1))))
    return r;
  c->frozen = 1;
  r = win_save(c, 0);
  for (int j = 0; r == CEM_OK && j + 1 < W.n_ck; ++j) {
    int len = std::min(every, n - j * every);
    r = run_steps(c, len);
    if (r == CEM_OK) r = win_save(c, j + 1);
  }
  c->frozen = 0;
  if (r) return r;
  if ((r = sync(c))) return r;
  W.n_split = c->n_split_host;
  W.gen = c->gen;
  return CEM_OK;
}

int cem_window_backward(cem_ctx* c, const double* gu, const double* gv, double* gu0, double* gv0,
                        double* gE) {
  if (!c) return CEM_EINVAL;
  int r = ensure_ready(c, true);
  if (r) return r;
  auto& W = c->win;
  if (W.gen != c->gen) return c->fail(CEM_ESTATE, "no gradient window pending (cem_window_forward)");
  Mesh& m = c->m;
  for (double& t : W.times) t = 0;
  if ((r = timing_events(c))) return r;
  hipEvent_t e0 = c->tev[0], e1 = c->tev[1];
  HIPCHK(c, hipEventRecord(e0, c->stream));
  // sensitivities at the window's end
  std::vector<double4> tmp(W.nodes, make_double4(0, 0, 0, 0));
  if (gu) pad3(c, gu, tmp, W.nodes);
  if ((r = upload(c, W.p, tmp.data(), W.nodes))) return r;
  tmp.assign(W.nodes, make_double4(0, 0, 0, 0));
  if (gv) pad3(c, gv, tmp, W.nodes);
  if ((r = upload(c, W.q, tmp.data(), W.nodes))) return r;
  HIPCHK(c, hipMemsetAsync(W.gE, 0, sizeof(double) * m.T_cap, c->stream));
  const int En = edges_now_host(c);
  if (c->mixed) HIPCHK(c, Adjoint<float>::inv_volumes(m, W.einv0, En, c->stream));
  else HIPCHK(c, Adjoint<double>::inv_volumes(m, W.einv0, En, c->stream));
  HIPCHK(c, launch_adj_init(m, W.q, W.lam, W.n > 0 ? 0.5 : 0.0, c->d_ctr, c->stream));
  c->frozen = 1;
  r = c->mixed ? reverse_window<float>(c) : reverse_window<double>(c);
  c->frozen = 0;
  if (r) return r;
  // back to the window's end
  if ((r = win_load(c, W.n_ck - 1))) return r;
  HIPCHK(c, hipEventRecord(e1, c->stream));
  if ((r = check_device_error(c))) return r;
  float ms = 0;
  (void)hipEventElapsedTime(&ms, e0, e1);
  W.times[0] = ms;
  // read back in the caller's numbering
  std::vector<double4> h(W.nodes);
  double4* src[2] = {W.p, W.q};
  double* dst[2] = {gu0, gv0};
  for (int k = 0; k < 2; ++k) {
    if (!dst[k]) continue;
    HIPCHK(c, hipMemcpyAsync(h.data(), src[k], sizeof(double4) * W.nodes, hipMemcpyDeviceToHost, c->stream));
    if ((r = sync(c))) return r;
    unpad3(c, h, dst[k], W.nodes);
  }
  if (gE) {
    const int ns = m.mode == MODE_PHANTOM ? c->n_split_host : 0;
    std::vector<double> g((size_t)m.T0 + ns);
    std::vector<int> par(std::max(ns, 1));
    HIPCHK(c, hipMemcpyAsync(g.data(), W.gE, sizeof(double) * g.size(), hipMemcpyDeviceToHost, c->stream));
    if (ns) HIPCHK(c, hipMemcpyAsync(par.data(), m.rec_tet, sizeof(int) * ns, hipMemcpyDeviceToHost, c->stream));
    if ((r = sync(c))) return r;
    for (int s = 0; s < ns; ++s) g[par[s]] += g[(size_t)m.T0 + s];  // a copy adds to its parent
    for (int t = 0; t < m.T0; ++t) gE[t] = g[c->tet_new[t]];
  }
  return CEM_OK;
}

int cem_strain_energy_grad(cem_ctx* c, const double* u, double* se, double* gu, double* gE) {
  if (!c) return CEM_EINVAL;
  int r = ensure_ready(c, false);
  if (r) return r;
  if (c->m.etype == 8) return c->fail(CEM_ESTATE, "a per-element modulus is for tetrahedral meshes");
  Mesh& m = c->m;
  if ((r = win_fixed(c))) return r;
  int n = nodes_now_host(c);
  const double4* src = c->st.u;
  if (u) {
    std::vector<double4> tmp;
    pad3(c, u, tmp, n);
    if ((r = upload(c, c->d_tmp, tmp.data(), n))) return r;
    src = c->d_tmp;
  }
  const int np = c->n_partial;
  // SE = 1/2 sum_k V_k sigma_k . eps_k
  if (c->mixed) {
    HIPCHK(c, Launch<float>::strain(m, src, c->w, c->d_ctr, c->stream));
    HIPCHK(c, launch_strain_energy<float>(m, c->w, c->d_ctr, c->w.partial, np, -1, c->stream));
  } else {
    HIPCHK(c, Launch<double>::strain(m, src, c->w, c->d_ctr, c->stream));
    HIPCHK(c, launch_strain_energy<double>(m, c->w, c->d_ctr, c->w.partial, np, -1, c->stream));
  }
  HIPCHK(c, launch_sum(c->w.partial, np, c->d_out, c->stream));
  // dSE/du = f_int(u)
  if ((r = strain_stress(c, src))) return r;
  if ((r = node_pass(c, NODE_FORCE, c->d_tmp2))) return r;
  // dSE/dE_j = 1/2 (V_j / 6) sum_{k in edges(j)} eps_k . Chat eps_k: the reverse
  // kernels with lambda = u accumulate minus twice that
  auto& W = c->win;
  HIPCHK(c, hipMemsetAsync(W.gE, 0, sizeof(double) * m.T_cap, c->stream));
  const int En = edges_now_host(c);
  const double nu = c->mat.nu;
  const double lh = nu / ((1.0 + nu) * (1.0 - 2.0 * nu)), mh = 1.0 / (2.0 * (1.0 + nu));
  if (c->mixed) {
    HIPCHK(c, Adjoint<float>::inv_volumes(m, W.einv0, En, c->stream));
    HIPCHK(c, Adjoint<float>::strain2(m, src, src, c->w.veps, W.vu, c->d_ctr, c->stream));
    HIPCHK(c, Adjoint<float>::edge2(m, c->w.veps, W.vu, c->w.einvV, W.einv0, c->w.esig, W.z, lh, mh,
                                    c->d_ctr, c->stream));
    HIPCHK(c, Adjoint<float>::elem(m, c->w.esig, W.z, c->w.contrib, W.gE, c->d_ctr, c->stream));
  } else {
    HIPCHK(c, Adjoint<double>::inv_volumes(m, W.einv0, En, c->stream));
    HIPCHK(c, Adjoint<double>::strain2(m, src, src, c->w.veps, W.vu, c->d_ctr, c->stream));
    HIPCHK(c, Adjoint<double>::edge2(m, c->w.veps, W.vu, c->w.einvV, W.einv0, c->w.esig, W.z, lh, mh,
                                     c->d_ctr, c->stream));
    HIPCHK(c, Adjoint<double>::elem(m, c->w.esig, W.z, c->w.contrib, W.gE, c->d_ctr, c->stream));
  }
  double seh = 0;
  HIPCHK(c, hipMemcpyAsync(&seh, c->d_out, sizeof(double), hipMemcpyDeviceToHost, c->stream));
  std::vector<double4> fh(n);
  HIPCHK(c, hipMemcpyAsync(fh.data(), c->d_tmp2, sizeof(double4) * n, hipMemcpyDeviceToHost, c->stream));
  const int ns = m.mode == MODE_PHANTOM ? c->n_split_host : 0;
  std::vector<double> g((size_t)m.T0 + ns);
  std::vector<int> par(std::max(ns, 1));
  HIPCHK(c, hipMemcpyAsync(g.data(), W.gE, sizeof(double) * g.size(), hipMemcpyDeviceToHost, c->stream));
  if (ns) HIPCHK(c, hipMemcpyAsync(par.data(), m.rec_tet, sizeof(int) * ns, hipMemcpyDeviceToHost, c->stream));
  if ((r = sync(c))) return r;
  if ((r = check_device_error(c))) return r;
  if (se) *se = seh;
  if (gu) unpad3(c, fh, gu, n);
  if (gE) {
    for (int s = 0; s < ns; ++s) g[par[s]] += g[(size_t)m.T0 + s];
    for (int t = 0; t < m.T0; ++t) gE[t] = -0.5 * g[c->tet_new[t]];
  }
  return CEM_OK;
}

int cem_window_times(cem_ctx* c, double* out) {
  if (!c || !out) return CEM_EINVAL;
  for (int i = 0; i < 6; ++i) out[i] = c->win.times[i];
  return CEM_OK;
}

int cem_set_topology_mode(cem_ctx* c, int32_t mode) {
  if (!c) return CEM_EINVAL;
  if (mode < 0 || mode > 2) return c->fail(CEM_EINVAL, "topology mode must be 0, 1 or 2");
  c->topo_mode = mode;
  const int multi = mode == 2 ? 1 : 0;
  if (mode != 0 && multi != c->m.topo_multi) {
    c->m.topo_multi = multi;
    drop_graph(c);
  }
  return CEM_OK;
}

int cem_set_profiling(cem_ctx* c, int32_t on) {
  if (!c) return CEM_EINVAL;
  c->profiling = on ? 1 : 0;
  return CEM_OK;
}

int cem_kernel_times(cem_ctx* c, double* out) {
  if (!c || !out) return CEM_EINVAL;
  for (int q = 0; q < 7; ++q) out[q] = c->times[q];
  return CEM_OK;
}

}  // extern "C"
