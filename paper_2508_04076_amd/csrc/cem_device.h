// Device data layout and kernel launchers of the ES-T-FEM crack-element step.
// Internal to libcem; the public interface is include/cem.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cem {

constexpr int kBlock = 256;          // 4 wave64 per workgroup
constexpr int kTopoBlock = 1024;     // single-workgroup topology update
#ifndef CEM_TOPO_INLINE
#define CEM_TOPO_INLINE 128
#endif
constexpr int kTopoInline = CEM_TOPO_INLINE;  // larger batches sum masses and volumes in k_topo_sums
constexpr int kDefaultLanes = 8;         // lanes per node in the node pass
constexpr int kDefaultGridCap = 2048;    // workgroups of the persistent step launches
// workgroup of the tiled force pass: float32 tiles fill a CU's LDS with one
// 1,024-thread workgroup, float64 tiles take two of 512 threads
template <class R> constexpr int tile_block() { return sizeof(R) == 8 ? 512 : 1024; }
// node-list entries of one tile (LDS: 3 values each, 72 KB in float64, 144 KB in float32)
constexpr int kTileEntries64 = 3072;
constexpr int kTileEntries32 = 12288;
// nodes per tile of the fixed-point tiled force pass: three 64-bit sums per
// node in LDS (36 KB; the registers leave room for two 512-thread workgroups
// per CU in float32, one in float64).  Meshes with fewer
// than kFxTargetTiles full tiles take smaller tiles (down to kFxMinNodes, in
// steps of 64) so that the launch still spreads over every CU.
constexpr int kFxNodes = 1536;
constexpr int kFxBlock = 512;
constexpr int kFxMinNodes = 128;
constexpr int kFxTargetTiles = 2048;
constexpr int kSigSlots = 64;        // one wave reads them all
constexpr int kSigStride = 32;       // 256 bytes apart
constexpr int kNodeBits = 28;        // node id bits in the packed node word
constexpr int kNodeMask = (1 << kNodeBits) - 1;

// Volume fraction codes carried in bits 28..31 of an element's first node word.
enum FracCode { FR_ZERO = 0, FR_ONE = 1, FR_HALF = 2, FR_EIGHTH = 3, FR_SEVEN8 = 4 };

enum SplitMode { MODE_PHANTOM = 0, MODE_ERODE = 1 };
enum NodeMode { NODE_FORCE = 0, NODE_INIT = 1, NODE_STEP = 2 };

// Device-resident scalars of one simulation.
struct Counters {
  long long step;                 // steps completed
  int n_split;                    // splits applied
  int n_flag;                     // tets flagged in the current step
  int n_cand;                     // length of the candidate list
  int err;                        // 0 or a negative status raised on the device
  unsigned long long gmax_key;    // ordered key of the running max G (this pass)
  unsigned long long gmax_last;   // key of the last completed crack pass
  double Ud;                      // dissipated energy
  int replay_cursor;              // next entry of the forced schedule
  int ticket;                     // crack pass last-block ticket
  int n_sched;                    // forced schedule length (0: G test decides)
  int n_cand_dead;                // candidate-list entries whose tet has split since
  unsigned long long lam_key;     // ordered key of max element eigenvalue (setup)
  double dt_crit;
  int batch_base;                 // first split of a batch whose masses and edge
  int batch_n;                    // volumes are left to k_topo_sums (0: none)
  int batch_apply_n;              // splits left to k_topo_apply / k_topo_finish (0: none)
  int dead_pending;               // candidates among them (dead list entries)
};

// Six float values of a symmetric tensor in Voigt order
// (xx, yy, zz, xy, yz, xz); strains carry engineering shear.
template <class R> struct alignas(2 * sizeof(R)) Six { R v[6]; };

// Everything a kernel needs, passed by value.
struct Mesh {
  int T0, N0, E0, S_cap;
  int T_cap, N_cap, E_cap;
  int mode;                 // SplitMode
  int gsig;                 // 0 principal, 1 normal
  int n_load;               // loaded nodes
  double lam, mu, rho, Gc;
  double ramp_t0, dt;
  double umax;              // runaway bound on |u|
  int grid_cap;             // workgroups of the persistent step launches (multiple of 8)
  int lanes;                // lanes per node in the node pass (4, 8 or 16)
  int topo_multi;           // 1: split batches over kTopoInline are applied by the whole chip
  int ssum;                 // tets: what the force pass hands to the node pass: 0 = nodal
                            // terms at node-list positions, 1 = per-tet stress sums (the
                            // node pass forms G_l from the corner coordinates)
  int tiled;                // tets: 1 = tiled force pass (terms in LDS per node tile),
                            // 2 = fixed-point tiled pass (64-bit node sums in LDS)
  int ntile[2];             // node tiles of the tiled force pass, float64 and float32 sets (0: none)
  int n_inst;               // independent instances of a batch (0: one simulation)
  int etype;                // nodes per element: 4 (tetrahedra) or 8 (hexahedra)

  int4* enodes;             // [T_cap] node ids; .x also holds the fraction code
  int2* et2e;               // [T_cap * 3] six edge ids (local edge order 01 02 03 12 13 23)
  double4* X;               // [N_cap] coordinates (extra nodes copy their twin)
  // [T_cap][9] g_1, g_2, g_3 (g_l = 6 V grad N_l, the corner face normals of
  // face_normals) of each element slot in float32, streamed by the
  // mixed-precision strain passes instead of four coordinate gathers (the
  // force passes, whose coordinate gathers hide behind their stress gathers,
  // keep forming them); a split copy takes its parent's row (the same corners)
  float* gtab;
  int* poff;                // [E_cap + 1] edge patch offsets
  int* pent;                // [6 T0 + 10 S_cap] element ids, -1 = removed
  int* noff;                // [N_cap + 1] node -> (element, local) offsets
  int* nent;                // [4 T0 + 4 S_cap] packed element << 2 | local
  double* invm;             // [N_cap] 1 / lumped mass (0 for a massless node)
  int* lslot;               // [N_cap] load slot or -1
  double4* Fload;           // [n_load] nodal load vector at full load
  double* wacc;             // [n_load] accumulated external work per loaded node
  int* lnode;               // [n_load] node of each load slot

  int4* nbr;                // [T0] face neighbour per local face, -1 at the boundary
  int* nbrface;             // [T0] packed 4 x 8 bits: neighbour's local face index
  int4* epos;               // [T_cap] position of each (element, local node) in the node lists
  double* vol;              // [T_cap] volume of the parent tetrahedron
  int* tet_ext;             // [T0] the caller's id of each tet (split order key)
  int2* patchpos;           // [T0 * 3] position of t in the patch of its 6 edges
  int4* front;              // [T0] lone node per local face on the crack front, -1 none
  int* smask;               // [T0] -1 intact, else the side mask of the split
  uint8_t* pmask;           // [T0] pending side mask
  uint8_t* ppat;            // [T0] pending pattern (1 = I, 2 = II)
  double* pG;               // [T0] pending release rate
  int* cand;                // [T0] candidate list
  int* candf;               // [T0] on the candidate list
  int* splitlist;           // [next pow2 of S_cap] tets to split this step
  double* area;             // [S_cap] crack area of each split (scratch)
  int* rec_step;            // [S_cap] split records
  int* rec_tet;
  int* rec_mask;
  int* rec_pat;
  double* rec_G;
  int* sched;               // forced schedule (step, tet, mask) triples
  double* rec_area;         // [S_cap] midpoint crack area of each split
  double* kap;              // [T_cap] modulus of each element slot over E (null: uniform E)
  int* split_of;            // [T0] split index of a split tet (its copy B is slot T0 + index)
  // tiles of the tiled force pass, one set per precision ([0] float64, [1] float32: the
  // float32 terms take half the LDS, so its tiles hold twice the entries)
  int* toff[2];             // [ntile + 1] first node of each tile
  int* ttoff[2];            // [ntile + 1] offsets into ttet
  int* ttet[2];             // tile element lists: parent tets with an entry in the tile, ascending
  // tiles of the fixed-point tiled pass (up to kFxNodes consecutive nodes each)
  int ntile_fx;
  int* toff_fx;
  int* ttoff_fx;
  int* ttet_fx;
  double fx_g1;             // max over tets and local nodes of |G_l|_1 (G_l = 6 V grad N_l)
  int fx_deg;               // longest node list of an original node
  // [kSigSlots slots, kSigStride apart] ordered keys of max |sigma| over the
  // edges of this step, each slot taken by every kSigSlots-th workgroup of
  // the edge pass (spread over memory so that the atomics do not queue on
  // one address); the force pass takes the largest
  unsigned long long* sig_slot;

  // trilinear hexahedra (etype 8; T_cap = T0).  A cracked hex keeps its slot
  // and carries the volume fraction its crack plane leaves (vol scaled);
  // smask holds its plane index, pmask the pending one.
  int4* hnodes;             // [2 T0] node ids 0-3, 4-7
  int2* he2e;               // [6 T0] twelve edge ids
  int* hnbr;                // [6 T0] neighbour across local face f: 8 hex + its local face, -1 none
  int* hfront;              // [6 T0] crack front on local face f: 16 qa + qb (its two cut local edges), -1 none

  // prescribed velocities in groups (all null, counts 0, when there are none)
  int n_bc, n_grp, hist_cap;
  int* bslot;               // [N_cap] slot of a constrained node, -1 none
  int* bnode;               // [n_bc] node of each slot
  int* bmask;               // [n_bc] dof mask (bit d) | group << 4
  double4* bv0;             // [n_bc] velocity after the ramp
  double4* bref;            // [n_bc] displacement when the group was added
  double4* breact;          // [n_bc] current reaction m a + f_int - f_ext
  double* bwork;            // [n_bc] accumulated work of the reaction
  double* gt0;              // [n_grp] ramp time of each group
  int* goff;                // [n_grp + 1] slot range of each group
  double* ghist;            // [n_grp][hist_cap][6] step, t, R_x, R_y, R_z, S(t)

  // batch of independent instances (all null when n_inst == 0)
  int* inst;                // [N_cap] instance of each node
  int* tinst;               // [T_cap] instance of each element slot
  int* einst;               // [E_cap] instance of each edge
  double* dti;              // [n_inst] time step of each instance
  unsigned long long* gmax_inst;  // [2 n_inst] running / last max G key per instance
  unsigned long long* lam_inst;   // [n_inst] max element eigenvalue key per instance
  double* dtc_inst;         // [n_inst] critical time step per instance
};

// Device pointers of the precision-dependent work arrays.
struct Work {
  void* veps;               // [T_cap] Six<R>: effective volume x element strain
  void* esig;               // [E_cap] Six<R>: smoothed edge stress
  void* einvV;              // [E_cap] R: kappa_k / sum of effective volumes of the patch,
                            // kappa_k the volume-averaged relative modulus (1 if uniform)
  void* contrib;            // [4 T_cap][3] R: nodal force term of each node-list entry, or
                            // [T_cap] Six<R>: (f/36) sum sigma per element (per hex: (1/12) sum sigma)
  double* partial;          // reduction partials
};

struct State {
  double4* u;   // displacement at step n
  double4* v;   // velocity at step n
  double4* a;   // acceleration at step n
  double4* uh;  // predictor u_n + dt v_n + dt^2/2 a_n (the u at which f is evaluated next)
};

// ---- launchers (kernels.hip) ----
template <class R> struct Launch {
  static hipError_t strain(const Mesh& m, const double4* u, const Work& w, Counters* c,
                           hipStream_t s);
  static hipError_t edge_stress(const Mesh& m, const Work& w, Counters* c, hipStream_t s);
  // front: -1 no crack pass; 1 crack pass with flagging; 0 crack pass for the
  // readbacks only, then the forced schedule's selection (replay)
  static hipError_t node(const Mesh& m, const State& st, const Work& w, Counters* c, int mode,
                         double4* fout, hipStream_t s, hipEvent_t mid = nullptr, int front = -1);
  // einvV of the first `count` edges (count < 0: the original edges)
  static hipError_t edge_volumes(const Mesh& m, const Work& w, int count, hipStream_t s);
  static hipError_t front_eval(const Mesh& m, const State& st, const Work& w, Counters* c,
                               int* out_tfl, double* out_g, int* out_n, hipStream_t s);
};

template <class R>
hipError_t launch_strain_energy(const Mesh& m, const Work& w, Counters* c, double* partial,
                                int nparts, int inst, hipStream_t s);
template <class R>
hipError_t launch_topology_t(const Mesh& m, const State& st, const Work& w, Counters* c,
                             int dynamic, int advance, int4* snodes, int* sedges, hipStream_t s);
hipError_t launch_replay_select(const Mesh& m, Counters* c, hipStream_t s);
hipError_t launch_masses(const Mesh& m, hipStream_t s);
hipError_t launch_normals(const Mesh& m, const Counters* c, hipStream_t s);
hipError_t launch_loads(const Mesh& m, const int4* ftri, const double4* ftrac, const int* lfoff,
                        const int* lfent, hipStream_t s);
hipError_t launch_dtcrit(const Mesh& m, Counters* c, hipStream_t s);
// readbacks: inst < 0 sums over everything, else over one instance of a batch
hipError_t launch_kinetic(const Mesh& m, const State& st, Counters* c, double* partial,
                          int nparts, int inst, hipStream_t s);
hipError_t launch_sum(const double* partial, int n, double* out, hipStream_t s);
hipError_t launch_count_fronts(const Mesh& m, Counters* c, int* out, int inst, hipStream_t s);
hipError_t launch_work_sum(const Mesh& m, double* out, int inst, hipStream_t s);
hipError_t launch_dissipated(const Mesh& m, Counters* c, double* out, int inst, hipStream_t s);
hipError_t launch_edge_instances(const Mesh& m, hipStream_t s);
// prescribed displacement of the constrained components at the current time
hipError_t launch_bc_apply(const Mesh& m, const State& st, const Counters* c, hipStream_t s);
// per-group reaction sums of the step just taken, into the history ring
hipError_t launch_reaction(const Mesh& m, const Counters* c, hipStream_t s);
// split copies take their parent's relative modulus (n_split copies)
hipError_t launch_kap_copies(const Mesh& m, int n_split, hipStream_t s);
hipError_t launch_set_presplit(const Mesh& m, Counters* c, const int* tets, const uint8_t* masks,
                               int n, hipStream_t s);
// ---- trilinear hexahedra (hex.hip) ----
hipError_t launch_hex_geometry(const Mesh& m, hipStream_t s);
template <class R>
hipError_t launch_strain_hex(const Mesh& m, const double4* u, void* veps, Counters* c, hipStream_t s);
template <class R>
hipError_t launch_elem_force_hex(const Mesh& m, const void* esig, void* contrib, const double4* uh,
                                 Counters* c, int fg, int flagging, hipStream_t s);
hipError_t launch_dtcrit_hex(const Mesh& m, Counters* c, hipStream_t s);

// ---- reverse sweep of a fixed-topology window (adjoint.hip) ----
template <class R> struct Adjoint {
  static hipError_t strain2(const Mesh& m, const double4* lam, const double4* u, void* vl,
                            void* vu, const Counters* c, hipStream_t s);
  // lh, mh: Lame constants at unit modulus
  static hipError_t edge2(const Mesh& m, const void* vl, const void* vu, const void* einvV,
                          const void* einv0, void* esig, void* z, double lh, double mh,
                          const Counters* c, hipStream_t s);
  static hipError_t elem(const Mesh& m, const void* esig, const void* z, void* contrib,
                         double* gE, const Counters* c, hipStream_t s);
  static hipError_t node(const Mesh& m, const void* contrib, double4* p, double4* q,
                         double4* lam, int last, int half, const Counters* c, hipStream_t s);
  static hipError_t inv_volumes(const Mesh& m, void* out, int count, hipStream_t s);
};
hipError_t launch_adj_init(const Mesh& m, const double4* q, double4* lam, double coef,
                           const Counters* c, hipStream_t s);

int grid_for(long long n);
double key_to_double_host(unsigned long long k);

}  // namespace cem
