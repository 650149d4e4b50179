/*
 * cem.h -- C-ABI of the MI355X (gfx950) explicit step of the 3D crack element
 * method: edge-based smoothed FEM on linear tetrahedra (ES-T-FEM) with split
 * crack elements.
 *
 * The method follows "A GPU-Accelerated Three-Dimensional Crack Element
 * Method for Transient Dynamic Fracture Simulation" (arXiv 2508.04076):
 *   - smoothed strain at every edge from the tets sharing it, weighted by
 *     volume (Section 2.2, Eqs. strain_discretization and
 *     CSTet_strain_discretization); stress sigma = C eps for isotropic linear
 *     elasticity (Section 2.1);
 *   - internal force from the edge smoothing domains (Eqs.
 *     fint_discretization and CSTet_fint_discretization, expanded form with
 *     V_k = (1/6) sum of the volumes sharing edge k), lumped mass (Eq.
 *     mass_discretization), face traction loads (the f_ext equation);
 *   - explicit Newmark, beta = 0, gamma = 1/2 (end of Section 2.2);
 *   - crack pass of Section 3: edge stretch (Eq. stretch-delta), release
 *     rates G_I and G_II of the two tetrahedral crack patterns (Eqs. G-I and
 *     G-II), Griffith test G >= Gc (Section 2.1) and element splitting.
 *
 * Conventions
 *   - Every call returns int status: CEM_OK (0) or a negative CEM_E* code; the
 *     message of the last failure is cem_last_error(ctx) (context-owned).
 *   - Ids are 0-based int32.  Coordinates, displacements, velocities and
 *     forces are row-major [n][3] float64 host arrays in SI units.
 *   - Host pointers are borrowed for the duration of the call and copied.
 *     Device pointers given to cem_bind_state are borrowed, must outlive the
 *     context and are never freed by it.
 *   - All device work is enqueued on the stream given at creation.  Calls that
 *     return data to the host synchronize that stream.
 *   - A context is single-threaded; separate contexts are independent.
 *   - cem_create performs no device call.  cem_upload_mesh validates and
 *     preprocesses on the host first, then allocates device memory.
 */
#ifndef CEM_H
#define CEM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  CEM_OK = 0,
  CEM_EINVAL = -1,     /* bad argument */
  CEM_ENOMEM = -2,     /* device or host allocation failed */
  CEM_EHIP = -3,       /* HIP runtime error (no device, launch failure) */
  CEM_EMESH = -4,      /* invalid mesh (degenerate or duplicated tet, face shared by > 2 tets) */
  CEM_ECAPACITY = -5,  /* split capacity exhausted; state left at the start of the failing step */
  CEM_EUNSTABLE = -6,  /* non-finite or runaway state (time step above the stability limit) */
  CEM_ESTATE = -7      /* call out of order (e.g. step before upload or before cem_set_dt) */
};

enum { CEM_FP64 = 0, CEM_MIXED = 1 };          /* force arithmetic precision */
enum { CEM_PHANTOM = 0, CEM_ERODE = 1 };       /* what a split does to the tet */
enum { CEM_GSIG_PRINCIPAL = 0, CEM_GSIG_NORMAL = 1 };
/* what the tet element force pass hands to the node pass (cem_set_launch) */
enum { CEM_LAYOUT_TERMS = 0, CEM_LAYOUT_STRESS_SUMS = 1, CEM_LAYOUT_TILES = 2, CEM_LAYOUT_TILES_FX = 3 };

typedef struct cem_ctx cem_ctx;

typedef struct {
  int32_t device;       /* HIP device ordinal */
  void* stream;         /* hipStream_t, borrowed; NULL: the context creates and
                           owns a non-blocking stream */
  int32_t precision;    /* CEM_FP64: all force arithmetic in float64.
                           CEM_MIXED: gradients, strains, stresses and nodal
                           force terms in float32; u, v, a, time step, forces
                           sums, energies and G in float64 */
  int32_t split_mode;   /* CEM_PHANTOM: a split tet becomes two copies that
                           each carry the parent's gradients, a volume
                           fraction (1/2,1/2 for a 2|2 partition; 1/8 on the
                           lone-node side and 7/8 on the other for 1|3) and
                           four fresh extra nodes for the other side.
                           CEM_ERODE: the split tet carries no volume (the
                           "deactivated" element of Section 3) */
  int32_t gsig;         /* stress term of Eqs. G-I/G-II: CEM_GSIG_PRINCIPAL
                           uses sigma_1 |P_1 n| (largest principal stress,
                           P_1 projector on its eigenspace); CEM_GSIG_NORMAL
                           uses n.sigma.n */
  int32_t max_splits;   /* split capacity (host pre-splits + splits in steps) */
  int32_t graph_steps;  /* steps per captured HIP graph in cem_step; 0 = plain launches */
} cem_options;

typedef struct {
  double E;    /* Young's modulus (Pa) */
  double nu;   /* Poisson ratio */
  double rho;  /* density (kg/m^3) */
  double Gc;   /* critical energy release rate (J/m^2); +inf disables splitting */
} cem_material;

typedef struct {
  int64_t step;     /* steps taken */
  double t;         /* step * dt */
  double KE;        /* 1/2 sum m |v|^2 */
  double SE;        /* 1/2 sum_k V_k sigma_k . eps_k over edges (engineering shear) */
  double Wext;      /* work of the external load, trapezoidal in time */
  double Ud;        /* Gc * midpoint crack area, summed over splits decided by the G test */
  double Gmax;      /* largest G over the candidates of the last crack pass (0 if none) */
  int32_t n_split;  /* split tets so far (pre-splits included) */
  int32_t n_front;  /* crack-front faces of the current topology */
  int32_t n_nodes;  /* nodes now (original + extra) */
  int32_t n_elems;  /* element slots in use */
} cem_energy;

typedef struct {
  int32_t step;       /* step at whose end the split was applied (0: before stepping) */
  int32_t tet;        /* original tet id (hex meshes: hex id) */
  int32_t side_mask;  /* bit l set: local node l on side B (the lone node's side); hexes: crack plane 0-22 */
  int32_t pattern;    /* 1 = pattern I (quadrilateral), 2 = pattern II (triangle), hexes 3-6 = III-VI,
                         0 = host pre-split */
  double G;           /* release rate that triggered the split (0 for pre-splits) */
} cem_split_event;

typedef struct {
  int32_t tet;   /* intact candidate tet (hex meshes: hex) */
  int32_t face;  /* its local face on the crack front (face opposite local node `face`; hexes:
                    2 axis + (side > 0)) */
  int32_t lone;  /* node of that face alone on its side of the neighbour's cut (N2); hexes: the
                    candidate's crack plane */
  int32_t pad;
  double G_I;    /* Eq. G-I (hexes: the candidate's G, Eq. G-I or G-II) */
  double G_II;   /* Eq. G-II (hexes: the candidate's pattern, 3-6) */
} cem_front_g;

/* Create a context.  Validates the options only (no device call). */
int cem_create(const cem_options* opt, cem_ctx** out);
void cem_destroy(cem_ctx* ctx);
const char* cem_last_error(const cem_ctx* ctx);

/* Mesh upload (Section 2.2).  X: [n_nodes][3]; tets: [n_tets][4].  Each tet is
 * reordered to positive volume by swapping its local nodes 2 and 3; a tet with
 * |V| <= 1e-12 (mean edge length)^3, a duplicated tet or a face shared by more
 * than two tets gives CEM_EMESH.  Builds edges, edge patches, node and face
 * adjacency on the host, then computes volumes and lumped masses on the
 * device.  Callable once per context. */
int cem_upload_mesh(cem_ctx* ctx, int32_t n_nodes, const double* X, int32_t n_tets,
                    const int32_t* tets, const cem_material* mat);

/* Trilinear hexahedral mesh instead of tetrahedra (the paper's second element
 * family, Eqs. hex_strain_discretization and hex_fint_discretization): hexes
 * [H][8] with nodes 0-1-2-3 counter-clockwise on the bottom face (seen from
 * above) and 4-7 above them; a hex inverted throughout is mirrored, one whose
 * Jacobian determinant changes sign over its Gauss points and edge midpoints
 * is CEM_EMESH.  Each hex enters the smoothing domain of each of its
 * 12 edges with its shape-function gradients at that edge's midpoint G_k
 * (Eq. strain_discretization evaluates dN/dx at G_k), the smoothing domains
 * have V_k = (1/12) sum of the patch volumes (volumes by 2 x 2 x 2 Gauss
 * points), and the lumped mass is rho V / 8 per node.
 * Cracks (Section 3, patterns III-VI of the parallelepiped element) grow from
 * hexes cracked by cem_presplit, whose side_mask then holds a crack plane
 * index: planes c . xi = d through edge midpoints in the hex's natural
 * coordinates, 0-2 the mid-planes xi_a = 0, 3-14 the wedge planes
 * +-xi_a +-xi_b = 1 (axis pairs (0,1), (0,2), (1,2); index 3 + 4 pair +
 * 2 [c_a > 0] + [c_b > 0]), 15-22 the corner planes +-xi_0 +-xi_1 +-xi_2 = 2
 * (index 15 + 4 [c0 > 0] + 2 [c1 > 0] + [c2 > 0]).  A face of an intact hex cut
 * by a cracked neighbour's plane (at two of its edge midpoints G1, G2) is a
 * crack front; opposite edges give III (the mid-plane, Eq. G-I; the hex is
 * deactivated) and IV (the two wedge planes tilted toward either side, Eq.
 * G-I), neighbouring edges V (the wedge plane along the face normal, Eq. G-I)
 * and VI (the corner plane at their shared corner, Eq. G-II).  After IV-VI the
 * hex keeps its gradients and half its volume (the triangular prism of its
 * own nodes on the far side); masses stay; a hex cracks once; ties: larger
 * G, lower local face (2 axis + (side > 0)), then III, IV toward -1, IV toward
 * +1, V, VI.  Split events report the plane in side_mask and the pattern 3-6;
 * cem_read_front_G gives one row per candidate: (hex, face, plane in `lone`),
 * G in G_I and the pattern in G_II.  Forced schedules, batches, the
 * per-element modulus, gradient windows and the static front readback return
 * CEM_ESTATE for hexes.  Tractions (triangles), prescribed velocities, steps,
 * energies and checkpoints work as for tetrahedra. */
int cem_upload_hex_mesh(cem_ctx* ctx, int32_t n_nodes, const double* X, int32_t n_hex,
                        const int32_t* hexes, const cem_material* m);

/* Face tractions (the f_ext equation): boundary triangles tri [n_faces][3]
 * with traction vectors t [n_faces][3] (Pa).  Each triangle adds t A / 3 to
 * each vertex.  Load factor r(t) = t / ramp_t0 below ramp_t0, else 1
 * (ramp_t0 = 0: full load from t = 0).  Replaces earlier tractions. */
int cem_set_traction(cem_ctx* ctx, int32_t n_faces, const int32_t* tri, const double* t,
                     double ramp_t0);

/* Split tets from the host (e.g. a pre-notch): side_mask bit l puts local node
 * l (after orientation) on side B; it must be a 1|3 or 2|2 partition.  Already
 * split tets are ignored.  No dissipated energy is booked.  On a hex mesh the
 * elements are hexes and side_mask is a crack plane index 0-22
 * (cem_upload_hex_mesh). */
int cem_presplit(cem_ctx* ctx, int32_t n, const int32_t* tet, const uint8_t* side_mask);

/* dt_crit = 2 / sqrt(max_e (4 / rho) lambda_max(B_e^T C B_e)): the element
 * bound on the largest frequency of M^-1 K, valid for every split state. */
int cem_critical_dt(cem_ctx* ctx, double* dt_crit);
int cem_set_dt(cem_ctx* ctx, double dt);

/* Switch the force arithmetic (CEM_FP64 or CEM_MIXED) of an uploaded
 * context, keeping its mesh, topology and state (u, v, a and the predictor
 * carry over as they are): the per-edge inverse patch volumes are recomputed
 * in the new type and a captured graph is dropped.  Checkpoints name the
 * precision they were taken at and load only into a context at that
 * precision. */
int cem_set_precision(cem_ctx* ctx, int32_t precision);

/* Steps per captured HIP graph in cem_step from now on (0 = plain launches);
 * drops a captured graph. */
int cem_set_graph_steps(cem_ctx* ctx, int32_t graph_steps);

/* How the last cem_step call ran: out[0] steps, out[1] graph launches,
 * out[2] steps per graph, out[3] steps enqueued as plain launches (a call
 * with fewer steps than a graph, a remainder, or profiling on). */
int cem_last_run(cem_ctx* ctx, int64_t* out);

/* Use caller device buffers for u and v (e.g. torch tensors of shape
 * [capacity_nodes][4], float64): each holds capacity_nodes rows of four
 * float64 (x, y, z, unused), capacity_nodes >= n_nodes + 4 max_splits in
 * CEM_PHANTOM mode, >= n_nodes otherwise (CEM_EINVAL below).  The current
 * state is copied into them and the context works in them from then on; they
 * are borrowed, must outlive the context and are never freed by it.  Rows are
 * in the library's internal node order (a locality order of its own): row
 * cem_node_rows gives for caller node i.  Work on them is enqueued on the
 * context's stream; synchronize it before reading them elsewhere. */
int cem_bind_state(cem_ctx* ctx, double* d_u, double* d_v, int64_t capacity_nodes);

/* row[i] = the internal row of caller node i, for the first n nodes now
 * (original nodes, then the extra nodes of the splits in split order, whose
 * rows are their ids). */
int cem_node_rows(cem_ctx* ctx, int32_t n, int32_t* row);

/* Host state in and out, [n_nodes_now][3].  Either pointer may be NULL.  After
 * cem_set_state the next step first recomputes a = M^-1 (f_ext - f(u)). */
int cem_set_state(cem_ctx* ctx, const double* u, const double* v);
int cem_get_state(cem_ctx* ctx, double* u, double* v, double* a, int32_t* n_nodes_now);

/* Internal force f(u) on the current topology, [n_nodes_now][3] in and out. */
int cem_internal_force(cem_ctx* ctx, const double* u, double* f);

/* n_steps explicit steps.  Each step: smoothed strain (per tet), smoothed
 * stress (per edge), crack pass (per candidate), node force and Newmark
 * update, topology update of the new splits. */
int cem_step(cem_ctx* ctx, int32_t n_steps);

/* Forced split schedule (step, tet, side_mask; other fields ignored), applied
 * at the end of the listed steps instead of the G test. */
int cem_replay_splits(cem_ctx* ctx, int32_t n, const cem_split_event* ev);

int cem_read_energy(cem_ctx* ctx, cem_energy* e);
/* Split events in order (pre-splits first); *n = total, at most cap written. */
int cem_read_splits(cem_ctx* ctx, int32_t cap, cem_split_event* out, int32_t* n);
/* G_I and G_II of every current crack-front face, at the current state,
 * sorted by (tet, face); *n = total, at most cap written. */
int cem_read_front_G(cem_ctx* ctx, int32_t cap, cem_front_g* out, int32_t* n);

/* Allocation-free variant of cem_read_front_G for callers that cannot
 * allocate device memory (tight serving loops, harnesses that forbid
 * hipMalloc): the same records in the same order, staged in one static
 * device array per GPU (set up by the mesh upload) instead of buffers
 * allocated per call.  The array holds 65,536 front slots, four per
 * crack-front candidate tet: more than 16,384 candidates give CEM_ECAPACITY.
 * cap = 0 only sets *n; otherwise cap must be at least *n (CEM_EINVAL,
 * nothing written).  All contexts on one GPU share its array, which keeps the
 * last call's contents: calls that overlap on one GPU (from several host
 * threads) race.  Tetrahedral meshes only (CEM_ESTATE on a hex mesh). */
int cem_read_front_G_static(cem_ctx* ctx, int32_t cap, cem_front_g* out, int32_t* n);

/* Checkpoint of the whole simulation state into a host buffer (buf may be
 * NULL to query the size) and restore into a context created with the same
 * options and mesh. */
int cem_save_state(cem_ctx* ctx, void* buf, int64_t cap, int64_t* used);
int cem_load_state(cem_ctx* ctx, const void* buf, int64_t size);

/* out[0..5]: nodes now, element slots now, edges now, splits, fronts,
 * original edge count. */
int cem_counts(cem_ctx* ctx, int32_t* out);

/* ---- Batches (ensembles of independent simulations in one launch per pass)
 *
 * Declare the uploaded mesh as n independent instances: instance i owns the
 * caller's nodes [node_off[i], node_off[i+1]) and tets [tet_off[i],
 * tet_off[i+1]); no tet may join two instances.  All instances step together
 * in the same kernel launches, each with its own time step.  Call after
 * cem_upload_mesh and before cem_presplit / cem_step. */
int cem_set_instances(cem_ctx* ctx, int32_t n, const int32_t* node_off, const int32_t* tet_off);
/* Time step of each instance, dt[n] (replaces cem_set_dt for a batch). */
int cem_set_dt_instances(cem_ctx* ctx, const double* dt);
/* Critical time step of each instance (same bound as cem_critical_dt). */
int cem_critical_dt_instances(cem_ctx* ctx, double* dt_crit);
/* Energies, Gmax and counts of each instance; n must equal the batch size. */
int cem_read_energy_instances(cem_ctx* ctx, int32_t n, cem_energy* out);

/* Launch shape of the step passes: persistent grid size (a positive multiple
 * of 8 workgroups), lanes per node in the node pass (4, 8 or 16) and the tet
 * force layout: CEM_LAYOUT_TERMS (default) stores the four nodal terms
 * (f/36) G_l^T s of each tet (s = sum of its six edge stresses, G_l = 6 V grad
 * N_l, Eq. fint_discretization in its element form) at the node-list
 * positions; CEM_LAYOUT_STRESS_SUMS stores (f/36) s once per tet and the node
 * pass forms G_l^T from the corner coordinates; CEM_LAYOUT_TILES forms the
 * terms and the node sums in one launch, a workgroup per tile of consecutive
 * nodes, the terms kept on chip (the same bits as CEM_LAYOUT_TERMS at equal
 * lanes; the crack-front pass then takes a launch of its own);
 * CEM_LAYOUT_TILES_FX does the same with tiles of up to 1,536 nodes whose
 * sums are 64-bit fixed point in LDS (each term rounded to a multiple of
 * 2^-k, k from the step's largest edge stress so that no node sum can reach
 * 2^61; integer additions make the sums independent of their order; lanes are
 * ignored).  The same forces in every layout up to rounding; which is faster
 * depends on the mesh size and precision.  Hexahedra always hand over nodal
 * terms and ignore the layout.  Lanes and layout set the order of the node
 * sums, hence the rounding.  A tiled layout on a mesh without tiles (a node
 * with more than 3,072 list entries for CEM_LAYOUT_TILES, or hexahedra) is
 * CEM_EINVAL. */
int cem_set_launch(cem_ctx* ctx, int32_t grid_cap, int32_t lanes, int32_t layout);
/* Autotuner of the launch shape: times trial_steps steps of the live
 * simulation for each candidate (layout x grid 1024..8192 x lanes 4, 8, 16;
 * one lane count for CEM_LAYOUT_TILES_FX),
 * restores the state after every trial and keeps the fastest (any output may
 * be NULL). */
int cem_autotune(cem_ctx* ctx, int32_t trial_steps, int32_t* best_grid, int32_t* best_lanes,
                 int32_t* best_layout, double* best_ms_per_step);

/* ---- Heterogeneous modulus and fixed-topology gradient windows
 *
 * Young's modulus of every tet, E[n_tets] in Pa in the caller's tet order
 * (NULL: back to the material's scalar E).  Each split copy takes its
 * parent's modulus.  The smoothing domain of edge k gets the volume-averaged
 * elasticity C_k = sum_{j in patch k} w_jk C(E_j) of the expanded form of
 * Eq. CSTet_fint_discretization, so sigma_k = C_k eps_k.  Any value that is
 * not finite and positive is CEM_EINVAL.  Call cem_critical_dt again after a
 * change: the bound scales with the largest modulus. */
int cem_set_modulus(cem_ctx* ctx, int32_t n_tets, const double* E);

/* ---- Prescribed velocities (Dirichlet boundaries) and reactions
 *
 * One group per call, before the first step: the components selected by
 * dof_mask[b] (bit d = component d, 1..7) of node[b] (caller's ids) follow
 * the velocity v0[b][d] * V(t) with V = t / t0 up to t0, then 1 (t0 = 0: 1 from
 * the start), the ramp of the paper's Dirichlet examples (Sections 4.1, 4.2,
 * 4.3 and 4.5).  The displacement is u_ref + v0 S(t) (S the integral of V,
 * u_ref the node's u when the group is added), the acceleration v0 dV/dt
 * (1/t0 on the ramp, taken on the ramp at t = t0).  Each step records, per
 * group, the summed reaction m a + f_int - f_ext on the constrained
 * components (the force the support exerts on the body).  Extra nodes of
 * split copies are free.  A node may belong to one group only; at most 64
 * groups; not with batches or gradient windows (CEM_ESTATE).  *group gets
 * the group id (may be NULL). */
int cem_add_velocity_bc(cem_ctx* ctx, int32_t n, const int32_t* node, const int32_t* dof_mask,
                        const double* v0, double t0, int32_t* group);
/* Reaction history of a group, oldest first: rows[n][6] = step, t, R_x, R_y,
 * R_z, S(t) (the loading points' displacement is u_ref + v0 S(t)).  The last
 * 65,536 steps are kept; *n = rows available, at most cap written.  *work
 * (may be NULL) = the group's reaction work, trapezoid rule per step. */
int cem_read_reactions(cem_ctx* ctx, int32_t group, int32_t cap, double* rows, int32_t* n,
                       double* work);

/* Set the step counter, hence the time t = step * dt at which the load ramp
 * is evaluated (the state and the accumulated external work are kept; the
 * next step recomputes a from u). */
int cem_set_step(cem_ctx* ctx, int64_t step);

/* Forward half of a gradient window: n_steps steps (Newmark beta = 0,
 * gamma = 1/2, end of Section 2.2) from the current state with the crack pass
 * off, so the topology stays fixed.  The state (u, v, a, predictor,
 * counters, external work) is checkpointed in device memory at the start,
 * every `every` steps and at the end: about 128 (n_steps / every + 2) bytes
 * per node, plus (every + 1) * 32 bytes per node of recompute tape at the
 * backward.  The state is left at the end of the window, as cem_step leaves
 * it.  Any call that changes the state, the mesh or the launch shape
 * afterwards (cem_step, cem_set_state, cem_set_modulus, ...) discards the
 * window. */
int cem_window_forward(cem_ctx* ctx, int32_t n_steps, int32_t every);

/* Reverse half: given gu = dJ/du_n and gv = dJ/dv_n at the window's end
 * ([n_nodes_now][3] in the caller's node order, either may be NULL = 0),
 * returns dJ/du_0 and dJ/dv_0 ([n_nodes_now][3]) and dJ/dE ([n_tets], per Pa;
 * copies add to their parent tet); any output may be NULL.  This is the
 * discrete adjoint of the window's update: each checkpoint segment is
 * recomputed forward, then reversed step by step with K^T = K.  The state is
 * restored to the window's end.  CEM_ESTATE if no window is pending. */
int cem_window_backward(cem_ctx* ctx, const double* gu, const double* gv, double* gu0,
                        double* gv0, double* gE);

/* Strain energy SE = 1/2 sum_k V_k sigma_k . eps_k at displacement u
 * ([n_nodes_now][3], caller's order; NULL: the current state) and its
 * sensitivities: gu = dSE/du (the internal force, [n_nodes_now][3]) and
 * gE = dSE/dE_j at fixed u ([n_tets], per Pa; copies add to their parent).
 * With gu as the window's end sensitivity, gE plus the window's dJ/dE is the
 * gradient of the end-of-window strain energy.  Any output may be NULL;
 * tetrahedral meshes only. */
int cem_strain_energy_grad(cem_ctx* ctx, const double* u, double* se, double* gu, double* gE);

/* Time of the last cem_window_backward, in milliseconds: out[0] whole call,
 * out[1] forward recompute of the segments, out[2] reverse strain pass,
 * out[3] reverse edge pass, out[4] reverse element pass, out[5] reverse node
 * pass.  out[1..5] are recorded only when profiling is on. */
int cem_window_times(cem_ctx* ctx, double* out);

/* Time of the kernels of the last cem_step, in milliseconds, measured with
 * HIP events on the context stream: out[0] whole call, out[1] strain pass,
 * out[2] edge stress pass, out[3] crack pass, out[4] element force terms,
 * out[5] node sums and update, out[6] topology pass.  Per-pass times are
 * recorded only when profiling is on (cem_set_profiling(ctx, 1)); the steps
 * then run as plain launches (HIP cannot time events recorded inside a
 * graph). */
int cem_set_profiling(cem_ctx* ctx, int32_t on);

/* How a step's splits are applied (Section 3, split elements): 0 = automatic
 * (default: the whole chip for batches over 128 splits while the run splits
 * more than 64 tets per step, until it drops below 16), 1 = one workgroup
 * always, 2 = the whole chip for every batch over 128 splits.  The results
 * are the same in every mode; only the launches differ (the whole-chip path
 * takes two more per step).  CEM_EINVAL for another value. */
int cem_set_topology_mode(cem_ctx* ctx, int32_t mode);
int cem_kernel_times(cem_ctx* ctx, double* out);

#ifdef __cplusplus
}
#endif
#endif /* CEM_H */
