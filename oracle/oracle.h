/*
 * Oracle for the 3D crack element method step -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, FP64 CPU implementation of edge-based smoothed FEM on linear
 * tetrahedra (ES-T-FEM, Section 2.2), explicit Newmark time stepping
 * (beta = 0, gamma = 1/2, end of Section 2.2) and the crack element pass of
 * Section 3 (edge stretch, Eq. stretch-delta; release rates G_I and G_II,
 * Eqs. G-I and G-II; Griffith test of Section 2.1) with element splitting.
 *
 * Only the tests, the smoke check and the CPU-baseline leg of the bench may
 * load this library.  It shares no code with the GPU library.
 *
 * All ids 0-based int32; coordinates, displacements, forces row-major [n][3].
 * Every call returns 0 on success and a negative code on error (message via
 * orc_error).
 */
#ifndef CEM_ORACLE_H
#define CEM_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct orc_ctx orc_ctx;

/* split_mode: 0 = phantom-node copies (element splitting), 1 = erosion
 * (the split element is removed).  gsig: 0 = largest principal stress times
 * the length of the projection of n onto its eigenspace, 1 = normal stress
 * n.sigma.n. */
orc_ctx* orc_create(int n_nodes, const double* X, int n_tets, const int* tets,
                    double E, double nu, double rho, double Gc,
                    int split_mode, int gsig);
/* Trilinear hexahedra, 8 nodes each (bottom face 0-1-2-3 counter-clockwise
 * seen from above, top face 4-7 above them).  Crack patterns III-VI grow from
 * hexes precracked by orc_presplit, whose mask argument then holds crack
 * plane indices 0-22 (0-2 mid-planes, 3-14 wedge planes, 15-22 corner
 * planes); split events report the plane in their mask column and the
 * pattern (3-6; 0 for a precrack); orc_front_G gives one row per candidate:
 * (hex, local face, plane) and (G, pattern). */
orc_ctx* orc_create_hex(int n_nodes, const double* X, int n_hex, const int* hex,
                        double E, double nu, double rho, double Gc, int gsig);
/* Cut-edge bit masks of the 23 hex crack planes. */
int orc_hex_plane_masks(int* out23);
int orc_create_status(const orc_ctx* c);
const char* orc_error(const orc_ctx* c);
void orc_destroy(orc_ctx* c);

int orc_set_traction(orc_ctx* c, int n_faces, const int* tri, const double* t,
                     double ramp_t0);
int orc_presplit(orc_ctx* c, int n, const int* tet, const unsigned char* mask);
int orc_critical_dt(orc_ctx* c, double* dt_crit);
int orc_set_dt(orc_ctx* c, double dt);
/* out: n_nodes_now, n_elems_now, n_edges_now, n_split, n_front */
int orc_counts(orc_ctx* c, int* out);
int orc_set_state(orc_ctx* c, const double* u, const double* v);
int orc_get_state(orc_ctx* c, double* u, double* v, double* a);
int orc_internal_force(orc_ctx* c, const double* u, double* f);
int orc_step(orc_ctx* c, int n_steps);
/* out[10]: step, t, KE, SE, Wext, Ud, Gmax, n_split, n_front, n_nodes */
int orc_energy(orc_ctx* c, double* out);
/* events: step, tet, side mask, pattern (1 = I, 2 = II, 0 = host pre-split) */
int orc_splits(orc_ctx* c, int cap, int* ev4, double* G, int* n_out);
/* current fronts sorted by (tet, face): tet, face, lone node; G_I, G_II */
int orc_front_G(orc_ctx* c, int cap, int* tfl3, double* g2, int* n_out);
/* forced split schedule (step, tet, mask), sorted by step then tet */
int orc_replay(orc_ctx* c, int n, const int* ev3);

/* Young's modulus per original tet (Pa); split copies use their parent's */
int orc_set_modulus(orc_ctx* c, const double* E_tet);
/* 1: steps skip the crack pass (fixed topology) */
int orc_set_frozen(orc_ctx* c, int on);
/* Threads of the element, edge and node loops (default 1).  Each thread owns
 * a contiguous range of elements, edges or nodes and every sum keeps the
 * serial order, so results are bitwise the same at any count. */
int orc_set_threads(orc_ctx* c, int n);
/* Runs n fixed-topology steps from the current state and returns the
 * sensitivities of J = gu . u_n + gv . v_n (either may be NULL = 0) to the
 * initial u and v ([n_nodes_now][3]) and to each tet's modulus ([n_tets]).
 * The state is left at the end of the window. */
int orc_window_gradient(orc_ctx* c, int n_steps, const double* gu, const double* gv,
                        double* gu0, double* gv0, double* gE);

/* Prescribed velocities, one group per call (before the first step): node[n],
 * dof mask (bit d = component d), v0[n][3]; velocity v0 t/t0 up to t0, then
 * v0 (t0 = 0: v0 from the start).  *group receives the group id. */
int orc_add_velocity_bc(orc_ctx* c, int n, const int* node, const int* mask,
                        const double* v0, double t0, int* group);
/* one row per step of a group: step, t, summed reaction (x, y, z), S(t);
 * work: the group's reactions' accumulated work */
int orc_reactions(orc_ctx* c, int group, int cap, double* rows6, int* n_out, double* work);

/* dSE/dE_j at fixed displacement (u = NULL: the current state): the explicit
 * part of the strain energy's sensitivity to each tet's modulus, [n_tets] */
int orc_strain_energy_grad(orc_ctx* c, const double* u, double* gE);

/* inspection */
int orc_masses(orc_ctx* c, double* m);
int orc_loads(orc_ctx* c, double* F);
int orc_elements(orc_ctx* c, int* nodes4, double* Veff, double* V, int* parent);
int orc_grad(orc_ctx* c, double* g12);
int orc_edges(orc_ctx* c, const double* u, int* nodes2, double* eps6, double* sig6);
int orc_elem_lambda_max(orc_ctx* c, double* lam);

/* stand-alone helpers */
void orc_lame(double E, double nu, double* lam, double* mu);
int orc_sym_eig3(const double* sig6, double* lam3, double* vec9);
double orc_stress_term(const double* sig6, const double* n, int gsig);
double orc_crack_area(const double* X4, int mask);

#ifdef __cplusplus
}
#endif
#endif
