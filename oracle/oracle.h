/*
 * Plain FP64 CPU oracle for one coupled step of the lattice-Boltzmann /
 * dynamic immersed-boundary method of Coclite, de Tullio, Pascazio and
 * Politi, "Characterization of micro-Capsules Deformation in Branching
 * Channels" (arXiv 2207.06043), Section "Numerical method and computational
 * procedure".
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the package smoke check and
 * the benchmark's CPU-baseline leg may load this library.  It shares no code
 * with the GPU library; both read the same synthetic inputs.
 *
 * Status codes use the same numbers as the GPU library's C interface.
 */
#ifndef ORACLE_H
#define ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_OK = 0, ORC_E_INVAL = 1, ORC_E_NOMEM = 2, ORC_E_UNSTABLE = 4,
       ORC_E_DAMAGED = 5, ORC_E_STATE = 6 };

typedef struct orc_sim orc_sim;

/* Lattice of nx*ny*nz nodes, linear index x + nx*(y + ny*z).
 * node_type: 0 fluid, 1 solid, 2 velocity inlet, 3 density outlet.
 * Wall links (node, dir, q): node + e_dir is solid, wall at fraction q.
 * inlet_u: 3 values per inlet node, inlet nodes in increasing index order.
 * init_rho [N] / init_u [3][N] may be NULL (rho = 1, u = 0).
 * body_force: uniform force density added to the immersed-boundary force. */
orc_sim *orc_create(int nx, int ny, int nz, const int32_t *periodic, double tau,
                    double u_max, const double *body_force, const uint8_t *node_type,
                    int64_t n_links, const int64_t *link_node, const uint8_t *link_dir,
                    const double *link_q, const double *inlet_u, double outlet_rho,
                    const double *init_rho, const double *init_u, char *err, int errlen);
void orc_destroy(orc_sim *s);
void orc_set_threads(int n);
int orc_threads(void);

/* Body: closed outward-oriented triangle mesh.  rigid/fixed flags; material
 * in the paper's terms (capillary number, bending number, volume penalty
 * kv (<= 0 -> 10*ks0/r_ref), density ratio, reference radius and velocity).
 * Returns the body id (>= 0) or -status. */
int orc_add_body(orc_sim *s, int nv, int nf, const double *x, const int32_t *faces,
                 int rigid, int fixed, double ca, double eb, double kv, double rho_ratio,
                 double r_ref, double u_ref, const double *v0);

int orc_step(orc_sim *s, int n_steps);
int64_t orc_steps_done(const orc_sim *s);
int orc_status(const orc_sim *s);
int orc_mls_singular_count(const orc_sim *s);

/* Outputs: rho [N], u [3][N] of the last step (solid nodes: 0); populations
 * [19][N] post-collision; force field [3][N] of the last step. */
void orc_get_fields(const orc_sim *s, double *rho, double *u);
void orc_get_populations(const orc_sim *s, double *f);
void orc_set_populations(orc_sim *s, const double *f);
void orc_get_populations_at(const orc_sim *s, long n, const long *nodes, double *f);
void orc_get_force(const orc_sim *s, double *fib);
void orc_get_body(const orc_sim *s, int id, double *x, double *v);
/* V, S, V0, S0, max l/l0, mass, kv, ks0, centre (3), rigid u (3),
 * omega (3), vertex mass, rigid flag, face count */
void orc_body_diag(const orc_sim *s, int id, double *out20);

/* Interface operators (section on moving immersed boundaries):
 * interpolation of a [3][N] field at n points and spreading of c*F. */
void orc_ib_interpolate(const orc_sim *s, int64_t n, const double *pts, const double *field,
                        double *out);
void orc_ib_spread(const orc_sim *s, int64_t n, const double *pts, const double *F,
                   const double *c, double *fib);
/* MLS stencil of one point: node index (-1 excluded) and 4 coefficient
 * weights per node (value, d/dx, d/dy, d/dz). Returns 0 if singular. */
int orc_mls_point(const orc_sim *s, const double *p, int64_t *node27, double *psi27x4);

/* Element helpers used by the pins. */
void orc_lattice(int32_t *e57, double *w19);
void orc_feq(double rho, const double *u, double *out19);
void orc_guo(double tau, const double *u, const double *F, double *out19);
double orc_bfl(double q, double fi_x, double fi_xm1, double fi_xm2, double fj_x,
               double fj_xm1, int avail1, int avail2);
double orc_zouhe(double *f19, int face, int kind, const double *u_w, double rho_w);
/* Internal membrane forces on body id for arbitrary vertex positions x:
 * which = 1 stretching, 2 bending, 4 volume (bit mask).  Returns the energy. */
double orc_membrane(const orc_sim *s, int id, const double *x, int which, double *F);
/* Hydrodynamic force per face (nf*3) of body id from the current rho, u. */
void orc_body_hydro(const orc_sim *s, int id, double *Fface);
/* External force per face (nf*3) of body id used by the last completed step:
 * the hydrodynamic force plus the inter-body repulsion. */
void orc_body_fext(const orc_sim *s, int id, double *Fface);

/* Pins of the rigid-body update: the body-frame inertia tensor (about the
 * centre of mass, orientation at creation) of body id; the rotation matrix
 * of a rotation vector (Rodrigues); one rigid-body update of body id with
 * given vertex forces [nv*3] in place of the step's external forces
 * (ORC_E_INVAL for a soft body). */
void orc_body_inertia(const orc_sim *s, int id, double *I9);
void orc_rodrigues(const double *phi, double *R9);
int orc_move_rigid(orc_sim *s, int id, const double *Fv);

#ifdef __cplusplus
}
#endif
#endif
