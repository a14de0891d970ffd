/*
 * Plain FP64 CPU oracle for the coupled lattice-Boltzmann / dynamic
 * immersed-boundary step of Coclite, de Tullio, Pascazio and Politi,
 * "Characterization of micro-Capsules Deformation in Branching Channels"
 * (arXiv 2207.06043).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the package smoke check and
 * the benchmark's CPU-baseline leg, never by the product path.  It shares no
 * code, header, table or helper with the GPU library.
 *
 * The step follows the paper's order and notation, in plain loops over
 * nodes in x-fastest order and over bodies/faces/vertices in index order:
 *   S1 pull-streaming, with interpolated bounce-back on wall links
 *      (section "No-slip boundary conditions for stationary immersed
 *      boundaries", Eq. bbouzidi);
 *   S2 Zou-He velocity/density Dirichlet nodes on open faces (section
 *      "Dirichlet conditions for external boundaries", Eq. extbound, written
 *      for a general face normal);
 *   S3 moments (section "Fluid evolution");
 *   S4 dynamic-IB direct forcing with moving-least-squares transfer
 *      (section "No-slip conditions for moving immersed boundaries",
 *      Eqs. uLag, l2norm, intKernel, the direct-forcing equation, bodyforce);
 *   S5 BGK collision with the forcing term (Eqs. evoleq, eqfunc, forcing);
 *   S6 membrane forces (Eqs. strainPot/strainFor, bendPot/bendFor, volFor),
 *      repulsion (Eq. collision);
 *   S7 hydrodynamic tractions (Eqs. hydroForP, hydroForNu);
 *   S8 motion: Verlet with tentative velocity for soft bodies (Eqs.
 *      newtonSoft, verletPos, verletVel, verletPosC) and the second-order
 *      backward update of the Newton-Euler system for rigid bodies
 *      (Eq. angularVelRig).
 * Where the paper is silent or garbled, the reading taken is stated at the
 * point of use.
 *
 * Storage: populations are kept as deviations d_i = f_i - w_i from the rest
 * weights.  This is an exact change of variables: streaming, the
 * interpolated bounce-back (its coefficients add up to 1 and link directions
 * of equal weight) and the Zou-He rule map deviations to deviations, and the
 * moments are rho = 1 + sum d, rho u = sum d e.  Full populations (about
 * 1/3) lose about 3e-17 to rounding at every store; in a steady flow that
 * loss has the same sign step after step and adds up to about 1e-12 of the
 * velocity scale within a few thousand steps, which the deviations (about
 * 1e-3) avoid.
 */
#include "oracle.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { T_FLUID = 0, T_SOLID = 1, T_INLET = 2, T_OUTLET = 3 };

/* Type of the fluid state and arithmetic (populations, moments, collision).
 * double in the oracle; the measurement build ORC_LDOUBLE makes it long
 * double (64-bit significand) to give a near-exact trajectory against which
 * the rounding of the double builds is measured. */
#if defined(ORC_LDOUBLE)
typedef long double preal;
#define PR(x) x##L
#elif defined(ORC_FLOAT)
/* measurement build only: the fluid state and arithmetic in binary32, to
 * gauge how far FP32 arithmetic (not only FP32 storage) moves a trajectory */
typedef float preal;
#define PR(x) x##f
#else
typedef double preal;
#define PR(x) x
#endif

/* D3Q19 velocity set in the column order printed in the "Fluid evolution"
 * section (Eq. e_i); weights 1/3, 1/18 (axis), 1/36 (diagonal) from the text
 * following Eq. eqfunc. */
static const int E[19][3] = {
    {0, 0, 0},   {1, 0, 0},  {-1, 0, 0}, {0, 1, 0},  {0, -1, 0}, {0, 0, 1},  {0, 0, -1},
    {1, 1, 0},   {1, -1, 0}, {1, 0, 1},  {1, 0, -1}, {-1, 1, 0}, {-1, -1, 0}, {-1, 0, 1},
    {-1, 0, -1}, {0, 1, 1},  {0, 1, -1}, {0, -1, 1}, {0, -1, -1}};
static const preal Wt[19] = {PR(1.0) / 3,  PR(1.0) / 18, PR(1.0) / 18, PR(1.0) / 18, PR(1.0) / 18,
                             PR(1.0) / 18, PR(1.0) / 18, PR(1.0) / 36, PR(1.0) / 36, PR(1.0) / 36,
                             PR(1.0) / 36, PR(1.0) / 36, PR(1.0) / 36, PR(1.0) / 36, PR(1.0) / 36,
                             PR(1.0) / 36, PR(1.0) / 36, PR(1.0) / 36, PR(1.0) / 36};
static const double CS2 = 1.0 / 3.0; /* c_s^2, c_s = 1/sqrt(3) */
static const preal CS2P = PR(1.0) / PR(3.0);

/* Opposite direction: the one whose vector is -e_i (found by search). */
static int opposite_search(int i) {
  for (int k = 0; k < 19; k++)
    if (E[k][0] == -E[i][0] && E[k][1] == -E[i][1] && E[k][2] == -E[i][2]) return k;
  return -1;
}
static int OPP[19] = {-1};
static int opposite(int i) {
  if (OPP[0] < 0)
    for (int k = 0; k < 19; k++) OPP[k] = opposite_search(k);
  return OPP[i];
}

/* ------------------------------------------------------------------ types */
typedef struct {
  int nv, nf, ne, nh;
  int rigid, fixed;
  double *x, *xprev, *v;   /* [nv*3]: x^n, x^{n-1}, u_v^n */
  int *faces;              /* [nf*3] outward CCW */
  int *edges;              /* [ne*2] */
  double *l0, *kl;         /* rest length, stiffness per edge */
  int *hinge;              /* [nh*4]: a, b shared edge (as a->b in face 1), c wing of face 1, d wing of face 2 */
  double *theta0, *kb;     /* rest dihedral angle, bending stiffness per hinge */
  double *Fext;            /* [nf*3] hydrodynamic + repulsion force per face of the last step */
  double V0, S0, ks0, kv, eb, rho_ratio, r_ref, u_ref, m_v, mass;
  /* rigid state */
  double xc[3], u[3], uprev[3], w[3], wprev[3], R[9], Ibody[9];
  double *X;               /* body-frame vertex offsets [nv*3] */
  double V, S, max_strain;
} body_t;

struct orc_sim {
  int nx, ny, nz, per[3];
  long N;
  double tau, nu, umax, g[3];
  unsigned char *type;
  long *lk_start;          /* CSR over nodes */
  unsigned char *lk_dir;
  double *lk_q;
  double *uin;             /* [N*3], inlet nodes only */
  double rho_out;
  preal *fs;               /* post-collision populations, as f - w [N*19] (the state) */
  preal *f;                /* streamed populations, as f - w [N*19] (work) */
  preal *rho;              /* density of the last step [N] */
  double *u;               /* velocity of the last step [N*3] */
  preal *mom;              /* pre-collision momentum sum_i f_i e_i [N*3] */
  double *ustar;           /* pre-force velocity m/rho [N*3] */
  double *fib;             /* immersed-boundary force density [N*3] */
  int nbody;
  body_t *bodies;
  long steps_done;
  int status;
  int mls_singular;
};

static int g_threads = 0;
void orc_set_threads(int n) { g_threads = n; }
int orc_threads(void) {
#ifdef _OPENMP
  return g_threads > 0 ? g_threads : omp_get_max_threads();
#else
  return 1;
#endif
}

/* ------------------------------------------------------- small vector ops */
static void cross(const double *a, const double *b, double *c) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}
static double dot(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static double norm(const double *a) { return sqrt(dot(a, a)); }
static void sub(const double *a, const double *b, double *c) {
  c[0] = a[0] - b[0]; c[1] = a[1] - b[1]; c[2] = a[2] - b[2];
}

/* ------------------------------------------------------- lattice helpers */
static void coords(const orc_sim *s, long n, int *x, int *y, int *z) {
  *x = (int)(n % s->nx);
  *y = (int)((n / s->nx) % s->ny);
  *z = (int)(n / ((long)s->nx * s->ny));
}

/* Node at (x,y,z)+(dx,dy,dz): wrapped on periodic axes, -1 if it leaves the
 * box through a non-periodic face. */
static long neighbour(const orc_sim *s, int x, int y, int z, int dx, int dy, int dz) {
  int c[3] = {x + dx, y + dy, z + dz};
  int n[3] = {s->nx, s->ny, s->nz};
  for (int a = 0; a < 3; a++) {
    if (c[a] < 0 || c[a] >= n[a]) {
      if (!s->per[a]) return -1;
      c[a] = ((c[a] % n[a]) + n[a]) % n[a];
    }
  }
  return c[0] + (long)s->nx * (c[1] + (long)s->ny * c[2]);
}

static double find_q(const orc_sim *s, long n, int dir) {
  for (long k = s->lk_start[n]; k < s->lk_start[n + 1]; k++)
    if (s->lk_dir[k] == dir) return s->lk_q[k];
  return -1.0;
}

/* Eq. eqfunc: second-order expansion of the Maxwell-Boltzmann distribution. */
static preal feq_i(int i, preal rho, const preal *u) {
  preal eu = E[i][0] * u[0] + E[i][1] * u[1] + E[i][2] * u[2];
  preal uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  return Wt[i] * rho * (PR(1.0) + eu / CS2P + eu * eu / (PR(2.0) * CS2P * CS2P) - uu / (PR(2.0) * CS2P));
}

/* f^eq_i - w_i, the same expansion written as a deviation from the rest
 * weights (the form the populations are stored in, below). */
__attribute__((unused)) static preal feq_dev_i(int i, preal rho, const preal *u) {
  preal eu = E[i][0] * u[0] + E[i][1] * u[1] + E[i][2] * u[2];
  preal uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  return Wt[i] * ((rho - PR(1.0)) + rho * (eu / CS2P + eu * eu / (PR(2.0) * CS2P * CS2P) - uu / (PR(2.0) * CS2P)));
}

/* The stored form of the equilibrium: deviations f^eq - w (full
 * populations in the measurement build ORC_FULL_POP). */
static preal feq_store_i(int i, preal rho, const preal *u) {
#ifdef ORC_FULL_POP
  return feq_i(i, rho, u);
#else
  return feq_dev_i(i, rho, u);
#endif
}

/* Eq. forcing: the discrete forcing term projected on direction i. */
static preal guo_i(int i, preal tau, const preal *u, const preal *F) {
  preal eu = E[i][0] * u[0] + E[i][1] * u[1] + E[i][2] * u[2];
  preal acc = PR(0.0);
  for (int a = 0; a < 3; a++) acc += ((E[i][a] - u[a]) / CS2P + eu * E[i][a] / (CS2P * CS2P)) * F[a];
  return (PR(1.0) - PR(1.0) / (PR(2.0) * tau)) * Wt[i] * acc;
}

void orc_lattice(int32_t *e57, double *w19) {
  for (int i = 0; i < 19; i++) {
    for (int a = 0; a < 3; a++) e57[3 * i + a] = E[i][a];
    w19[i] = (double)Wt[i];
  }
}
void orc_feq(double rho, const double *u, double *out19) {
  preal up[3] = {u[0], u[1], u[2]};
  for (int i = 0; i < 19; i++) out19[i] = (double)feq_i(i, rho, up);
}
void orc_guo(double tau, const double *u, const double *F, double *out19) {
  preal up[3] = {u[0], u[1], u[2]}, Fp[3] = {F[0], F[1], F[2]};
  for (int i = 0; i < 19; i++) out19[i] = (double)guo_i(i, tau, up, Fp);
}

/* Eq. bbouzidi: interpolated bounce-back for the population j = opposite(i)
 * entering a wall node x whose link i meets the wall at fraction q.
 * fi_x = f*_i(x), fi_xm1 = f*_i(x - e_i), fi_xm2 = f*_i(x - 2e_i),
 * fj_x = f*_j(x), fj_xm1 = f*_j(x - e_i) (post-collision values).
 * Reading of the q >= 1/2 branch: the printed 2nd and 3rd terms carry f_i;
 * they are taken on the opposite population, which makes the rule the
 * quadratic interpolation through the bounced particle at distance 2q-1 and
 * the two opposite populations behind x, as in the q < 1/2 branch.
 * Reading where the paper is silent (x - e_i or x - 2e_i solid or outside):
 * drop to the linear interpolation through the points that remain, and to
 * the plain bounce-back f*_i(x) when none remains (q < 1/2).
 * Every branch's coefficients add up to 1, so the rule applies unchanged to
 * deviations f - w (w_i = w_j for a link and its opposite). */
static preal bfl(preal q, preal fi_x, preal fi_xm1, preal fi_xm2, preal fj_x, preal fj_xm1,
                 int avail1, int avail2) {
  if (q < PR(0.5)) {
    if (avail1 && avail2)
      return q * (PR(1.0) + PR(2.0) * q) * fi_x + (PR(1.0) - PR(4.0) * q * q) * fi_xm1 -
             q * (PR(1.0) - PR(2.0) * q) * fi_xm2;
    if (avail1) return PR(2.0) * q * fi_x + (PR(1.0) - PR(2.0) * q) * fi_xm1;
    return fi_x;
  }
  if (avail1)
    return fi_x / (q * (PR(2.0) * q + PR(1.0))) + (PR(2.0) * q - PR(1.0)) / q * fj_x +
           (PR(1.0) - PR(2.0) * q) / (PR(1.0) + PR(2.0) * q) * fj_xm1;
  return fi_x / (PR(2.0) * q) + (PR(2.0) * q - PR(1.0)) / (PR(2.0) * q) * fj_x;
}

double orc_bfl(double q, double fi_x, double fi_xm1, double fi_xm2, double fj_x,
               double fj_xm1, int avail1, int avail2) {
  return (double)bfl(q, fi_x, fi_xm1, fi_xm2, fj_x, fj_xm1, avail1, avail2);
}

/* Inward unit normal of box face: 0 x=0, 1 x=nx-1, 2 y=0, 3 y=ny-1, 4 z=0, 5 z=nz-1. */
static void face_normal(int face, int *n) {
  n[0] = n[1] = n[2] = 0;
  n[face / 2] = (face % 2 == 0) ? 1 : -1;
}

/* Eq. extbound (Zou-He) written for a general face with inward normal n:
 * the five populations with e.n = +1 are unknown.  kind 0: velocity face
 * (u_w imposed), kind 1: density face (rho_w imposed, tangential velocity
 * zero).  Readings: the printed block is indexed in a different D3Q19 order
 * than Eq. e_i, so it is applied through direction vectors; its 1/6 terms
 * carry the wall density rho_w, which the momentum balance requires.
 * Fills the unknowns of f19 in place and returns rho_w. */
static preal zouhe_dev(preal *d, int face, int kind, const double *u_w_in, preal rho_w) {
  int n[3];
  face_normal(face, n);
  /* with d = f - w: sum_{e.n=0} f + 2 sum_{e.n=-1} f = 1 + D0 + 2 Dout, since
   * the rest weights of those sets add up to 2/3 and 1/6 (in the
   * measurement build ORC_FULL_POP, d holds f itself and the 1 is dropped) */
#ifdef ORC_FULL_POP
  const preal one = PR(0.0);
#else
  const preal one = PR(1.0);
#endif
  preal D0 = PR(0.0), Dout = PR(0.0);
  for (int j = 0; j < 19; j++) {
    int en = E[j][0] * n[0] + E[j][1] * n[1] + E[j][2] * n[2];
    if (en == 0) D0 += d[j];
    else if (en == -1) Dout += d[j];
  }
  preal uw[3];
  if (kind == 0) {
    for (int a = 0; a < 3; a++) uw[a] = u_w_in[a];
    preal un = uw[0] * n[0] + uw[1] * n[1] + uw[2] * n[2];
    rho_w = (one + D0 + PR(2.0) * Dout) / (PR(1.0) - un);
  } else {
    preal un = (rho_w - one - D0 - PR(2.0) * Dout) / rho_w;
    for (int a = 0; a < 3; a++) uw[a] = un * n[a];
  }
  preal un = uw[0] * n[0] + uw[1] * n[1] + uw[2] * n[2];
  for (int j = 0; j < 19; j++) {
    int en = E[j][0] * n[0] + E[j][1] * n[1] + E[j][2] * n[2];
    if (en != 1) continue;
    int jb = opposite(j);
    int t[3] = {E[j][0] - n[0], E[j][1] - n[1], E[j][2] - n[2]};
    if (t[0] == 0 && t[1] == 0 && t[2] == 0) {
      d[j] = d[jb] + rho_w / PR(3.0) * un;
    } else {
      preal ut = uw[0] * t[0] + uw[1] * t[1] + uw[2] * t[2];
      /* the rest weights cancel in this sum (symmetric pairs) */
      preal Nt = PR(0.0);
      for (int k = 0; k < 19; k++) {
        int ek = E[k][0] * n[0] + E[k][1] * n[1] + E[k][2] * n[2];
        if (ek == 0) Nt += d[k] * (E[k][0] * t[0] + E[k][1] * t[1] + E[k][2] * t[2]);
      }
      Nt = PR(0.5) * Nt - rho_w / PR(3.0) * ut;
      d[j] = d[jb] + rho_w / PR(6.0) * (un + ut) - Nt;
    }
  }
  return rho_w;
}

/* The same condition on full populations f (public entry, plain build). */
double orc_zouhe(double *f, int face, int kind, const double *u_w_in, double rho_w) {
  preal d[19];
#ifdef ORC_FULL_POP
  for (int j = 0; j < 19; j++) d[j] = f[j];
#else
  for (int j = 0; j < 19; j++) d[j] = f[j] - Wt[j];
#endif
  double r = (double)zouhe_dev(d, face, kind, u_w_in, rho_w);
#ifdef ORC_FULL_POP
  for (int j = 0; j < 19; j++) f[j] = (double)d[j];
#else
  for (int j = 0; j < 19; j++) f[j] = (double)(Wt[j] + d[j]);
#endif
  return r;
}

/* Box face on which an open node lies (the face whose outside its unknown
 * populations come from); -1 if none. */
static int open_face(const orc_sim *s, long n) {
  int x, y, z;
  coords(s, n, &x, &y, &z);
  int c[3] = {x, y, z}, dim[3] = {s->nx, s->ny, s->nz};
  for (int a = 0; a < 3; a++) {
    if (s->per[a]) continue;
    if (c[a] == 0) return 2 * a;
    if (c[a] == dim[a] - 1) return 2 * a + 1;
  }
  return -1;
}

/* ------------------------------------------------------------- creation */
static void set_err(char *err, int len, const char *msg) {
  if (err && len > 0) {
    strncpy(err, msg, (size_t)len - 1);
    err[len - 1] = 0;
  }
}

orc_sim *orc_create(int nx, int ny, int nz, const int32_t *periodic, double tau, double u_max,
                    const double *body_force, const uint8_t *node_type, int64_t n_links,
                    const int64_t *link_node, const uint8_t *link_dir, const double *link_q,
                    const double *inlet_u, double outlet_rho, const double *init_rho,
                    const double *init_u, char *err, int errlen) {
  char msg[256];
  if (nx < 1 || ny < 1 || nz < 1 || !(tau > 0.5) || !node_type) {
    set_err(err, errlen, "bad sizes or tau <= 1/2");
    return NULL;
  }
  (void)opposite(0);
  orc_sim *s = (orc_sim *)calloc(1, sizeof(orc_sim));
  s->nx = nx; s->ny = ny; s->nz = nz;
  for (int a = 0; a < 3; a++) s->per[a] = periodic ? periodic[a] != 0 : 0;
  s->N = (long)nx * ny * nz;
  s->tau = tau;
  s->nu = CS2 * (tau - 0.5); /* nu = c_s^2 (tau - dt/2) */
  s->umax = u_max;
  for (int a = 0; a < 3; a++) s->g[a] = body_force ? body_force[a] : 0.0;
  s->rho_out = outlet_rho;
  long N = s->N;
  s->type = (unsigned char *)malloc(N);
  memcpy(s->type, node_type, N);
  s->lk_start = (long *)calloc(N + 1, sizeof(long));
  s->lk_dir = (unsigned char *)malloc(n_links > 0 ? n_links : 1);
  s->lk_q = (double *)malloc(sizeof(double) * (n_links > 0 ? n_links : 1));
  s->uin = (double *)calloc(N * 3, sizeof(double));
  s->fs = (preal *)malloc(sizeof(preal) * N * 19);
  s->f = (preal *)malloc(sizeof(preal) * N * 19);
  s->rho = (preal *)calloc(N, sizeof(preal));
  s->u = (double *)calloc(N * 3, sizeof(double));
  s->mom = (preal *)calloc(N * 3, sizeof(preal));
  s->ustar = (double *)calloc(N * 3, sizeof(double));
  s->fib = (double *)calloc(N * 3, sizeof(double));
  if (!s->fs || !s->f || !s->rho || !s->u || !s->ustar || !s->fib || !s->mom) {
    set_err(err, errlen, "out of memory");
    orc_destroy(s);
    return NULL;
  }
  for (long n = 0; n < N; n++)
    if (s->type[n] > 3) { set_err(err, errlen, "bad node type"); orc_destroy(s); return NULL; }
  /* links: counting sort by node, keeping the input order within a node */
  for (long k = 0; k < n_links; k++) {
    long n = link_node[k];
    if (n < 0 || n >= N || link_dir[k] < 1 || link_dir[k] > 18 || !(link_q[k] >= 0.0) ||
        !(link_q[k] <= 1.0) || s->type[n] == T_SOLID) {
      snprintf(msg, sizeof msg, "bad wall link %ld", k);
      set_err(err, errlen, msg); orc_destroy(s); return NULL;
    }
    int x, y, z;
    coords(s, n, &x, &y, &z);
    int d = link_dir[k];
    long nb = neighbour(s, x, y, z, E[d][0], E[d][1], E[d][2]);
    if (nb < 0 || s->type[nb] != T_SOLID) {
      snprintf(msg, sizeof msg, "wall link %ld does not point at a solid node", k);
      set_err(err, errlen, msg); orc_destroy(s); return NULL;
    }
    s->lk_start[n + 1]++;
  }
  for (long n = 0; n < N; n++) s->lk_start[n + 1] += s->lk_start[n];
  {
    long *fill = (long *)calloc(N, sizeof(long));
    for (long k = 0; k < n_links; k++) {
      long n = link_node[k];
      long at = s->lk_start[n] + fill[n]++;
      s->lk_dir[at] = link_dir[k];
      s->lk_q[at] = link_q[k];
    }
    free(fill);
  }
  /* every non-solid node: solid neighbours need a link, outside sources need an open face */
  long n_in = 0;
  for (long n = 0; n < N; n++) {
    if (s->type[n] == T_SOLID) continue;
    int x, y, z;
    coords(s, n, &x, &y, &z);
    int outside = 0;
    for (int i = 1; i < 19; i++) {
      long nb = neighbour(s, x, y, z, E[i][0], E[i][1], E[i][2]);
      if (nb < 0) outside = 1;
      else if (s->type[nb] == T_SOLID && find_q(s, n, i) < 0.0) {
        snprintf(msg, sizeof msg, "node %ld has a solid neighbour in direction %d without a wall link", n, i);
        set_err(err, errlen, msg); orc_destroy(s); return NULL;
      }
    }
    int open = s->type[n] == T_INLET || s->type[n] == T_OUTLET;
    if (outside && !open) {
      snprintf(msg, sizeof msg, "fluid node %ld on a closed box face", n);
      set_err(err, errlen, msg); orc_destroy(s); return NULL;
    }
    if (open) {
      int nfaces = 0, dim[3] = {nx, ny, nz}, c[3] = {x, y, z};
      for (int a = 0; a < 3; a++)
        if (!s->per[a] && (c[a] == 0 || c[a] == dim[a] - 1)) nfaces += (dim[a] == 1) ? 2 : 1;
      if (nfaces != 1) {
        snprintf(msg, sizeof msg, "open node %ld must lie on exactly one non-periodic face", n);
        set_err(err, errlen, msg); orc_destroy(s); return NULL;
      }
    }
    if (s->type[n] == T_INLET) {
      for (int a = 0; a < 3; a++) s->uin[3 * n + a] = inlet_u ? inlet_u[3 * n_in + a] : 0.0;
      n_in++;
    }
  }
  /* initial state: f = f^eq(rho0, u0) on non-solid nodes (stored as f - w) */
  for (long n = 0; n < N; n++) {
    preal r = init_rho ? init_rho[n] : 1.0;
    preal uu[3] = {0, 0, 0};
    if (init_u)
      for (int a = 0; a < 3; a++) uu[a] = init_u[(long)a * N + n];
    if (s->type[n] == T_SOLID) {
      for (int i = 0; i < 19; i++) s->fs[19 * n + i] = 0.0;
      continue;
    }
    for (int i = 0; i < 19; i++) s->fs[19 * n + i] = feq_store_i(i, r, uu);
    s->rho[n] = r;
    for (int a = 0; a < 3; a++) s->u[3 * n + a] = (double)uu[a];
  }
  return s;
}

static void free_body(body_t *b) {
  free(b->x); free(b->xprev); free(b->v); free(b->faces); free(b->edges); free(b->l0);
  free(b->kl); free(b->hinge); free(b->theta0); free(b->kb); free(b->Fext); free(b->X);
}

void orc_destroy(orc_sim *s) {
  if (!s) return;
  free(s->type); free(s->lk_start); free(s->lk_dir); free(s->lk_q); free(s->uin);
  free(s->fs); free(s->f); free(s->rho); free(s->u); free(s->mom); free(s->ustar); free(s->fib);
  for (int b = 0; b < s->nbody; b++) free_body(&s->bodies[b]);
  free(s->bodies);
  free(s);
}

/* ------------------------------------------------------------ mesh geometry */
static void face_geom(const double *x, const int *f, double *centroid, double *nhat, double *area) {
  const double *a = x + 3 * f[0], *b = x + 3 * f[1], *c = x + 3 * f[2];
  double ab[3], ac[3], N[3];
  sub(b, a, ab);
  sub(c, a, ac);
  cross(ab, ac, N);
  double l = norm(N);
  for (int k = 0; k < 3; k++) {
    centroid[k] = (a[k] + b[k] + c[k]) / 3.0;
    nhat[k] = N[k] / l;
  }
  *area = 0.5 * l;
}

/* Enclosed volume of the closed mesh, sum over faces of a.(b x c)/6. */
static double mesh_volume(const double *x, const int *faces, int nf) {
  double V = 0.0;
  for (int f = 0; f < nf; f++) {
    const double *a = x + 3 * faces[3 * f], *b = x + 3 * faces[3 * f + 1], *c = x + 3 * faces[3 * f + 2];
    double bc[3];
    cross(b, c, bc);
    V += dot(a, bc) / 6.0;
  }
  return V;
}

static double mesh_area(const double *x, const int *faces, int nf) {
  double S = 0.0, c[3], n[3], A;
  for (int f = 0; f < nf; f++) {
    face_geom(x, faces + 3 * f, c, n, &A);
    S += A;
  }
  return S;
}

/* Signed dihedral angle of hinge (a, b, c, d): angle between the outward
 * normals of faces (a, b, c) and (b, a, d), positive for a convex fold. */
static double dihedral(const double *x, const int *h, double *n1, double *n2) {
  const double *a = x + 3 * h[0], *b = x + 3 * h[1], *c = x + 3 * h[2], *d = x + 3 * h[3];
  double e[3], ac[3], ab[3], bd[3], t[3];
  sub(b, a, e);
  sub(c, a, ac);
  cross(e, ac, n1);
  sub(a, b, ab);
  sub(d, b, bd);
  cross(ab, bd, n2);
  double l1 = norm(n1), l2 = norm(n2), le = norm(e);
  double m1[3], m2[3];
  for (int k = 0; k < 3; k++) { m1[k] = n1[k] / l1; m2[k] = n2[k] / l2; }
  cross(m1, m2, t);
  return atan2(dot(t, e) / le, dot(m1, m2));
}

int orc_add_body(orc_sim *s, int nv, int nf, const double *x, const int32_t *faces, int rigid,
                 int fixed, double ca, double eb, double kv, double rho_ratio, double r_ref,
                 double u_ref, const double *v0) {
  if (!s || nv < 4 || nf < 4 || !x || !faces) return -ORC_E_INVAL;
  for (int k = 0; k < 3 * nf; k++)
    if (faces[k] < 0 || faces[k] >= nv) return -ORC_E_INVAL;
  /* edges and hinges from the faces: every edge must be shared by exactly two
   * faces with opposite orientation (closed, consistently oriented mesh) */
  int maxe = 3 * nf;
  int *ea = (int *)malloc(sizeof(int) * maxe), *eb_ = (int *)malloc(sizeof(int) * maxe);
  int *ef1 = (int *)malloc(sizeof(int) * maxe), *ef2 = (int *)malloc(sizeof(int) * maxe);
  int ne = 0;
  for (int f = 0; f < nf; f++) {
    for (int k = 0; k < 3; k++) {
      int a = faces[3 * f + k], b = faces[3 * f + (k + 1) % 3];
      int found = -1;
      for (int e = 0; e < ne; e++)
        if (ea[e] == b && eb_[e] == a) { found = e; break; }
      if (found >= 0) {
        if (ef2[found] >= 0) { free(ea); free(eb_); free(ef1); free(ef2); return -ORC_E_INVAL; }
        ef2[found] = f;
      } else {
        for (int e = 0; e < ne; e++)
          if (ea[e] == a && eb_[e] == b) { free(ea); free(eb_); free(ef1); free(ef2); return -ORC_E_INVAL; }
        ea[ne] = a; eb_[ne] = b; ef1[ne] = f; ef2[ne] = -1; ne++;
      }
    }
  }
  for (int e = 0; e < ne; e++)
    if (ef2[e] < 0) { free(ea); free(eb_); free(ef1); free(ef2); return -ORC_E_INVAL; }

  s->bodies = (body_t *)realloc(s->bodies, sizeof(body_t) * (s->nbody + 1));
  body_t *B = &s->bodies[s->nbody];
  memset(B, 0, sizeof(*B));
  B->nv = nv; B->nf = nf; B->ne = ne; B->nh = ne;
  B->rigid = rigid || fixed; B->fixed = fixed;
  B->x = (double *)malloc(sizeof(double) * 3 * nv);
  B->xprev = (double *)malloc(sizeof(double) * 3 * nv);
  B->v = (double *)calloc(3 * nv, sizeof(double));
  B->X = (double *)malloc(sizeof(double) * 3 * nv);
  B->faces = (int *)malloc(sizeof(int) * 3 * nf);
  B->edges = (int *)malloc(sizeof(int) * 2 * ne);
  B->l0 = (double *)malloc(sizeof(double) * ne);
  B->kl = (double *)malloc(sizeof(double) * ne);
  B->hinge = (int *)malloc(sizeof(int) * 4 * ne);
  B->theta0 = (double *)malloc(sizeof(double) * ne);
  B->kb = (double *)malloc(sizeof(double) * ne);
  B->Fext = (double *)calloc(3 * nf, sizeof(double));
  memcpy(B->x, x, sizeof(double) * 3 * nv);
  for (int k = 0; k < 3 * nf; k++) B->faces[k] = faces[k];
  if (v0 && !fixed) memcpy(B->v, v0, sizeof(double) * 3 * nv);
  /* history consistent with the initial velocity: x^{-1} = x^0 - u^0 dt */
  for (int k = 0; k < 3 * nv; k++) B->xprev[k] = x[k] - B->v[k];

  B->V0 = mesh_volume(x, B->faces, nf);
  B->S0 = mesh_area(x, B->faces, nf);
  B->V = B->V0;
  B->S = B->S0;
  B->eb = eb;
  B->rho_ratio = rho_ratio;
  B->r_ref = r_ref;
  B->u_ref = u_ref;
  /* Capillary number Ca = rho nu u_ref / k_s0 with rho = 1 ("Deforming
   * bodies constitutive model"). */
  B->ks0 = (ca > 0.0) ? s->nu * u_ref / ca : 0.0;
  /* Volume-penalty constant: not given in the paper; default 10 k_s0 / r. */
  B->kv = (kv > 0.0) ? kv : 10.0 * B->ks0 / r_ref;
  /* Mass uniformly spread over the vertices: m = (rho_s/rho_f) V0, rho_f = 1. */
  B->mass = rho_ratio * B->V0;
  B->m_v = B->mass / nv;

  /* per-edge stiffness k_s,l = k_s0 T (A1 + A2) / l^2 with thickness T = 1
   * and the rest length and rest areas of the two faces sharing the edge */
  for (int e = 0; e < ne; e++) {
    double c[3], n[3], A1, A2, d[3];
    face_geom(x, B->faces + 3 * ef1[e], c, n, &A1);
    face_geom(x, B->faces + 3 * ef2[e], c, n, &A2);
    B->edges[2 * e] = ea[e];
    B->edges[2 * e + 1] = eb_[e];
    sub(x + 3 * ea[e], x + 3 * eb_[e], d);
    B->l0[e] = norm(d);
    B->kl[e] = B->ks0 * 1.0 * (A1 + A2) / (B->l0[e] * B->l0[e]);
    /* hinge: a->b is the edge as it runs in face 1; c the third vertex of face 1,
     * d the third vertex of face 2 */
    int *h = B->hinge + 4 * e;
    h[0] = ea[e];
    h[1] = eb_[e];
    for (int k = 0; k < 3; k++) {
      int v = B->faces[3 * ef1[e] + k];
      if (v != ea[e] && v != eb_[e]) h[2] = v;
      v = B->faces[3 * ef2[e] + k];
      if (v != ea[e] && v != eb_[e]) h[3] = v;
    }
    double n1[3], n2[3];
    B->theta0[e] = dihedral(x, h, n1, n2);
    /* Eb = k_b / (k_s,l r^2) with r the capsule radius */
    B->kb[e] = eb * B->kl[e] * r_ref * r_ref;
  }
  free(ea); free(eb_); free(ef1); free(ef2);

  /* rigid bodies: centre of mass and inertia tensor of the uniform solid
   * enclosed by the rest mesh (tetrahedra against the origin) */
  {
    double vol = 0.0, cm[3] = {0, 0, 0}, C[9] = {0};
    for (int f = 0; f < nf; f++) {
      const double *P[3] = {x + 3 * B->faces[3 * f], x + 3 * B->faces[3 * f + 1], x + 3 * B->faces[3 * f + 2]};
      double bc[3];
      cross(P[1], P[2], bc);
      double vt = dot(P[0], bc) / 6.0;
      vol += vt;
      for (int a = 0; a < 3; a++) cm[a] += vt * (P[0][a] + P[1][a] + P[2][a]) / 4.0;
      for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
          double sp = 0.0, si = 0.0, sj = 0.0;
          for (int k = 0; k < 3; k++) { sp += P[k][i] * P[k][j]; si += P[k][i]; sj += P[k][j]; }
          C[3 * i + j] += vt / 20.0 * (sp + si * sj);
        }
    }
    for (int a = 0; a < 3; a++) cm[a] /= vol;
    for (int i = 0; i < 3; i++)
      for (int j = 0; j < 3; j++) C[3 * i + j] -= vol * cm[i] * cm[j];
    double tr = C[0] + C[4] + C[8];
    for (int i = 0; i < 3; i++)
      for (int j = 0; j < 3; j++) B->Ibody[3 * i + j] = rho_ratio * ((i == j ? tr : 0.0) - C[3 * i + j]);
    for (int a = 0; a < 3; a++) B->xc[a] = cm[a];
    for (int v = 0; v < nv; v++)
      for (int a = 0; a < 3; a++) B->X[3 * v + a] = x[3 * v + a] - cm[a];
    for (int k = 0; k < 9; k++) B->R[k] = (k % 4 == 0) ? 1.0 : 0.0;
    if (rigid && !fixed && v0) {
      for (int a = 0; a < 3; a++) {
        double m = 0.0;
        for (int v = 0; v < nv; v++) m += v0[3 * v + a];
        B->u[a] = B->uprev[a] = m / nv;
      }
      for (int v = 0; v < nv; v++)
        for (int a = 0; a < 3; a++) B->v[3 * v + a] = B->u[a];
    }
  }
  return s->nbody++;
}

/* ------------------------------------------------------------------- MLS */
/* Moving-least-squares transfer (Eqs. uLag, l2norm, intKernel): the 27
 * lattice nodes of the 3x3x3 block around the node nearest to p (base node
 * floor(p + 1/2)), weights W = exp(-(r/alpha)^2) for r <= 1 with alpha = 0.3
 * and r the distance normalised by the support side 2 r_w = 2.6, linear basis
 * p(x) = (1, x - p) (local coordinates, so the fitted value at p is the first
 * coefficient), moment matrix A = sum W p p^T, coefficients a = A^{-1} sum W p u.
 * Readings: the fixed 27-node block is the support (every node of it lies
 * within r <= 1); solid nodes and nodes outside a non-periodic box face are
 * excluded from the sums.  psi[k][0..3] = W_k (A^{-1} p_k): psi[k][0] is the
 * interpolation weight phi_k, psi[k][1..3] give the gradient of the fit.
 * A singular moment matrix (pivot below 1e-10 of the largest diagonal)
 * gives all-zero weights and returns 0. */
static int mls_point(const orc_sim *s, const double *p, long *node, double psi[27][4]) {
  int b[3];
  for (int a = 0; a < 3; a++) b[a] = (int)floor(p[a] + 0.5);
  double Wk[27], P[27][4];
  double A[4][4] = {{0}};
  int dim[3] = {s->nx, s->ny, s->nz};
  for (int k = 0; k < 27; k++) {
    int d[3] = {k % 3 - 1, (k / 3) % 3 - 1, k / 9 - 1};
    int c[3];
    long idx = 0;
    int ok = 1;
    for (int a = 0; a < 3; a++) {
      c[a] = b[a] + d[a];
      int w = c[a];
      if (w < 0 || w >= dim[a]) {
        if (!s->per[a]) ok = 0;
        else w = ((w % dim[a]) + dim[a]) % dim[a];
      }
      if (a == 0) idx = w;
      else if (a == 1) idx += (long)s->nx * w;
      else idx += (long)s->nx * s->ny * w;
    }
    if (ok && s->type[idx] == T_SOLID) ok = 0;
    P[k][0] = 1.0;
    for (int a = 0; a < 3; a++) P[k][1 + a] = c[a] - p[a];
    double r = sqrt(P[k][1] * P[k][1] + P[k][2] * P[k][2] + P[k][3] * P[k][3]) / 2.6;
    Wk[k] = (ok && r <= 1.0) ? exp(-(r / 0.3) * (r / 0.3)) : 0.0;
    node[k] = ok ? idx : -1;
    for (int i = 0; i < 4; i++)
      for (int j = 0; j < 4; j++) A[i][j] += Wk[k] * P[k][i] * P[k][j];
  }
  /* Cholesky A = L L^T */
  double L[4][4] = {{0}};
  double dmax = 0.0;
  for (int i = 0; i < 4; i++) dmax = fmax(dmax, A[i][i]);
  int ok = dmax > 0.0;
  for (int j = 0; j < 4 && ok; j++) {
    double d = A[j][j];
    for (int k = 0; k < j; k++) d -= L[j][k] * L[j][k];
    if (!(d > 1e-10 * dmax)) { ok = 0; break; }
    L[j][j] = sqrt(d);
    for (int i = j + 1; i < 4; i++) {
      double v = A[i][j];
      for (int k = 0; k < j; k++) v -= L[i][k] * L[j][k];
      L[i][j] = v / L[j][j];
    }
  }
  if (!ok) {
    for (int k = 0; k < 27; k++)
      for (int i = 0; i < 4; i++) psi[k][i] = 0.0;
    return 0;
  }
  /* A^{-1} column by column */
  double Ainv[4][4];
  for (int c = 0; c < 4; c++) {
    double y[4], z[4];
    for (int i = 0; i < 4; i++) {
      double v = (i == c) ? 1.0 : 0.0;
      for (int k = 0; k < i; k++) v -= L[i][k] * y[k];
      y[i] = v / L[i][i];
    }
    for (int i = 3; i >= 0; i--) {
      double v = y[i];
      for (int k = i + 1; k < 4; k++) v -= L[k][i] * z[k];
      z[i] = v / L[i][i];
    }
    for (int i = 0; i < 4; i++) Ainv[i][c] = z[i];
  }
  for (int k = 0; k < 27; k++)
    for (int i = 0; i < 4; i++) {
      double v = 0.0;
      for (int j = 0; j < 4; j++) v += Ainv[i][j] * P[k][j];
      psi[k][i] = Wk[k] * v;
    }
  return 1;
}

int orc_mls_point(const orc_sim *s, const double *p, int64_t *node27, double *psi27x4) {
  long node[27];
  double psi[27][4];
  int ok = mls_point(s, p, node, psi);
  for (int k = 0; k < 27; k++) {
    node27[k] = node[k];
    for (int i = 0; i < 4; i++) psi27x4[4 * k + i] = psi[k][i];
  }
  return ok;
}

/* Eq. uLag on a [3][N] field. */
void orc_ib_interpolate(const orc_sim *s, int64_t n, const double *pts, const double *field,
                        double *out) {
  for (int64_t l = 0; l < n; l++) {
    long node[27];
    double psi[27][4];
    mls_point(s, pts + 3 * l, node, psi);
    for (int a = 0; a < 3; a++) {
      double U = 0.0;
      for (int k = 0; k < 27; k++)
        if (node[k] >= 0) U += psi[k][0] * field[(long)a * s->N + node[k]];
      out[3 * l + a] = U;
    }
  }
}

/* Eq. bodyforce on a [3][N] field (added to fib): the sums run over the
 * points in index order. */
void orc_ib_spread(const orc_sim *s, int64_t n, const double *pts, const double *F,
                   const double *c, double *fib) {
  for (int64_t l = 0; l < n; l++) {
    long node[27];
    double psi[27][4];
    mls_point(s, pts + 3 * l, node, psi);
    for (int k = 0; k < 27; k++) {
      if (node[k] < 0) continue;
      for (int a = 0; a < 3; a++) fib[(long)a * s->N + node[k]] += c[l] * psi[k][0] * F[3 * l + a];
    }
  }
}

/* ------------------------------------------------------------ the step */
/* S1 + S2 + S3 for one node: streamed populations into s->f, moments. */
static void stream_node(orc_sim *s, long n) {
  preal *f = s->f + 19 * n;
  const preal *fs = s->fs;
  int x, y, z;
  coords(s, n, &x, &y, &z);
  f[0] = fs[19 * n + 0];
  for (int j = 1; j < 19; j++) {
    long src = neighbour(s, x, y, z, -E[j][0], -E[j][1], -E[j][2]);
    if (src < 0) {
      f[j] = 0.0; /* unknown: filled by the open-face condition below */
    } else if (s->type[src] == T_SOLID) {
      int i = opposite(j); /* x + e_i = src is solid */
      preal q = find_q(s, n, i);
      long a1 = neighbour(s, x, y, z, -E[i][0], -E[i][1], -E[i][2]);
      long a2 = neighbour(s, x, y, z, -2 * E[i][0], -2 * E[i][1], -2 * E[i][2]);
      int av1 = a1 >= 0 && s->type[a1] != T_SOLID;
      int av2 = a2 >= 0 && s->type[a2] != T_SOLID;
      f[j] = bfl(q, fs[19 * n + i], av1 ? fs[19 * a1 + i] : PR(0.0), av2 ? fs[19 * a2 + i] : PR(0.0),
                 fs[19 * n + j], av1 ? fs[19 * a1 + j] : PR(0.0), av1, av2);
    } else {
      f[j] = fs[19 * src + j];
    }
  }
  if (s->type[n] == T_INLET || s->type[n] == T_OUTLET) {
    int face = open_face(s, n);
    if (s->type[n] == T_INLET) zouhe_dev(f, face, 0, s->uin + 3 * n, PR(0.0));
    else zouhe_dev(f, face, 1, NULL, s->rho_out);
  }
  /* moments of f = w + d: the weights add up to 1 and carry no momentum */
  preal dsum = PR(0.0), m[3] = {0, 0, 0};
  for (int i = 0; i < 19; i++) {
    dsum += f[i];
    for (int a = 0; a < 3; a++) m[a] += f[i] * E[i][a];
  }
#ifdef ORC_FULL_POP
  preal rho = dsum;
#else
  preal rho = PR(1.0) + dsum;
#endif
  s->rho[n] = rho;
  for (int a = 0; a < 3; a++) {
    s->mom[3 * n + a] = m[a];
    s->ustar[3 * n + a] = (double)(m[a] / rho);
  }
}

/* S5 for one node: BGK collision with the forcing term. */
static int collide_node(orc_sim *s, long n) {
  preal *f = s->f + 19 * n;
  preal rho = s->rho[n];
  preal F[3], u[3];
  for (int a = 0; a < 3; a++) {
    F[a] = (preal)s->g[a] + s->fib[3 * n + a];
    /* rho u = sum f e + (dt/2) f_ib */
    u[a] = (s->mom[3 * n + a] + PR(0.5) * F[a]) / rho;
  }
  for (int i = 0; i < 19; i++) {
    preal v = f[i] - (f[i] - feq_store_i(i, rho, u)) / s->tau + guo_i(i, s->tau, u, F);
#ifdef ORC_STORE_F32
    /* measurement build only: the state rounded to FP32 at every store, to
     * gauge how far FP32 storage alone moves a trajectory */
    v = (preal)(float)v;
#endif
#ifdef ORC_STORE_F16
    /* measurement build only: the state rounded to binary16 (11 significant
     * bits, subnormal spacing 2^-24, ties to even) at every store */
    if (v != 0.0) {
      int ex;
      frexp(v, &ex);
      const double ulp = ldexp(1.0, (ex - 11 < -24) ? -24 : ex - 11);
      v = nearbyint(v / ulp) * ulp;
    }
#endif
    s->fs[19 * n + i] = v;
  }
  double ud[3];
  for (int a = 0; a < 3; a++) s->u[3 * n + a] = ud[a] = (double)u[a];
  double uu = dot(ud, ud);
  return !(uu <= 0.09) || !(rho == rho);
}

/* Current marker velocity U_b at point p of body B: the mean of the three
 * vertex velocities of the face for a soft body; the rigid-body velocity
 * field u + omega x (p - x_c) for a rigid one. */
static void body_velocity_at(const body_t *B, int f, const double *p, double *Ub) {
  if (B->rigid) {
    double r[3], wr[3];
    sub(p, B->xc, r);
    cross(B->w, r, wr);
    for (int a = 0; a < 3; a++) Ub[a] = B->u[a] + wr[a];
  } else {
    for (int a = 0; a < 3; a++)
      Ub[a] = (B->v[3 * B->faces[3 * f] + a] + B->v[3 * B->faces[3 * f + 1] + a] +
               B->v[3 * B->faces[3 * f + 2] + a]) / 3.0;
  }
}

/* S4: direct forcing at the face centroids (the Lagrangian markers).  The
 * per-marker transfer weights are independent and computed in parallel; the
 * force is then accumulated serially, marker by marker in index order. */
static void ib_forcing(orc_sim *s) {
  memset(s->fib, 0, sizeof(double) * 3 * s->N);
  int nthr = orc_threads();
  for (int b = 0; b < s->nbody; b++) {
    body_t *B = &s->bodies[b];
    long *node = (long *)malloc(sizeof(long) * 27 * B->nf);
    double *phiF = (double *)malloc(sizeof(double) * 27 * 3 * B->nf);
    int sing = 0;
#pragma omp parallel for schedule(static) num_threads(nthr) reduction(+ : sing)
    for (int f = 0; f < B->nf; f++) {
      double xl[3], nh[3], A;
      face_geom(B->x, B->faces + 3 * f, xl, nh, &A);
      double psi[27][4];
      if (!mls_point(s, xl, node + 27 * f, psi)) sing++;
      double U[3] = {0, 0, 0}, Ub[3], F[3];
      for (int k = 0; k < 27; k++)
        if (node[27 * f + k] >= 0)
          for (int a = 0; a < 3; a++) U[a] += psi[k][0] * s->ustar[3 * node[27 * f + k] + a];
      body_velocity_at(B, f, xl, Ub);
      /* F_l = (U_b - U) / dt with dt = 1 */
      for (int a = 0; a < 3; a++) F[a] = Ub[a] - U[a];
      /* c_l: marker volume A_l * h / dx^3 with h = dx (total-force
       * conservation between the two grids; reading of the text that cites
       * it without a formula) */
      double cl = A;
      for (int k = 0; k < 27; k++)
        for (int a = 0; a < 3; a++) phiF[(27 * f + k) * 3 + a] = cl * psi[k][0] * F[a];
    }
    s->mls_singular += sing;
    for (int f = 0; f < B->nf; f++)
      for (int k = 0; k < 27; k++) {
        long n = node[27 * f + k];
        if (n < 0) continue;
        for (int a = 0; a < 3; a++) s->fib[3 * n + a] += phiF[(27 * f + k) * 3 + a];
      }
    free(node);
    free(phiF);
  }
}

/* MLS fit of p = c_s^2 rho, rho and u (value and gradient) at a point. */
static void probe(const orc_sim *s, const double *p, double *pr, double *rh, double gradu[3][3]) {
  long node[27];
  double psi[27][4];
  mls_point(s, p, node, psi);
  *pr = 0.0;
  *rh = 0.0;
  for (int a = 0; a < 3; a++)
    for (int c = 0; c < 3; c++) gradu[a][c] = 0.0;
  for (int k = 0; k < 27; k++) {
    if (node[k] < 0) continue;
    double r = s->rho[node[k]];
    *pr += psi[k][0] * CS2 * r;
    *rh += psi[k][0] * r;
    for (int a = 0; a < 3; a++)
      for (int c = 0; c < 3; c++) gradu[a][c] += psi[k][1 + c] * s->u[3 * node[k] + a];
  }
}

/* S7: hydrodynamic force on each face (Eqs. hydroForP, hydroForNu): pressure
 * and viscous stress tau = rho nu (grad u + grad u^T) fitted 1.2 dx outside
 * (+) and inside (-) the face along its outward normal. */
static void hydro_faces(const orc_sim *s, const body_t *B, double *Fface) {
#pragma omp parallel for schedule(static) num_threads(orc_threads())
  for (int f = 0; f < B->nf; f++) {
    double xc[3], nh[3], A;
    face_geom(B->x, B->faces + 3 * f, xc, nh, &A);
    double pp[2], rr[2], G[2][3][3];
    for (int side = 0; side < 2; side++) {
      double sg = side == 0 ? 1.0 : -1.0, xp[3];
      for (int a = 0; a < 3; a++) xp[a] = xc[a] + sg * 1.2 * nh[a];
      probe(s, xp, &pp[side], &rr[side], G[side]);
    }
    for (int a = 0; a < 3; a++) {
      double tn = 0.0;
      for (int c = 0; c < 3; c++) {
        double tp = rr[0] * s->nu * (G[0][a][c] + G[0][c][a]);
        double tm = rr[1] * s->nu * (G[1][a][c] + G[1][c][a]);
        tn += (tp - tm) * nh[c];
      }
      Fface[3 * f + a] = (-(pp[0] - pp[1]) * nh[a] + tn) * A;
    }
  }
}

void orc_body_hydro(const orc_sim *s, int id, double *Fface) {
  hydro_faces(s, &s->bodies[id], Fface);
}

void orc_body_fext(const orc_sim *s, int id, double *Fface) {
  const body_t *B = &s->bodies[id];
  memcpy(Fface, B->Fext, sizeof(double) * 3 * B->nf);
}

/* S6 repulsion (Eq. collision): centroid pairs of different bodies closer
 * than dx push the receiving face along its inward normal with magnitude
 * u_max dt / (8 sqrt 2) sqrt(dx / d^5).  Pairs of bodies whose bounding
 * boxes are more than dx apart are skipped (they have no such pair). */
static void repulsion(orc_sim *s) {
  if (s->nbody < 2) return;
  const double pref = s->umax / (8.0 * sqrt(2.0));
  /* centroid, outward normal and bounding box of every body */
  double **cen = (double **)calloc(s->nbody, sizeof(double *));
  double **nrm = (double **)calloc(s->nbody, sizeof(double *));
  double *box = (double *)malloc(sizeof(double) * 6 * s->nbody);
  for (int b = 0; b < s->nbody; b++) {
    body_t *B = &s->bodies[b];
    cen[b] = (double *)malloc(sizeof(double) * 3 * B->nf);
    nrm[b] = (double *)malloc(sizeof(double) * 3 * B->nf);
    for (int f = 0; f < B->nf; f++) {
      double A;
      face_geom(B->x, B->faces + 3 * f, cen[b] + 3 * f, nrm[b] + 3 * f, &A);
    }
    double *lo = box + 6 * b, *hi = box + 6 * b + 3;
    for (int a = 0; a < 3; a++) { lo[a] = 1e300; hi[a] = -1e300; }
    for (int v = 0; v < B->nv; v++)
      for (int a = 0; a < 3; a++) { lo[a] = fmin(lo[a], B->x[3 * v + a]); hi[a] = fmax(hi[a], B->x[3 * v + a]); }
  }
  for (int b = 0; b < s->nbody; b++) {
    body_t *B = &s->bodies[b];
    for (int o = 0; o < s->nbody; o++) {
      if (o == b) continue;
      const double *lo = box + 6 * b, *hi = box + 6 * b + 3, *lo2 = box + 6 * o, *hi2 = box + 6 * o + 3;
      int far = 0;
      for (int a = 0; a < 3; a++)
        if (lo[a] > hi2[a] + 1.0 || lo2[a] > hi[a] + 1.0) far = 1;
      if (far) continue;
      const int nfo = s->bodies[o].nf;
#pragma omp parallel for schedule(static) num_threads(orc_threads())
      for (int f = 0; f < B->nf; f++) {
        const double *ci = cen[b] + 3 * f, *ni = nrm[b] + 3 * f;
        for (int g = 0; g < nfo; g++) {
          double d[3];
          sub(ci, cen[o] + 3 * g, d);
          double dist = norm(d);
          if (dist < 1.0 && dist > 0.0) {
            double mag = pref * sqrt(1.0 / pow(dist, 5.0));
            for (int a = 0; a < 3; a++) B->Fext[3 * f + a] += mag * (-ni[a]);
          }
        }
      }
    }
  }
  for (int b = 0; b < s->nbody; b++) { free(cen[b]); free(nrm[b]); }
  free(cen); free(nrm); free(box);
}

/* Internal membrane forces for positions x (Eqs. strainFor, bendFor, volFor)
 * and the matching energy. */
static double membrane(const orc_sim *s, const body_t *B, const double *x, int which, double *F) {
  (void)s;
  double E_tot = 0.0;
  memset(F, 0, sizeof(double) * 3 * B->nv);
  if (which & 1) {
    /* stretching: V = 1/2 k (l - l0)^2, F_1 = -k (l - l0) r_12 / l */
    for (int e = 0; e < B->ne; e++) {
      int a = B->edges[2 * e], b = B->edges[2 * e + 1];
      double r[3];
      sub(x + 3 * a, x + 3 * b, r);
      double l = norm(r), dl = l - B->l0[e];
      E_tot += 0.5 * B->kl[e] * dl * dl;
      for (int c = 0; c < 3; c++) {
        double fc = -B->kl[e] * dl * r[c] / l;
        F[3 * a + c] += fc;
        F[3 * b + c] -= fc;
      }
    }
  }
  if (which & 2) {
    /* bending.  Reading: the printed hinge forces are garbled (b_11 = b_22 = 1
     * by their own definition); the amplitude beta_b printed with them is
     * k_b sin(theta - theta0)/sin(theta), i.e. the force of the hinge energy
     * k_b (1 - cos(theta - theta0)) ~ 1/2 k_b (theta - theta0)^2 (the
     * quadratic bending potential).  F = -k_b sin(theta - theta0) dtheta/dx,
     * with the exact gradient of the dihedral angle. */
    for (int h = 0; h < B->nh; h++) {
      const int *H = B->hinge + 4 * h;
      double n1[3], n2[3];
      double th = dihedral(x, H, n1, n2);
      double dth = th - B->theta0[h];
      E_tot += B->kb[h] * (1.0 - cos(dth));
      const double *a = x + 3 * H[0], *b = x + 3 * H[1], *c = x + 3 * H[2], *d = x + 3 * H[3];
      double e[3], ca[3], da[3];
      sub(b, a, e);
      sub(c, a, ca);
      sub(d, a, da);
      double le2 = dot(e, e), le = sqrt(le2);
      double q1 = dot(n1, n1), q2 = dot(n2, n2);
      double gc[3], gd[3], ga[3], gb[3];
      double al_c = dot(ca, e) / le2, al_d = dot(da, e) / le2;
      for (int k = 0; k < 3; k++) {
        gc[k] = -le * n1[k] / q1;
        gd[k] = -le * n2[k] / q2;
        gb[k] = -(al_c * gc[k] + al_d * gd[k]);
        ga[k] = -((1.0 - al_c) * gc[k] + (1.0 - al_d) * gd[k]);
      }
      double amp = -B->kb[h] * sin(dth);
      for (int k = 0; k < 3; k++) {
        F[3 * H[0] + k] += amp * ga[k];
        F[3 * H[1] + k] += amp * gb[k];
        F[3 * H[2] + k] += amp * gc[k];
        F[3 * H[3] + k] += amp * gd[k];
      }
    }
  }
  if (which & 4) {
    /* volume penalty.  Reading of the sign: with n the outward normal the
     * force k_v (1 - V/V0) n A restores the volume (the printed minus sign
     * holds for an inward normal); it is -grad of 1/2 (k_v/V0)(V - V0)^2,
     * one third of each face's share going to each of its vertices. */
    double V = mesh_volume(x, B->faces, B->nf);
    E_tot += 0.5 * B->kv / B->V0 * (V - B->V0) * (V - B->V0);
    for (int f = 0; f < B->nf; f++) {
      double c[3], n[3], A;
      face_geom(x, B->faces + 3 * f, c, n, &A);
      for (int v = 0; v < 3; v++)
        for (int k = 0; k < 3; k++) F[3 * B->faces[3 * f + v] + k] += B->kv * (1.0 - V / B->V0) * A * n[k] / 3.0;
    }
  }
  return E_tot;
}

double orc_membrane(const orc_sim *s, int id, const double *x, int which, double *F) {
  return membrane(s, &s->bodies[id], x, which, F);
}

/* Rotation matrix of the rotation vector phi (Rodrigues). */
static void rodrigues(const double *phi, double *Rm) {
  double th = norm(phi);
  if (th == 0.0) {
    for (int k = 0; k < 9; k++) Rm[k] = (k % 4 == 0) ? 1.0 : 0.0;
    return;
  }
  double k[3] = {phi[0] / th, phi[1] / th, phi[2] / th};
  double c = cos(th), sn = sin(th), omc = 2.0 * sin(0.5 * th) * sin(0.5 * th);
  double K[9] = {0, -k[2], k[1], k[2], 0, -k[0], -k[1], k[0], 0};
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) Rm[3 * i + j] = (i == j ? c : 0.0) + sn * K[3 * i + j] + omc * k[i] * k[j];
}

static void mat3_mul(const double *A, const double *B, double *C) {
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) {
      double v = 0.0;
      for (int k = 0; k < 3; k++) v += A[3 * i + k] * B[3 * k + j];
      C[3 * i + j] = v;
    }
}

static void solve3(const double *A, const double *b, double *x) {
  double det = A[0] * (A[4] * A[8] - A[5] * A[7]) - A[1] * (A[3] * A[8] - A[5] * A[6]) +
               A[2] * (A[3] * A[7] - A[4] * A[6]);
  for (int c = 0; c < 3; c++) {
    double M[9];
    memcpy(M, A, sizeof M);
    for (int r = 0; r < 3; r++) M[3 * r + c] = b[r];
    x[c] = (M[0] * (M[4] * M[8] - M[5] * M[7]) - M[1] * (M[3] * M[8] - M[5] * M[6]) +
            M[2] * (M[3] * M[7] - M[4] * M[6])) / det;
  }
}

/* S8 for a soft body: Verlet with the MLS tentative velocity (Eqs. verletPos,
 * verletVel, verletPosC, dt = 1).  Reading of the time levels: u_v,0 is the
 * MLS interpolation of the velocity just produced by the collision, at x^n. */
static void move_soft(orc_sim *s, body_t *B, const double *F) {
  double *xn = (double *)malloc(sizeof(double) * 3 * B->nv);
  double *u0 = (double *)malloc(sizeof(double) * 3 * B->nv);
  int sing = 0;
#pragma omp parallel for schedule(static) num_threads(orc_threads()) reduction(+ : sing)
  for (int v = 0; v < B->nv; v++) {
    long node[27];
    double psi[27][4];
    if (!mls_point(s, B->x + 3 * v, node, psi)) sing++;
    for (int a = 0; a < 3; a++) {
      double U = 0.0;
      for (int k = 0; k < 27; k++)
        if (node[k] >= 0) U += psi[k][0] * s->u[3 * node[k] + a];
      u0[3 * v + a] = U;
    }
  }
  s->mls_singular += sing;
  for (int v = 0; v < B->nv; v++)
    for (int a = 0; a < 3; a++) {
      int i = 3 * v + a;
      double acc = 0.5 * F[i] / B->m_v;
      double xt = B->x[i] + u0[i] + acc;                       /* predictor */
      double un = 1.5 * xt - 2.0 * B->x[i] + 0.5 * B->xprev[i]; /* velocity */
      xn[i] = B->x[i] + un + acc;                               /* corrector */
      B->v[i] = un;
    }
  memcpy(B->xprev, B->x, sizeof(double) * 3 * B->nv);
  memcpy(B->x, xn, sizeof(double) * 3 * B->nv);
  free(xn);
  free(u0);
}

/* S8 for a rigid body (Eq. angularVelRig and the Newton-Euler system): the
 * total force and moment about the centre of mass, second-order backward
 * update of u and omega, then x_c += u dt and a rotation by omega dt.
 * Readings: inertia tensor of the uniform solid enclosed by the mesh
 * rotated with the body; no gyroscopic term (the printed system has none);
 * the moment is taken from the vertex forces (one third of each face force). */
static void move_rigid(body_t *B, const double *Fv) {
  if (B->fixed) return;
  double F[3] = {0, 0, 0}, M[3] = {0, 0, 0};
  for (int v = 0; v < B->nv; v++) {
    double r[3], t[3];
    sub(B->x + 3 * v, B->xc, r);
    cross(r, Fv + 3 * v, t);
    for (int a = 0; a < 3; a++) { F[a] += Fv[3 * v + a]; M[a] += t[a]; }
  }
  double RI[9], Rt[9], Iw[9], alpha[3];
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) Rt[3 * i + j] = B->R[3 * j + i];
  mat3_mul(B->R, B->Ibody, RI);
  mat3_mul(RI, Rt, Iw);
  solve3(Iw, M, alpha);
  double un[3], wn[3];
  for (int a = 0; a < 3; a++) {
    un[a] = 2.0 / 3.0 * (2.0 * B->u[a] - 0.5 * B->uprev[a] + F[a] / B->mass);
    wn[a] = 2.0 / 3.0 * (2.0 * B->w[a] - 0.5 * B->wprev[a] + alpha[a]);
  }
  for (int a = 0; a < 3; a++) {
    B->uprev[a] = B->u[a]; B->u[a] = un[a];
    B->wprev[a] = B->w[a]; B->w[a] = wn[a];
    B->xc[a] += un[a];
  }
  double Rr[9], Rn[9];
  rodrigues(wn, Rr);
  mat3_mul(Rr, B->R, Rn);
  memcpy(B->R, Rn, sizeof Rn);
  memcpy(B->xprev, B->x, sizeof(double) * 3 * B->nv);
  for (int v = 0; v < B->nv; v++) {
    double r[3], wr[3];
    for (int a = 0; a < 3; a++)
      r[a] = B->R[3 * a] * B->X[3 * v] + B->R[3 * a + 1] * B->X[3 * v + 1] + B->R[3 * a + 2] * B->X[3 * v + 2];
    cross(B->w, r, wr);
    for (int a = 0; a < 3; a++) {
      B->x[3 * v + a] = B->xc[a] + r[a];
      B->v[3 * v + a] = B->u[a] + wr[a];
    }
  }
}

/* Test hooks of the rigid-body update (they change nothing in the step). */
void orc_body_inertia(const orc_sim *s, int id, double *I9) {
  memcpy(I9, s->bodies[id].Ibody, sizeof(double) * 9);
}

void orc_rodrigues(const double *phi, double *R9) { rodrigues(phi, R9); }

/* One S8 update of rigid body id driven by the given vertex forces [nv][3]
 * (in place of the hydrodynamic and repulsion forces of a step). */
int orc_move_rigid(orc_sim *s, int id, const double *Fv) {
  if (!s || id < 0 || id >= s->nbody || !s->bodies[id].rigid) return ORC_E_INVAL;
  move_rigid(&s->bodies[id], Fv);
  return ORC_OK;
}

static int one_step(orc_sim *s) {
  long N = s->N;
  int nthr = orc_threads();
  /* S1-S3 */
#pragma omp parallel for schedule(static) num_threads(nthr)
  for (long n = 0; n < N; n++)
    if (s->type[n] != T_SOLID) stream_node(s, n);
  /* S4 */
  if (s->nbody > 0) ib_forcing(s);
  else memset(s->fib, 0, sizeof(double) * 3 * N);
  /* S5 */
  int bad = 0;
#pragma omp parallel for schedule(static) num_threads(nthr) reduction(| : bad)
  for (long n = 0; n < N; n++)
    if (s->type[n] != T_SOLID) bad |= collide_node(s, n);
  /* S6-S8 */
  int damaged = 0;
  for (int b = 0; b < s->nbody; b++) {
    body_t *B = &s->bodies[b];
    hydro_faces(s, B, B->Fext);
  }
  repulsion(s);
  for (int b = 0; b < s->nbody; b++) {
    body_t *B = &s->bodies[b];
    double *Fv = (double *)calloc(3 * B->nv, sizeof(double));
    if (!B->rigid) membrane(s, B, B->x, 7, Fv);
    for (int f = 0; f < B->nf; f++)
      for (int v = 0; v < 3; v++)
        for (int a = 0; a < 3; a++) Fv[3 * B->faces[3 * f + v] + a] += B->Fext[3 * f + a] / 3.0;
    if (B->rigid) move_rigid(B, Fv);
    else move_soft(s, B, Fv);
    free(Fv);
    /* diagnostics: volume, area, largest stretch; a link whose length
     * doubles its rest length is damaged and stops the computation */
    B->V = mesh_volume(B->x, B->faces, B->nf);
    B->S = mesh_area(B->x, B->faces, B->nf);
    B->max_strain = 0.0;
    for (int e = 0; e < B->ne; e++) {
      double r[3];
      sub(B->x + 3 * B->edges[2 * e], B->x + 3 * B->edges[2 * e + 1], r);
      double st = norm(r) / B->l0[e];
      if (st > B->max_strain) B->max_strain = st;
      if (!B->rigid && st >= 2.0) damaged = 1;
    }
    for (int k = 0; k < 3 * B->nv; k++)
      if (!(B->x[k] == B->x[k])) bad = 1;
  }
  s->steps_done++;
  if (damaged) return ORC_E_DAMAGED;
  if (bad) return ORC_E_UNSTABLE;
  return ORC_OK;
}

int orc_step(orc_sim *s, int n_steps) {
  if (!s) return ORC_E_INVAL;
  for (int k = 0; k < n_steps; k++) {
    if (s->status != ORC_OK) return s->status;
    s->status = one_step(s);
  }
  return s->status;
}

int64_t orc_steps_done(const orc_sim *s) { return s->steps_done; }
int orc_status(const orc_sim *s) { return s->status; }
int orc_mls_singular_count(const orc_sim *s) { return s->mls_singular; }

void orc_get_fields(const orc_sim *s, double *rho, double *u) {
  for (long n = 0; n < s->N; n++) {
    int solid = s->type[n] == T_SOLID;
    if (rho) rho[n] = solid ? 0.0 : (double)s->rho[n];
    if (u)
      for (int a = 0; a < 3; a++) u[(long)a * s->N + n] = solid ? 0.0 : s->u[3 * n + a];
  }
}

/* The stored value of population i at node n as a full population f_i. */
static preal full_pop(const orc_sim *s, long n, int i) {
#ifdef ORC_FULL_POP
  return s->fs[19 * n + i];
#else
  return Wt[i] + s->fs[19 * n + i];
#endif
}

void orc_get_populations(const orc_sim *s, double *f) {
  for (long n = 0; n < s->N; n++)
    for (int i = 0; i < 19; i++)
      f[(long)i * s->N + n] = s->type[n] == T_SOLID ? 0.0 : (double)full_pop(s, n, i);
}

/* The inverse of orc_get_populations: the stored post-collision
 * populations become f ([19][N]); entries at solid nodes are ignored. */
void orc_set_populations(orc_sim *s, const double *f) {
  for (long n = 0; n < s->N; n++)
    if (s->type[n] != T_SOLID)
      for (int i = 0; i < 19; i++) {
#ifdef ORC_FULL_POP
        s->fs[19 * n + i] = f[(long)i * s->N + n];
#else
        s->fs[19 * n + i] = f[(long)i * s->N + n] - Wt[i];
#endif
      }
}

/* The populations f_i of the listed nodes only: f[i * n + k] for node
 * nodes[k] (the same values as orc_get_populations). */
void orc_get_populations_at(const orc_sim *s, long n, const long *nodes, double *f) {
  for (long k = 0; k < n; k++)
    for (int i = 0; i < 19; i++)
      f[(long)i * n + k] = s->type[nodes[k]] == T_SOLID ? 0.0 : (double)full_pop(s, nodes[k], i);
}

void orc_get_force(const orc_sim *s, double *fib) {
  for (long n = 0; n < s->N; n++)
    for (int a = 0; a < 3; a++) fib[(long)a * s->N + n] = s->fib[3 * n + a];
}

void orc_get_body(const orc_sim *s, int id, double *x, double *v) {
  const body_t *B = &s->bodies[id];
  if (x) memcpy(x, B->x, sizeof(double) * 3 * B->nv);
  if (v) memcpy(v, B->v, sizeof(double) * 3 * B->nv);
}

void orc_body_diag(const orc_sim *s, int id, double *o) {
  const body_t *B = &s->bodies[id];
  o[0] = B->V; o[1] = B->S; o[2] = B->V0; o[3] = B->S0; o[4] = B->max_strain; o[5] = B->mass;
  o[6] = B->kv; o[7] = B->ks0;
  for (int a = 0; a < 3; a++) { o[8 + a] = B->xc[a]; o[11 + a] = B->u[a]; o[14 + a] = B->w[a]; }
  o[17] = B->m_v; o[18] = B->rigid; o[19] = B->nf;
}
