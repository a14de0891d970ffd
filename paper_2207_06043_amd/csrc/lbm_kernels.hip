// gfx950 kernels of the coupled lattice-Boltzmann / dynamic immersed-boundary
// step (Coclite, de Tullio, Pascazio, Politi, arXiv 2207.06043, section
// "Numerical method and computational procedure").
//
// One step is five launches on one stream:
//   k_ib_force   MLS interpolation of the streamed (pre-force) velocity at the
//                face centroids, direct forcing and spreading (fixed-point
//                atomics, deterministic), clearing of the previous step's
//                spread buffer;
//   k_fluid      fused pull-stream + wall links (interpolated bounce-back) +
//                Zou-He + moments + forced BGK collision; bulk tiles use
//                128-bit SoA loads/stores, boundary nodes use compact records;
//   k_mls_post   hydrodynamic probes (pressure and viscous stress from MLS
//                fits at +-1.2 dx), repulsion, MLS velocity at the vertices;
//   k_body_post  membrane forces and Verlet (soft) / Newton-Euler (rigid);
//   k_diag       volume, area, bounding box, damage and the step bookkeeping.
// Populations are stored as deviations g_i = f_i - w_i from the rest
// equilibrium; the collision is written for g (algebraically identical to the
// BGK rule on f, with smaller rounding).
#include <float.h>
#include <limits.h>
#include <math.h>

#include "lbm_internal.h"

namespace lbm {

// D3Q19 velocity set in the order of the paper's Eq. e_i.
constexpr int EX[19] = {0, 1, -1, 0, 0, 0, 0, 1, 1, 1, 1, -1, -1, -1, -1, 0, 0, 0, 0};
constexpr int EY[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, 0, 0, 1, -1, 0, 0, 1, 1, -1, -1};
constexpr int EZ[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 1, -1, 0, 0, 1, -1, 1, -1, 1, -1};
constexpr int OPP[19] = {0, 2, 1, 4, 3, 6, 5, 12, 11, 14, 13, 8, 7, 10, 9, 18, 17, 16, 15};
constexpr double WD[19] = {1.0 / 3,  1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18,
                           1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36,
                           1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};

// ---------------------------------------------------------------- storage
__device__ __forceinline__ double to_c(double v) { return v; }
__device__ __forceinline__ float to_c(float v) { return v; }
__device__ __forceinline__ float to_c(_Float16 v) { return (float)v; }

template <class S>
struct Store;
template <>
struct Store<double> {
  typedef double C;
  static constexpr int V = 2;
  typedef double vec __attribute__((ext_vector_type(2)));
  typedef double vecu __attribute__((ext_vector_type(2), aligned(8)));
};
template <>
struct Store<float> {
  typedef float C;
  static constexpr int V = 4;
  typedef float vec __attribute__((ext_vector_type(4)));
  typedef float vecu __attribute__((ext_vector_type(4), aligned(4)));
};
template <>
struct Store<_Float16> {
  typedef float C;
  static constexpr int V = 8;
  typedef _Float16 vec __attribute__((ext_vector_type(8)));
  typedef _Float16 vecu __attribute__((ext_vector_type(8), aligned(2)));
};

// ------------------------------------------------------------ index helpers
__device__ __forceinline__ int wrapc(int c, int n) {
  if (c < 0 || c >= n) c = ((c % n) + n) % n;
  return c;
}

// Node at (x,y,z)+(dx,dy,dz) with periodic wrap (the host guarantees the
// target is inside the box or across a periodic face).
__device__ __forceinline__ long long nbr(const Grid& G, int x, int y, int z, int dx, int dy,
                                         int dz) {
  x = wrapc(x + dx, G.nx);
  y = wrapc(y + dy, G.ny);
  z = wrapc(z + dz, G.nz);
  return x + (long long)G.px * (y + (long long)G.ny * z);
}

__device__ __forceinline__ void coords(const Grid& G, long long n, int& x, int& y, int& z) {
  x = (int)(n % G.px);
  long long t = n / G.px;
  y = (int)(t % G.ny);
  z = (int)(t / G.ny);
}

// Blocks are dispatched round-robin over the 8 XCDs; give every XCD a
// contiguous run of tiles so that neighbouring rows share its L2.
__device__ __forceinline__ int xcd_remap(int b, int n) {
  int full = n & ~7;
  if (b >= full) return b;
  return (b & 7) * (full >> 3) + (b >> 3);
}

__device__ __forceinline__ void fx_add(long long* p, double v, DevFlags* fl) {
  if (!(fabs(v) <= 1.0)) atomicOr(&fl->overflow, 1u);
  long long q = __double2ll_rn(v * FX_SCALE);
  atomicAdd((unsigned long long*)p, (unsigned long long)q);
}

// ---------------------------------------------------------------- collision
// BGK with the forcing term on deviations g = f - w (Eqs. evoleq, eqfunc,
// forcing): rho = 1 + sum g, rho u = sum g e + F/2,
// g^eq_i = w_i (drho + rho (3 e.u + 9/2 (e.u)^2 - 3/2 u.u)),
// F_i = (1 - 1/(2 tau)) w_i (3 (e_i - u) + 9 (e_i.u) e_i).F.
template <class C>
__device__ __forceinline__ void collide(C (&g)[19], C Fx, C Fy, C Fz, C omega, C& rho, C& ux,
                                        C& uy, C& uz) {
  C drho = 0;
#pragma unroll
  for (int i = 0; i < 19; i++) drho += g[i];
  C mx = (g[1] - g[2]) + (g[7] + g[8]) + (g[9] + g[10]) - (g[11] + g[12]) - (g[13] + g[14]);
  C my = (g[3] - g[4]) + (g[7] - g[8]) + (g[11] - g[12]) + (g[15] + g[16]) - (g[17] + g[18]);
  C mz = (g[5] - g[6]) + (g[9] - g[10]) + (g[13] - g[14]) + (g[15] - g[16]) + (g[17] - g[18]);
  rho = C(1) + drho;
  C ir = C(1) / rho;
  ux = (mx + C(0.5) * Fx) * ir;
  uy = (my + C(0.5) * Fy) * ir;
  uz = (mz + C(0.5) * Fz) * ir;
  C usq = ux * ux + uy * uy + uz * uz;
  C uF = ux * Fx + uy * Fy + uz * Fz;
  C kf = C(1) - C(0.5) * omega;
#pragma unroll
  for (int i = 0; i < 19; i++) {
    C eu = C(EX[i]) * ux + C(EY[i]) * uy + C(EZ[i]) * uz;
    C eF = C(EX[i]) * Fx + C(EY[i]) * Fy + C(EZ[i]) * Fz;
    C w = C(WD[i]);
    C geq = w * (drho + rho * (C(3) * eu + C(4.5) * eu * eu - C(1.5) * usq));
    C Gi = kf * w * (C(3) * (eF - uF) + C(9) * eu * eF);
    g[i] = g[i] - omega * (g[i] - geq) + Gi;
  }
}

// ----------------------------------------------------- boundary nodes (S1/S2)
template <class S>
__device__ __forceinline__ typename Store<S>::C ldA(const FluidArgs& a, int j, long long node) {
  return to_c(((const S*)a.A)[(long long)j * a.g.plane + node]);
}

// Zou-He on an open face (Eq. extbound, general inward normal n = s e_ax),
// on deviations: rho_w = (1 + G0 + 2 Gout)/(1 - u_n) for a velocity face,
// u_n = (rho_w - 1 - G0 - 2 Gout)/rho_w for a density face (tangential u = 0).
template <class C>
__device__ void zouhe(C (&g)[19], int face, int kind, C bx, C by, C bz, C brho) {
  const int ax = face >> 1;
  const int s = (face & 1) ? -1 : 1;
  C G0 = 0, Gout = 0;
#pragma unroll
  for (int j = 0; j < 19; j++) {
    int e = ax == 0 ? EX[j] : (ax == 1 ? EY[j] : EZ[j]);
    int en = s * e;
    if (en == 0) G0 += g[j];
    else if (en == -1) Gout += g[j];
  }
  C u[3] = {bx, by, bz};
  C rho, un;
  if (kind == 0) {
    un = C(s) * u[ax];
    rho = (C(1) + G0 + C(2) * Gout) / (C(1) - un);
  } else {
    rho = brho;
    un = (rho - C(1) - G0 - C(2) * Gout) / rho;
    u[0] = u[1] = u[2] = 0;
    u[ax] = C(s) * un;
  }
#pragma unroll
  for (int j = 1; j < 19; j++) {
    int e[3] = {EX[j], EY[j], EZ[j]};
    if (s * e[ax] != 1) continue;
    int t[3] = {e[0], e[1], e[2]};
    t[ax] -= s;
    C val;
    if (t[0] == 0 && t[1] == 0 && t[2] == 0) {
      val = g[OPP[j]] + rho / C(3) * un;
    } else {
      C ut = u[0] * C(t[0]) + u[1] * C(t[1]) + u[2] * C(t[2]);
      C Nt = 0;
#pragma unroll
      for (int k = 0; k < 19; k++) {
        int ek[3] = {EX[k], EY[k], EZ[k]};
        if (ek[ax] != 0) continue;
        int et = ek[0] * t[0] + ek[1] * t[1] + ek[2] * t[2];
        if (et != 0) Nt += C(et) * g[k];
      }
      Nt = C(0.5) * Nt - rho / C(3) * ut;
      val = g[OPP[j]] + rho / C(6) * (un + ut) - Nt;
    }
    g[j] = val;
  }
}

// Streamed populations of a boundary record: plain pulls (periodic wrap),
// interpolated bounce-back on wall links (Eq. bbouzidi, modes fixed on the
// host), Zou-He for the populations entering through an open face.
template <class S>
__device__ void pull_general(const FluidArgs& a, int r, typename Store<S>::C (&g)[19]) {
  typedef typename Store<S>::C C;
  const Grid& G = a.g;
  const long long node = a.rec_node[r];
  int x, y, z;
  coords(G, node, x, y, z);
  const uint32_t mask = a.rec_mask[r];
  int lk = a.rec_link0[r];
  const int fc = a.rec_face[r];
  const int face = fc & 7, kind = (fc >> 4) & 1;
  const int ax = face >> 1, s = (face & 1) ? -1 : 1;
  g[0] = ldA<S>(a, 0, node);
#pragma unroll
  for (int j = 1; j < 19; j++) {
    if (mask & (1u << j)) {
      const int i = OPP[j];
      const uint8_t dm = a.lk_dm[lk];
      const C q = (C)a.lk_q[lk];
      ++lk;
      const int mode = dm >> 5;
      const C fi_x = ldA<S>(a, i, node);
      C v;
      if (mode == BFL_BB) {
        v = fi_x;
      } else if (mode == BFL_LIN_HI) {
        v = fi_x / (C(2) * q) + (C(2) * q - C(1)) / (C(2) * q) * ldA<S>(a, j, node);
      } else {
        const long long n1 = nbr(G, x, y, z, EX[j], EY[j], EZ[j]);  // x - e_i
        if (mode == BFL_QUAD_LO) {
          const long long n2 = nbr(G, x, y, z, 2 * EX[j], 2 * EY[j], 2 * EZ[j]);
          v = q * (C(1) + C(2) * q) * fi_x + (C(1) - C(4) * q * q) * ldA<S>(a, i, n1) -
              q * (C(1) - C(2) * q) * ldA<S>(a, i, n2);
        } else if (mode == BFL_LIN_LO) {
          v = C(2) * q * fi_x + (C(1) - C(2) * q) * ldA<S>(a, i, n1);
        } else {  // BFL_QUAD_HI
          v = fi_x / (q * (C(2) * q + C(1))) + (C(2) * q - C(1)) / q * ldA<S>(a, j, node) +
              (C(1) - C(2) * q) / (C(1) + C(2) * q) * ldA<S>(a, j, n1);
        }
      }
      g[j] = v;
    } else {
      int e[3] = {EX[j], EY[j], EZ[j]};
      if (fc != 0xff && s * e[ax] == 1) {
        g[j] = 0;  // unknown: Zou-He below
      } else {
        g[j] = ldA<S>(a, j, nbr(G, x, y, z, -EX[j], -EY[j], -EZ[j]));
      }
    }
  }
  if (fc != 0xff) {
    zouhe<C>(g, face, kind, (C)a.rec_bc[r], (C)a.rec_bc[a.nrec + r], (C)a.rec_bc[2 * a.nrec + r],
             (C)a.rec_bc[3 * a.nrec + r]);
  }
}

// Streamed populations at any non-solid node.
template <class S>
__device__ __forceinline__ void pull_node(const FluidArgs& a, long long node,
                                          typename Store<S>::C (&g)[19]) {
  if (a.ncls[node] == CLS_BULK) {
    const Grid& G = a.g;
#pragma unroll
    for (int j = 0; j < 19; j++) {
      long long off = EX[j] + (long long)G.px * (EY[j] + (long long)G.ny * EZ[j]);
      g[j] = ldA<S>(a, j, node - off);
    }
  } else {
    pull_general<S>(a, a.rec_of[node], g);
  }
}

template <class C>
__device__ __forceinline__ void node_force(const FluidArgs& a, long long node, bool flagged, C& Fx,
                                           C& Fy, C& Fz) {
  double fx = a.gx, fy = a.gy, fz = a.gz;
  if (flagged) {
    fx += (double)a.fx[node] * FX_INV;
    fy += (double)a.fx[a.g.Np + node] * FX_INV;
    fz += (double)a.fx[2 * a.g.Np + node] * FX_INV;
  }
  Fx = (C)fx;
  Fy = (C)fy;
  Fz = (C)fz;
}

// ------------------------------------------------------------- k_fluid
template <class S>
__device__ void fluid_bulk(const FluidArgs& a, int blk) {
  typedef typename Store<S>::C C;
  constexpr int V = Store<S>::V;
  typedef typename Store<S>::vec vec;
  typedef typename Store<S>::vecu vecu;
  const Grid& G = a.g;
  const long long tile = a.tile_list[blk];
  const long long base = tile * (256LL * V) + (long long)threadIdx.x * V;
  if (base >= G.Np) return;
  uint8_t cls[V];
  bool all = true, any = false;
#pragma unroll
  for (int k = 0; k < V; k++) {
    cls[k] = a.ncls[base + k];
    all = all && cls[k] == CLS_BULK;
    any = any || cls[k] == CLS_BULK;
  }
  if (!any) return;
  const bool flagged = a.tflag && a.tflag[base >> TILE_SHIFT];
  const S* A = (const S*)a.A;
  S* B = (S*)a.B;
  const C omega = (C)a.omega;
  if (all) {
    vec in[19];
#pragma unroll
    for (int j = 0; j < 19; j++) {
      const long long off = EX[j] + (long long)G.px * (EY[j] + (long long)G.ny * EZ[j]);
      const S* p = A + (long long)j * G.plane + base - off;
      if (EX[j] == 0) in[j] = *(const vec*)p;
      else in[j] = *(const vecu*)p;
    }
    bool bad = false;
#pragma unroll
    for (int k = 0; k < V; k++) {
      C g[19];
#pragma unroll
      for (int j = 0; j < 19; j++) g[j] = to_c(in[j][k]);
      C Fx, Fy, Fz, rho, ux, uy, uz;
      node_force<C>(a, base + k, flagged, Fx, Fy, Fz);
      collide<C>(g, Fx, Fy, Fz, omega, rho, ux, uy, uz);
      bad = bad || !(ux * ux + uy * uy + uz * uz <= C(0.09));
#pragma unroll
      for (int j = 0; j < 19; j++) in[j][k] = (S)g[j];
    }
#pragma unroll
    for (int j = 0; j < 19; j++) *(vec*)(B + (long long)j * G.plane + base) = in[j];
    if (bad) atomicOr(&a.flags->pending, ST_UNSTABLE);
  } else {
    bool bad = false;
    for (int k = 0; k < V; k++) {
      if (cls[k] != CLS_BULK) continue;
      const long long node = base + k;
      C g[19];
#pragma unroll
      for (int j = 0; j < 19; j++) {
        const long long off = EX[j] + (long long)G.px * (EY[j] + (long long)G.ny * EZ[j]);
        g[j] = to_c(A[(long long)j * G.plane + node - off]);
      }
      C Fx, Fy, Fz, rho, ux, uy, uz;
      node_force<C>(a, node, flagged, Fx, Fy, Fz);
      collide<C>(g, Fx, Fy, Fz, omega, rho, ux, uy, uz);
      bad = bad || !(ux * ux + uy * uy + uz * uz <= C(0.09));
#pragma unroll
      for (int j = 0; j < 19; j++) B[(long long)j * G.plane + node] = (S)g[j];
    }
    if (bad) atomicOr(&a.flags->pending, ST_UNSTABLE);
  }
}

template <class S>
__device__ void fluid_record(const FluidArgs& a, int r) {
  typedef typename Store<S>::C C;
  C g[19];
  pull_general<S>(a, r, g);
  const long long node = a.rec_node[r];
  const bool flagged = a.tflag && a.tflag[node >> TILE_SHIFT];
  C Fx, Fy, Fz, rho, ux, uy, uz;
  node_force<C>(a, node, flagged, Fx, Fy, Fz);
  collide<C>(g, Fx, Fy, Fz, (C)a.omega, rho, ux, uy, uz);
  S* B = (S*)a.B;
#pragma unroll
  for (int j = 0; j < 19; j++) B[(long long)j * a.g.plane + node] = (S)g[j];
  if (!(ux * ux + uy * uy + uz * uz <= C(0.09))) atomicOr(&a.flags->pending, ST_UNSTABLE);
}

template <class S>
__global__ __launch_bounds__(256) void k_fluid(FluidArgs a) {
  if (a.flags->stop) return;
  const int b = blockIdx.x;
  if (b < a.nbulk_blocks) {
    fluid_bulk<S>(a, xcd_remap(b, a.nbulk_blocks));
  } else {
    const int r = (b - a.nbulk_blocks) * 256 + threadIdx.x;
    if (r < a.nrec) fluid_record<S>(a, r);
  }
}

// ---------------------------------------------------------------- init
template <class S>
__global__ void k_init(Grid G, S* f, const uint8_t* ncls, const double* rho0, const double* u0) {
  long long n = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (n >= (long long)G.nx * G.ny * G.nz) return;
  int x = (int)(n % G.nx);
  long long t = n / G.nx;
  int y = (int)(t % G.ny), z = (int)(t / G.ny);
  long long p = x + (long long)G.px * (y + (long long)G.ny * z);
  const long long N = (long long)G.nx * G.ny * G.nz;
  double r = rho0 ? rho0[n] : 1.0;
  double ux = u0 ? u0[n] : 0.0, uy = u0 ? u0[N + n] : 0.0, uz = u0 ? u0[2 * N + n] : 0.0;
  bool solid = ncls[p] == CLS_SOLID;
  double usq = ux * ux + uy * uy + uz * uz;
  for (int i = 0; i < 19; i++) {
    double eu = EX[i] * ux + EY[i] * uy + EZ[i] * uz;
    double geq = WD[i] * ((r - 1.0) + r * (3.0 * eu + 4.5 * eu * eu - 1.5 * usq));
    f[(long long)i * G.plane + p] = solid ? (S)0 : (S)geq;
  }
}

// -------------------------------------------------------------------- MLS
// 32 lanes per point; lane k < 27 owns the stencil node b + (k%3-1,
// (k/3)%3-1, k/9-1) with b = floor(p + 1/2) (Eqs. uLag, l2norm, intKernel):
// W = exp(-(r/0.3)^2), r = |x_k - p| / 2.6, linear basis (1, x_k - p); solid
// nodes and nodes outside a non-periodic face are excluded.
struct Slot {
  long long node;
  double W, dx, dy, dz;
  bool valid;
};

__device__ __forceinline__ Slot stencil_slot(const Grid& G, const uint8_t* ncls, double X,
                                             double Y, double Z, int k) {
  Slot s;
  s.valid = false;
  s.W = 0.0;
  s.node = 0;
  s.dx = s.dy = s.dz = 0.0;
  if (k >= 27) return s;
  const int bx = (int)floor(X + 0.5), by = (int)floor(Y + 0.5), bz = (int)floor(Z + 0.5);
  int c[3] = {bx + k % 3 - 1, by + (k / 3) % 3 - 1, bz + k / 9 - 1};
  s.dx = c[0] - X;
  s.dy = c[1] - Y;
  s.dz = c[2] - Z;
  const int dim[3] = {G.nx, G.ny, G.nz};
  bool ok = true;
#pragma unroll
  for (int a = 0; a < 3; a++) {
    if (c[a] < 0 || c[a] >= dim[a]) {
      if (G.per[a]) c[a] = ((c[a] % dim[a]) + dim[a]) % dim[a];
      else ok = false;
    }
  }
  if (ok) {
    s.node = c[0] + (long long)G.px * (c[1] + (long long)G.ny * c[2]);
    ok = ncls[s.node] != CLS_SOLID;
  }
  const double r = sqrt(s.dx * s.dx + s.dy * s.dy + s.dz * s.dz) / 2.6;
  s.W = (ok && r <= 1.0) ? exp(-(r / 0.3) * (r / 0.3)) : 0.0;
  s.valid = ok;
  return s;
}

__device__ __forceinline__ double red32(double v) {
#pragma unroll
  for (int m = 16; m >= 1; m >>= 1) v += __shfl_xor(v, m, 32);
  return v;
}
__device__ __forceinline__ double red64(double v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
  return v;
}

// Moment matrix A = sum W p p^T over the 32-lane group, Cholesky, and
// psi = W A^{-1} p for this lane (psi[0] = phi).  Singular (pivot below
// 1e-10 of the largest diagonal): psi = 0, returns false.
__device__ bool mls_psi(const Slot& s, double (&psi)[4]) {
  const double P[4] = {1.0, s.dx, s.dy, s.dz};
  double A[4][4];
#pragma unroll
  for (int i = 0; i < 4; i++)
#pragma unroll
    for (int j = i; j < 4; j++) {
      A[i][j] = red32(s.W * P[i] * P[j]);
      A[j][i] = A[i][j];
    }
  double dmax = fmax(fmax(A[0][0], A[1][1]), fmax(A[2][2], A[3][3]));
  double L[4][4] = {{0}};
  bool ok = dmax > 0.0;
#pragma unroll
  for (int j = 0; j < 4; j++) {
    double d = A[j][j];
#pragma unroll
    for (int k = 0; k < j; k++) d -= L[j][k] * L[j][k];
    if (!(d > 1e-10 * dmax)) ok = false;
    L[j][j] = ok ? sqrt(d) : 1.0;
#pragma unroll
    for (int i = j + 1; i < 4; i++) {
      double v = A[i][j];
#pragma unroll
      for (int k = 0; k < j; k++) v -= L[i][k] * L[j][k];
      L[i][j] = v / L[j][j];
    }
  }
  if (!ok) {
    psi[0] = psi[1] = psi[2] = psi[3] = 0.0;
    return false;
  }
  // y = L^{-1} P, psi = W L^{-T} y
  double y[4];
#pragma unroll
  for (int i = 0; i < 4; i++) {
    double v = P[i];
#pragma unroll
    for (int k = 0; k < i; k++) v -= L[i][k] * y[k];
    y[i] = v / L[i][i];
  }
  double z[4];
#pragma unroll
  for (int i = 3; i >= 0; i--) {
    double v = y[i];
#pragma unroll
    for (int k = i + 1; k < 4; k++) v -= L[k][i] * z[k];
    z[i] = v / L[i][i];
  }
#pragma unroll
  for (int i = 0; i < 4; i++) psi[i] = s.W * z[i];
  return true;
}

// Post-collision macroscopic fields at a node: rho = sum f*, and the
// velocity of the step u = (sum f* e - F/2)/rho (the collision adds F to the
// momentum).
template <class S>
__device__ __forceinline__ void macro_at(const Grid& G, const S* f, const long long* fx,
                                         const uint8_t* tf, double gx, double gy, double gz,
                                         long long node, double& rho, double& ux, double& uy,
                                         double& uz) {
  typedef typename Store<S>::C C;
  C g[19];
#pragma unroll
  for (int j = 0; j < 19; j++) g[j] = to_c(f[(long long)j * G.plane + node]);
  C drho = 0;
#pragma unroll
  for (int j = 0; j < 19; j++) drho += g[j];
  C mx = (g[1] - g[2]) + (g[7] + g[8]) + (g[9] + g[10]) - (g[11] + g[12]) - (g[13] + g[14]);
  C my = (g[3] - g[4]) + (g[7] - g[8]) + (g[11] - g[12]) + (g[15] + g[16]) - (g[17] + g[18]);
  C mz = (g[5] - g[6]) + (g[9] - g[10]) + (g[13] - g[14]) + (g[15] - g[16]) + (g[17] - g[18]);
  double Fx = gx, Fy = gy, Fz = gz;
  if (fx && tf && tf[node >> TILE_SHIFT]) {
    Fx += (double)fx[node] * FX_INV;
    Fy += (double)fx[G.Np + node] * FX_INV;
    Fz += (double)fx[2 * G.Np + node] * FX_INV;
  }
  rho = 1.0 + (double)drho;
  ux = ((double)mx - 0.5 * Fx) / rho;
  uy = ((double)my - 0.5 * Fy) / rho;
  uz = ((double)mz - 0.5 * Fz) / rho;
}

__device__ __forceinline__ void face_geom(const double* X, const int32_t* faces, int f,
                                          double (&c)[3], double (&n)[3], double& area) {
  const int a = faces[3 * f], b = faces[3 * f + 1], d = faces[3 * f + 2];
  double pa[3], pb[3], pd[3];
#pragma unroll
  for (int k = 0; k < 3; k++) {
    pa[k] = X[3 * a + k];
    pb[k] = X[3 * b + k];
    pd[k] = X[3 * d + k];
  }
  double u[3] = {pb[0] - pa[0], pb[1] - pa[1], pb[2] - pa[2]};
  double v[3] = {pd[0] - pa[0], pd[1] - pa[1], pd[2] - pa[2]};
  double N[3] = {u[1] * v[2] - u[2] * v[1], u[2] * v[0] - u[0] * v[2], u[0] * v[1] - u[1] * v[0]};
  double l = sqrt(N[0] * N[0] + N[1] * N[1] + N[2] * N[2]);
#pragma unroll
  for (int k = 0; k < 3; k++) {
    c[k] = (pa[k] + pb[k] + pd[k]) / 3.0;
    n[k] = N[k] / l;
  }
  area = 0.5 * l;
}

// ---------------------------------------------------------- k_ib_force
// Direct forcing at the face centroids: U = sum phi u* with u* = sum f e / rho
// of the streamed populations (no force), F_l = U_b - U, spread of
// c_l phi_k F_l with c_l the face area.
template <class S>
__global__ __launch_bounds__(256) void k_ib_force(FluidArgs a, BodyArgs b, long long* fxc,
                                                  uint8_t* tfc, long long* fxp, uint8_t* tfp) {
  typedef typename Store<S>::C C;
  if (a.flags->stop) return;
  const int lane = threadIdx.x & 31;
  const int m = (blockIdx.x * 256 + threadIdx.x) >> 5;
  if (m >= b.nf) return;
  const Grid& G = a.g;
  // clear the previous step's spread buffer at the previous stencil
  const int pbx = b.base_prev[3 * m];
  if (pbx != INT_MIN && lane < 27) {
    int c[3] = {pbx + lane % 3 - 1, b.base_prev[3 * m + 1] + (lane / 3) % 3 - 1,
                b.base_prev[3 * m + 2] + lane / 9 - 1};
    const int dim[3] = {G.nx, G.ny, G.nz};
    bool ok = true;
    for (int k = 0; k < 3; k++) {
      if (c[k] < 0 || c[k] >= dim[k]) {
        if (G.per[k]) c[k] = ((c[k] % dim[k]) + dim[k]) % dim[k];
        else ok = false;
      }
    }
    if (ok) {
      long long node = c[0] + (long long)G.px * (c[1] + (long long)G.ny * c[2]);
      fxp[node] = 0;
      fxp[G.Np + node] = 0;
      fxp[2 * G.Np + node] = 0;
      tfp[node >> TILE_SHIFT] = 0;
    }
  }
  double cen[3], nrm[3], area;
  face_geom(b.Xcur, b.faces, m, cen, nrm, area);
  if (lane == 0) {
    b.centroid[3 * m] = cen[0];
    b.centroid[3 * m + 1] = cen[1];
    b.centroid[3 * m + 2] = cen[2];
    b.base_cur[3 * m] = (int)floor(cen[0] + 0.5);
    b.base_cur[3 * m + 1] = (int)floor(cen[1] + 0.5);
    b.base_cur[3 * m + 2] = (int)floor(cen[2] + 0.5);
  }
  const Slot s = stencil_slot(G, a.ncls, cen[0], cen[1], cen[2], lane);
  double us[3] = {0.0, 0.0, 0.0};
  if (s.valid) {
    C g[19];
    pull_node<S>(a, s.node, g);
    C drho = 0;
#pragma unroll
    for (int j = 0; j < 19; j++) drho += g[j];
    C mx = (g[1] - g[2]) + (g[7] + g[8]) + (g[9] + g[10]) - (g[11] + g[12]) - (g[13] + g[14]);
    C my = (g[3] - g[4]) + (g[7] - g[8]) + (g[11] - g[12]) + (g[15] + g[16]) - (g[17] + g[18]);
    C mz = (g[5] - g[6]) + (g[9] - g[10]) + (g[13] - g[14]) + (g[15] - g[16]) + (g[17] - g[18]);
    double rho = 1.0 + (double)drho;
    us[0] = (double)mx / rho;
    us[1] = (double)my / rho;
    us[2] = (double)mz / rho;
  }
  double psi[4];
  const bool ok = mls_psi(s, psi);
  if (!ok && lane == 0) atomicAdd(&a.flags->mls_singular, 1);
  double U[3];
#pragma unroll
  for (int k = 0; k < 3; k++) U[k] = red32(psi[0] * us[k]);
  // marker velocity
  const int body = b.face_body[m];
  double Ub[3];
  if (b.b_rigid[body]) {
    const double* rs = b.b_rig + 32 * body;
    double r[3] = {cen[0] - rs[0], cen[1] - rs[1], cen[2] - rs[2]};
    const double* w = rs + 9;
    Ub[0] = rs[3] + (w[1] * r[2] - w[2] * r[1]);
    Ub[1] = rs[4] + (w[2] * r[0] - w[0] * r[2]);
    Ub[2] = rs[5] + (w[0] * r[1] - w[1] * r[0]);
  } else {
    const int v0 = b.faces[3 * m], v1 = b.faces[3 * m + 1], v2 = b.faces[3 * m + 2];
#pragma unroll
    for (int k = 0; k < 3; k++)
      Ub[k] = (b.Vel[3 * v0 + k] + b.Vel[3 * v1 + k] + b.Vel[3 * v2 + k]) / 3.0;
  }
  if (s.valid && psi[0] != 0.0) {
    const double cp = area * psi[0];
    fx_add(fxc + s.node, cp * (Ub[0] - U[0]), a.flags);
    fx_add(fxc + G.Np + s.node, cp * (Ub[1] - U[1]), a.flags);
    fx_add(fxc + 2 * G.Np + s.node, cp * (Ub[2] - U[2]), a.flags);
    tfc[s.node >> TILE_SHIFT] = 1;
  }
}

// ---------------------------------------------------------- k_mls_post
// Faces (one wave each; lanes 0-31 the outer probe, 32-63 the inner one):
// pressure p = rho/3 and viscous stress rho nu (grad u + grad u^T) from MLS
// fits 1.2 dx along +-n (Eqs. hydroForP, hydroForNu), plus the repulsion of
// centroids of other bodies closer than dx (Eq. collision).  Soft vertices
// (two per wave): MLS velocity u_v,0 at x_v^n.
template <class S>
__global__ __launch_bounds__(256) void k_mls_post(FluidArgs a, BodyArgs b) {
  if (a.flags->stop) return;
  const int wave = (blockIdx.x * 256 + threadIdx.x) >> 6;
  const int l64 = threadIdx.x & 63, half = l64 >> 5, lane = l64 & 31;
  const Grid& G = a.g;
  const S* f = (const S*)a.B;
  if (wave < b.nf) {
    const int m = wave;
    double cen[3], nrm[3], area;
    face_geom(b.Xcur, b.faces, m, cen, nrm, area);
    const double sg = half == 0 ? 1.2 : -1.2;
    const Slot s = stencil_slot(G, a.ncls, cen[0] + sg * nrm[0], cen[1] + sg * nrm[1],
                                cen[2] + sg * nrm[2], lane);
    double rho = 0.0, u[3] = {0.0, 0.0, 0.0};
    if (s.valid) macro_at<S>(G, f, a.fx, a.tflag, a.gx, a.gy, a.gz, s.node, rho, u[0], u[1], u[2]);
    double psi[4];
    if (!mls_psi(s, psi) && lane == 0) atomicAdd(&a.flags->mls_singular, 1);
    double rfit = red32(psi[0] * rho);
    double Gm[3][3];
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
      for (int c = 0; c < 3; c++) Gm[i][c] = red32(psi[1 + c] * u[i]);
    // outer minus inner, on lane 0
    const double r_in = __shfl(rfit, 32, 64);
    double Gin[3][3];
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
      for (int c = 0; c < 3; c++) Gin[i][c] = __shfl(Gm[i][c], 32, 64);
    // repulsion from the other bodies
    const int body = b.face_body[m];
    double acc = 0.0;
    if (b.nbody > 1) {
      const double* bb = b.b_diag + 16 * body + 2;
      for (int o = 0; o < b.nbody; o++) {
        if (o == body) continue;
        const double* ob = b.b_diag + 16 * o + 2;
        bool far = false;
#pragma unroll
        for (int k = 0; k < 3; k++)
          if (bb[k] > ob[3 + k] + 1.0 || ob[k] > bb[3 + k] + 1.0) far = true;
        if (far) continue;
        const int f0 = b.b_face0[o], nf = b.b_nf[o];
        for (int g2 = l64; g2 < nf; g2 += 64) {
          const double* cj = b.centroid + 3 * (f0 + g2);
          const double dx = cen[0] - cj[0], dy = cen[1] - cj[1], dz = cen[2] - cj[2];
          const double d = sqrt(dx * dx + dy * dy + dz * dz);
          if (d < 1.0 && d > 0.0) acc += 1.0 / sqrt(d * d * d * d * d);
        }
      }
      acc = red64(acc);
    }
    if (l64 == 0) {
      const double nu = b.nu;
      const double dp = (rfit - r_in) / 3.0;
      double F[3];
#pragma unroll
      for (int i = 0; i < 3; i++) {
        double tn = 0.0;
#pragma unroll
        for (int c = 0; c < 3; c++) {
          const double tp = rfit * nu * (Gm[i][c] + Gm[c][i]);
          const double tm = r_in * nu * (Gin[i][c] + Gin[c][i]);
          tn += (tp - tm) * nrm[c];
        }
        F[i] = (-dp * nrm[i] + tn) * area;
      }
      const double pref = b.umax / (8.0 * sqrt(2.0));
#pragma unroll
      for (int i = 0; i < 3; i++) b.fext[3 * m + i] = F[i] - pref * acc * nrm[i];
    }
  } else {
    const int idx = (wave - b.nf) * 2 + half;
    if (idx >= b.nsoft_v) return;
    const int v = b.soft_vlist[idx];
    const double X = b.Xcur[3 * v], Y = b.Xcur[3 * v + 1], Z = b.Xcur[3 * v + 2];
    const Slot s = stencil_slot(G, a.ncls, X, Y, Z, lane);
    double rho = 0.0, u[3] = {0.0, 0.0, 0.0};
    if (s.valid) macro_at<S>(G, f, a.fx, a.tflag, a.gx, a.gy, a.gz, s.node, rho, u[0], u[1], u[2]);
    double psi[4];
    if (!mls_psi(s, psi) && lane == 0) atomicAdd(&a.flags->mls_singular, 1);
    double U[3];
#pragma unroll
    for (int k = 0; k < 3; k++) U[k] = red32(psi[0] * u[k]);
    if (lane == 0) {
      b.u0v[3 * v] = U[0];
      b.u0v[3 * v + 1] = U[1];
      b.u0v[3 * v + 2] = U[2];
    }
  }
}

// ----------------------------------------------------------- k_body_post
__device__ __forceinline__ void cross3(const double* a, const double* b, double* c) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}

// Gradient of the signed dihedral angle of hinge (a, b, c, d) (faces (a,b,c)
// and (b,a,d), outward normals) with respect to the vertex in `role`.
__device__ void hinge_grad(const double* X, const int32_t* h, int role, double& theta,
                           double (&gr)[3]) {
  const double* pa = X + 3 * h[0];
  const double* pb = X + 3 * h[1];
  const double* pc = X + 3 * h[2];
  const double* pd = X + 3 * h[3];
  double e[3], ca[3], da[3], ab[3], db[3], n1[3], n2[3];
  for (int k = 0; k < 3; k++) {
    e[k] = pb[k] - pa[k];
    ca[k] = pc[k] - pa[k];
    da[k] = pd[k] - pa[k];
    ab[k] = pa[k] - pb[k];
    db[k] = pd[k] - pb[k];
  }
  cross3(e, ca, n1);
  cross3(ab, db, n2);
  const double q1 = n1[0] * n1[0] + n1[1] * n1[1] + n1[2] * n1[2];
  const double q2 = n2[0] * n2[0] + n2[1] * n2[1] + n2[2] * n2[2];
  const double le2 = e[0] * e[0] + e[1] * e[1] + e[2] * e[2];
  const double le = sqrt(le2);
  const double l1 = sqrt(q1), l2 = sqrt(q2);
  double m1[3], m2[3], t[3];
  for (int k = 0; k < 3; k++) {
    m1[k] = n1[k] / l1;
    m2[k] = n2[k] / l2;
  }
  cross3(m1, m2, t);
  theta = atan2((t[0] * e[0] + t[1] * e[1] + t[2] * e[2]) / le,
                m1[0] * m2[0] + m1[1] * m2[1] + m1[2] * m2[2]);
  const double al_c = (ca[0] * e[0] + ca[1] * e[1] + ca[2] * e[2]) / le2;
  const double al_d = (da[0] * e[0] + da[1] * e[1] + da[2] * e[2]) / le2;
  for (int k = 0; k < 3; k++) {
    const double gc = -le * n1[k] / q1;
    const double gd = -le * n2[k] / q2;
    if (role == 0) gr[k] = -((1.0 - al_c) * gc + (1.0 - al_d) * gd);
    else if (role == 1) gr[k] = -(al_c * gc + al_d * gd);
    else if (role == 2) gr[k] = gc;
    else gr[k] = gd;
  }
}

__device__ __forceinline__ double block_sum(double v, double* sh) {
  // deterministic: fixed lane tree in each wave, then fixed order over waves
  v = red64(v);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[w] = v;
  __syncthreads();
  double t = 0.0;
  for (int k = 0; k < (int)(blockDim.x >> 6); k++) t += sh[k];
  return t;
}

__device__ void rodrigues(const double* phi, double* R) {
  const double th = sqrt(phi[0] * phi[0] + phi[1] * phi[1] + phi[2] * phi[2]);
  if (th == 0.0) {
    for (int k = 0; k < 9; k++) R[k] = (k % 4 == 0) ? 1.0 : 0.0;
    return;
  }
  const double k0 = phi[0] / th, k1 = phi[1] / th, k2 = phi[2] / th;
  const double c = cos(th), sn = sin(th), omc = 2.0 * sin(0.5 * th) * sin(0.5 * th);
  const double kk[3] = {k0, k1, k2};
  const double K[9] = {0, -k2, k1, k2, 0, -k0, -k1, k0, 0};
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) R[3 * i + j] = (i == j ? c : 0.0) + sn * K[3 * i + j] + omc * kk[i] * kk[j];
}

__device__ double det3(const double* A) {
  return A[0] * (A[4] * A[8] - A[5] * A[7]) - A[1] * (A[3] * A[8] - A[5] * A[6]) +
         A[2] * (A[3] * A[7] - A[4] * A[6]);
}

__global__ __launch_bounds__(256) void k_body_post(BodyArgs b, DevFlags* flags) {
  if (flags->stop) return;
  __shared__ double sh[8];
  __shared__ double rs[32];
  const int blk = blockIdx.x;
  if (blk < b.nbody) {
    // rigid (or fixed) body: one block
    if (!b.b_rigid[blk]) return;
    const int v0 = b.b_vert0[blk], nv = b.b_nv[blk];
    double* st = b.b_rig + 32 * blk;
    if (b.b_fixed[blk]) {
      for (int v = threadIdx.x; v < nv; v += blockDim.x)
        for (int k = 0; k < 3; k++) {
          b.Xnext[3 * (v0 + v) + k] = b.Xcur[3 * (v0 + v) + k];
          b.Vel[3 * (v0 + v) + k] = 0.0;
        }
      return;
    }
    const int f0 = b.b_face0[blk], nf = b.b_nf[blk];
    double F[3] = {0, 0, 0}, M[3] = {0, 0, 0};
    const double xc[3] = {st[0], st[1], st[2]};
    for (int f = threadIdx.x; f < nf; f += blockDim.x) {
      const double* Ff = b.fext + 3 * (f0 + f);
      for (int k = 0; k < 3; k++) F[k] += Ff[k];
      for (int c = 0; c < 3; c++) {
        const int v = b.faces[3 * (f0 + f) + c];
        double r[3] = {b.Xcur[3 * v] - xc[0], b.Xcur[3 * v + 1] - xc[1], b.Xcur[3 * v + 2] - xc[2]};
        double t[3];
        double Fv[3] = {Ff[0] / 3.0, Ff[1] / 3.0, Ff[2] / 3.0};
        cross3(r, Fv, t);
        for (int k = 0; k < 3; k++) M[k] += t[k];
      }
    }
    for (int k = 0; k < 3; k++) {
      F[k] = block_sum(F[k], sh);
      M[k] = block_sum(M[k], sh);
    }
    if (threadIdx.x == 0) {
      // state: x_c 0-2, u 3-5, u_prev 6-8, omega 9-11, omega_prev 12-14, R 15-23
      const double* R = st + 15;
      const double mass = b.b_param[8 * blk + 4];
      double RI[9], Iw[9];
      double Ibm[9];  // body-frame inertia tensor, stored after the [nbody][8] parameters
      for (int k = 0; k < 9; k++) Ibm[k] = b.b_param[8 * b.nbody + 9 * blk + k];
      for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
          double v = 0.0;
          for (int k = 0; k < 3; k++) v += R[3 * i + k] * Ibm[3 * k + j];
          RI[3 * i + j] = v;
        }
      for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
          double v = 0.0;
          for (int k = 0; k < 3; k++) v += RI[3 * i + k] * R[3 * j + k];
          Iw[3 * i + j] = v;
        }
      double al[3];
      const double dI = det3(Iw);
      for (int c = 0; c < 3; c++) {
        double Mm[9];
        for (int k = 0; k < 9; k++) Mm[k] = Iw[k];
        for (int r = 0; r < 3; r++) Mm[3 * r + c] = M[r];
        al[c] = det3(Mm) / dI;
      }
      double un[3], wn[3];
      for (int k = 0; k < 3; k++) {
        un[k] = 2.0 / 3.0 * (2.0 * st[3 + k] - 0.5 * st[6 + k] + F[k] / mass);
        wn[k] = 2.0 / 3.0 * (2.0 * st[9 + k] - 0.5 * st[12 + k] + al[k]);
      }
      for (int k = 0; k < 3; k++) {
        st[6 + k] = st[3 + k];
        st[3 + k] = un[k];
        st[12 + k] = st[9 + k];
        st[9 + k] = wn[k];
        st[k] += un[k];
      }
      double Rr[9], Rn[9];
      rodrigues(wn, Rr);
      for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
          double v = 0.0;
          for (int k = 0; k < 3; k++) v += Rr[3 * i + k] * R[3 * k + j];
          Rn[3 * i + j] = v;
        }
      for (int k = 0; k < 9; k++) st[15 + k] = Rn[k];
      for (int k = 0; k < 24; k++) rs[k] = st[k];
    }
    __syncthreads();
    for (int v = threadIdx.x; v < nv; v += blockDim.x) {
      const double* Xb = b.Xbody + 3 * (v0 + v);
      double r[3], wr[3];
      for (int i = 0; i < 3; i++) r[i] = rs[15 + 3 * i] * Xb[0] + rs[15 + 3 * i + 1] * Xb[1] + rs[15 + 3 * i + 2] * Xb[2];
      cross3(rs + 9, r, wr);
      for (int k = 0; k < 3; k++) {
        b.Xnext[3 * (v0 + v) + k] = rs[k] + r[k];
        b.Vel[3 * (v0 + v) + k] = rs[3 + k] + wr[k];
      }
    }
    return;
  }
  // soft vertices: membrane forces + Verlet (Eqs. verletPos, verletVel, verletPosC)
  const int idx = (blk - b.nbody) * 256 + threadIdx.x;
  if (idx >= b.nsoft_v) return;
  const int v = b.soft_vlist[idx];
  const int body = b.vert_body[v];
  const double* x = b.Xcur;
  const double xv[3] = {x[3 * v], x[3 * v + 1], x[3 * v + 2]};
  double F[3] = {0.0, 0.0, 0.0};
  // stretching: F_v = -k (l - l0) (x_v - x_w) / l
  for (int p = b.ve_ptr[v]; p < b.ve_ptr[v + 1]; p++) {
    const int e = b.ve_idx[p];
    const int w = b.edges[2 * e] == v ? b.edges[2 * e + 1] : b.edges[2 * e];
    double r[3] = {xv[0] - x[3 * w], xv[1] - x[3 * w + 1], xv[2] - x[3 * w + 2]};
    const double l = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
    const double c = -b.kl[e] * (l - b.l0[e]) / l;
    for (int k = 0; k < 3; k++) F[k] += c * r[k];
  }
  // bending: F = -k_b sin(theta - theta0) dtheta/dx
  for (int p = b.vh_ptr[v]; p < b.vh_ptr[v + 1]; p++) {
    const int hr = b.vh_idx[p];
    const int h = hr >> 2, role = hr & 3;
    double th, gr[3];
    hinge_grad(x, b.hinges + 4 * h, role, th, gr);
    const double amp = -b.kb[h] * sin(th - b.theta0[h]);
    for (int k = 0; k < 3; k++) F[k] += amp * gr[k];
  }
  // volume penalty k_v (1 - V/V0) A n / 3 and one third of each face's
  // hydrodynamic + repulsion force
  const double V0 = b.b_param[8 * body], kv = b.b_param[8 * body + 2];
  const double Vc = b.b_diag[16 * body];
  const double cv = kv * (1.0 - Vc / V0);
  for (int p = b.vf_ptr[v]; p < b.vf_ptr[v + 1]; p++) {
    const int f = b.vf_idx[p];
    double c[3], n[3], area;
    face_geom(x, b.faces, f, c, n, area);
    for (int k = 0; k < 3; k++) F[k] += (cv * area * n[k] + b.fext[3 * f + k]) / 3.0;
  }
  const double mv = b.b_param[8 * body + 3];
  for (int k = 0; k < 3; k++) {
    const double acc = 0.5 * F[k] / mv;
    const double xt = xv[k] + b.u0v[3 * v + k] + acc;
    const double un = 1.5 * xt - 2.0 * xv[k] + 0.5 * b.Xnext[3 * v + k];
    b.Xnext[3 * v + k] = xv[k] + un + acc;
    b.Vel[3 * v + k] = un;
  }
}

// --------------------------------------------------------------- k_diag
// Per body (one block): volume, area, bounding box, largest stretch of the
// new positions; a soft link at twice its rest length raises DAMAGED.  The
// last block to finish closes the step: steps_done += 1 and the bits raised
// during the step become sticky.
__global__ __launch_bounds__(256) void k_diag(BodyArgs b, const double* X, DevFlags* flags,
                                              unsigned int* counter, int count) {
  if (flags->stop) return;
  __shared__ double sh[8];
  __shared__ int last;
  const int blk = blockIdx.x;
  if (blk < b.nbody) {
    const int f0 = b.b_face0[blk], nf = b.b_nf[blk];
    double V = 0.0, S = 0.0;
    for (int f = threadIdx.x; f < nf; f += blockDim.x) {
      const int* F = b.faces + 3 * (f0 + f);
      const double* pa = X + 3 * F[0];
      const double* pb = X + 3 * F[1];
      const double* pc = X + 3 * F[2];
      double bc[3];
      cross3(pb, pc, bc);
      V += (pa[0] * bc[0] + pa[1] * bc[1] + pa[2] * bc[2]) / 6.0;
      double c[3], n[3], area;
      face_geom(X, b.faces, f0 + f, c, n, area);
      S += area;
    }
    V = block_sum(V, sh);
    S = block_sum(S, sh);
    const int v0 = b.b_vert0[blk], nv = b.b_nv[blk];
    double lo[3] = {DBL_MAX, DBL_MAX, DBL_MAX}, hi[3] = {-DBL_MAX, -DBL_MAX, -DBL_MAX};
    bool nan = false;
    for (int v = threadIdx.x; v < nv; v += blockDim.x)
      for (int k = 0; k < 3; k++) {
        const double c = X[3 * (v0 + v) + k];
        nan = nan || !(c == c);
        lo[k] = fmin(lo[k], c);
        hi[k] = fmax(hi[k], c);
      }
    double strain = 0.0;
    const int e0 = b.b_edge0[blk], ne = b.b_ne[blk];
    for (int e = threadIdx.x; e < ne; e += blockDim.x) {
      const int a = b.edges[2 * (e0 + e)], c = b.edges[2 * (e0 + e) + 1];
      double r[3] = {X[3 * a] - X[3 * c], X[3 * a + 1] - X[3 * c + 1], X[3 * a + 2] - X[3 * c + 2]};
      strain = fmax(strain, sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]) / b.l0[e0 + e]);
    }
    // min/max reductions (order independent)
    for (int k = 0; k < 3; k++) {
      for (int m = 32; m >= 1; m >>= 1) {
        lo[k] = fmin(lo[k], __shfl_xor(lo[k], m, 64));
        hi[k] = fmax(hi[k], __shfl_xor(hi[k], m, 64));
      }
    }
    for (int m = 32; m >= 1; m >>= 1) strain = fmax(strain, __shfl_xor(strain, m, 64));
    __shared__ double shm[4][7];
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) {
      for (int k = 0; k < 3; k++) {
        shm[w][k] = lo[k];
        shm[w][3 + k] = hi[k];
      }
      shm[w][6] = strain;
    }
    if (nan) atomicOr(&flags->pending, ST_UNSTABLE);
    __syncthreads();
    if (threadIdx.x == 0) {
      double* d = b.b_diag + 16 * blk;
      for (int k = 0; k < 3; k++) {
        double l = shm[0][k], h = shm[0][3 + k];
        for (int q = 1; q < (int)(blockDim.x >> 6); q++) {
          l = fmin(l, shm[q][k]);
          h = fmax(h, shm[q][3 + k]);
        }
        d[2 + k] = l;
        d[5 + k] = h;
      }
      double s = shm[0][6];
      for (int q = 1; q < (int)(blockDim.x >> 6); q++) s = fmax(s, shm[q][6]);
      d[0] = V;
      d[1] = S;
      d[8] = s;
      if (!b.b_rigid[blk] && s >= 2.0) atomicOr(&flags->pending, ST_DAMAGED);
    }
  }
  // step bookkeeping by the last block to finish
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    const unsigned int done = atomicAdd(counter, 1u);
    last = (done == gridDim.x - 1);
  }
  __syncthreads();
  if (last && threadIdx.x == 0) {
    const unsigned int pend = __hip_atomic_load(&flags->pending, __ATOMIC_RELAXED,
                                                __HIP_MEMORY_SCOPE_AGENT);
    if (count) flags->steps_done += 1;
    flags->stop |= pend;
    flags->pending = 0u;
    *counter = 0u;
  }
}

// ------------------------------------------------------------ API kernels
template <class S>
__global__ void k_get_fields(Grid G, const S* f0, const S* f1, const uint8_t* ncls,
                             const long long* fx0, const long long* fx1, const uint8_t* tf0,
                             const uint8_t* tf1, double gx, double gy, double gz,
                             const DevFlags* flags, double* rho, double* u, double* pops,
                             double* fib) {
  const long long N = (long long)G.nx * G.ny * G.nz;
  long long n = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (n >= N) return;
  const long long sd = flags->steps_done;
  const S* f = (sd & 1) ? f1 : f0;
  const int lp = (int)((sd - 1) & 1);
  const long long* fx = sd > 0 ? (lp ? fx1 : fx0) : nullptr;
  const uint8_t* tf = sd > 0 ? (lp ? tf1 : tf0) : nullptr;
  int x = (int)(n % G.nx);
  long long t = n / G.nx;
  int y = (int)(t % G.ny), z = (int)(t / G.ny);
  long long p = x + (long long)G.px * (y + (long long)G.ny * z);
  const bool solid = ncls[p] == CLS_SOLID;
  double bgx = sd > 0 ? gx : 0.0, bgy = sd > 0 ? gy : 0.0, bgz = sd > 0 ? gz : 0.0;
  if (rho || u) {
    double r = 0, ux = 0, uy = 0, uz = 0;
    if (!solid) macro_at<S>(G, f, fx, tf, bgx, bgy, bgz, p, r, ux, uy, uz);
    if (rho) rho[n] = r;
    if (u) {
      u[n] = ux;
      u[N + n] = uy;
      u[2 * N + n] = uz;
    }
  }
  if (pops)
    for (int i = 0; i < 19; i++)
      pops[(long long)i * N + n] = solid ? 0.0 : (double)to_c(f[(long long)i * G.plane + p]) + WD[i];
  if (fib) {
    const bool fl = fx && tf && tf[p >> TILE_SHIFT];
    for (int c = 0; c < 3; c++) fib[(long long)c * N + n] = fl ? (double)fx[c * G.Np + p] * FX_INV : 0.0;
  }
}

template <class S>
__global__ __launch_bounds__(256) void k_interp(Grid G, const S* f0, const S* f1,
                                                const uint8_t* ncls, const long long* fx0,
                                                const long long* fx1, const uint8_t* tf0,
                                                const uint8_t* tf1, double gx, double gy,
                                                double gz, const DevFlags* flags, long long n,
                                                const double* pts, const double* field,
                                                double* out) {
  const long long m = (blockIdx.x * 256LL + threadIdx.x) >> 5;
  const int lane = threadIdx.x & 31;
  if (m >= n) return;
  const long long N = (long long)G.nx * G.ny * G.nz;
  const Slot s = stencil_slot(G, ncls, pts[3 * m], pts[3 * m + 1], pts[3 * m + 2], lane);
  double u[3] = {0.0, 0.0, 0.0};
  if (s.valid) {
    if (field) {
      int x, y, z;
      coords(G, s.node, x, y, z);
      const long long ln = x + (long long)G.nx * (y + (long long)G.ny * z);
      u[0] = field[ln];
      u[1] = field[N + ln];
      u[2] = field[2 * N + ln];
    } else {
      const long long sd = flags->steps_done;
      const S* f = (sd & 1) ? f1 : f0;
      const int lp = (int)((sd - 1) & 1);
      const long long* fx = sd > 0 ? (lp ? fx1 : fx0) : nullptr;
      const uint8_t* tf = sd > 0 ? (lp ? tf1 : tf0) : nullptr;
      double r;
      macro_at<S>(G, f, fx, tf, sd > 0 ? gx : 0.0, sd > 0 ? gy : 0.0, sd > 0 ? gz : 0.0, s.node,
                  r, u[0], u[1], u[2]);
    }
  }
  double psi[4];
  mls_psi(s, psi);
  double U[3];
  for (int k = 0; k < 3; k++) U[k] = red32(psi[0] * u[k]);
  if (lane == 0)
    for (int k = 0; k < 3; k++) out[3 * m + k] = U[k];
}

__global__ __launch_bounds__(256) void k_spread_api(Grid G, const uint8_t* ncls, long long n,
                                                    const double* pts, const double* F,
                                                    const double* c, long long* fx,
                                                    DevFlags* flags) {
  const long long m = (blockIdx.x * 256LL + threadIdx.x) >> 5;
  const int lane = threadIdx.x & 31;
  if (m >= n) return;
  const Slot s = stencil_slot(G, ncls, pts[3 * m], pts[3 * m + 1], pts[3 * m + 2], lane);
  double psi[4];
  mls_psi(s, psi);
  if (s.valid && psi[0] != 0.0) {
    const double cp = c[m] * psi[0];
    fx_add(fx + s.node, cp * F[3 * m], flags);
    fx_add(fx + G.Np + s.node, cp * F[3 * m + 1], flags);
    fx_add(fx + 2 * G.Np + s.node, cp * F[3 * m + 2], flags);
  }
}

__global__ void k_flush_fx(Grid G, long long* fx, double* fib) {
  const long long N = (long long)G.nx * G.ny * G.nz;
  long long n = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (n >= N) return;
  int x = (int)(n % G.nx);
  long long t = n / G.nx;
  int y = (int)(t % G.ny), z = (int)(t / G.ny);
  long long p = x + (long long)G.px * (y + (long long)G.ny * z);
  for (int c = 0; c < 3; c++) {
    long long v = fx[c * G.Np + p];
    if (v != 0) {
      fib[c * N + n] += (double)v * FX_INV;
      fx[c * G.Np + p] = 0;
    }
  }
}

// --------------------------------------------------------------- launchers
#define DISPATCH(prec, KER, ...)                                 \
  switch (prec) {                                                \
    case 0: KER<double> __VA_ARGS__; break;                      \
    case 1: KER<float> __VA_ARGS__; break;                       \
    default: KER<_Float16> __VA_ARGS__; break;                   \
  }

static inline unsigned cdiv(long long a, long long b) { return (unsigned)((a + b - 1) / b); }

hipError_t launch_init(int prec, const Grid& g, void* f, const uint8_t* ncls, const double* rho,
                       const double* u, hipStream_t s) {
  const long long N = (long long)g.nx * g.ny * g.nz;
  switch (prec) {
    case 0: k_init<double><<<cdiv(N, 256), 256, 0, s>>>(g, (double*)f, ncls, rho, u); break;
    case 1: k_init<float><<<cdiv(N, 256), 256, 0, s>>>(g, (float*)f, ncls, rho, u); break;
    default: k_init<_Float16><<<cdiv(N, 256), 256, 0, s>>>(g, (_Float16*)f, ncls, rho, u); break;
  }
  return hipGetLastError();
}

hipError_t launch_fluid(int prec, const FluidArgs& a, hipStream_t s) {
  const unsigned grid = (unsigned)a.nbulk_blocks + cdiv(a.nrec, 256);
  if (grid == 0) return hipSuccess;
  switch (prec) {
    case 0: k_fluid<double><<<grid, 256, 0, s>>>(a); break;
    case 1: k_fluid<float><<<grid, 256, 0, s>>>(a); break;
    default: k_fluid<_Float16><<<grid, 256, 0, s>>>(a); break;
  }
  return hipGetLastError();
}

hipError_t launch_ib_force(int prec, const FluidArgs& a, const BodyArgs& b, long long* fxc,
                           uint8_t* tfc, long long* fxp, uint8_t* tfp, hipStream_t s) {
  if (b.nf == 0) return hipSuccess;
  const unsigned grid = cdiv((long long)b.nf * 32, 256);
  switch (prec) {
    case 0: k_ib_force<double><<<grid, 256, 0, s>>>(a, b, fxc, tfc, fxp, tfp); break;
    case 1: k_ib_force<float><<<grid, 256, 0, s>>>(a, b, fxc, tfc, fxp, tfp); break;
    default: k_ib_force<_Float16><<<grid, 256, 0, s>>>(a, b, fxc, tfc, fxp, tfp); break;
  }
  return hipGetLastError();
}

hipError_t launch_mls_post(int prec, const FluidArgs& a, const BodyArgs& b, hipStream_t s) {
  const long long waves = (long long)b.nf + (b.nsoft_v + 1) / 2;
  if (waves == 0) return hipSuccess;
  const unsigned grid = cdiv(waves * 64, 256);
  switch (prec) {
    case 0: k_mls_post<double><<<grid, 256, 0, s>>>(a, b); break;
    case 1: k_mls_post<float><<<grid, 256, 0, s>>>(a, b); break;
    default: k_mls_post<_Float16><<<grid, 256, 0, s>>>(a, b); break;
  }
  return hipGetLastError();
}

hipError_t launch_body_post(const BodyArgs& b, DevFlags* flags, hipStream_t s) {
  const unsigned grid = (unsigned)b.nbody + cdiv(b.nsoft_v, 256);
  if (grid == 0) return hipSuccess;
  k_body_post<<<grid, 256, 0, s>>>(b, flags);
  return hipGetLastError();
}

hipError_t launch_end(const BodyArgs& b, const double* X, DevFlags* flags, int count,
                      hipStream_t s) {
  const unsigned grid = b.nbody > 0 ? (unsigned)b.nbody : 1u;
  // the block counter lives right after the flags word
  k_diag<<<grid, 256, 0, s>>>(b, X, flags, (unsigned int*)(flags + 1), count);
  return hipGetLastError();
}

hipError_t launch_get_fields(int prec, const Grid& g, const void* f0, const void* f1,
                             const uint8_t* ncls, const long long* fx0, const long long* fx1,
                             const uint8_t* tf0, const uint8_t* tf1, double gx, double gy,
                             double gz, const DevFlags* flags, double* rho, double* u,
                             double* pops, double* fib, hipStream_t s) {
  const long long N = (long long)g.nx * g.ny * g.nz;
  switch (prec) {
    case 0:
      k_get_fields<double><<<cdiv(N, 256), 256, 0, s>>>(g, (const double*)f0, (const double*)f1,
                                                        ncls, fx0, fx1, tf0, tf1, gx, gy, gz,
                                                        flags, rho, u, pops, fib);
      break;
    case 1:
      k_get_fields<float><<<cdiv(N, 256), 256, 0, s>>>(g, (const float*)f0, (const float*)f1, ncls,
                                                       fx0, fx1, tf0, tf1, gx, gy, gz, flags,
                                                       rho, u, pops, fib);
      break;
    default:
      k_get_fields<_Float16><<<cdiv(N, 256), 256, 0, s>>>(
          g, (const _Float16*)f0, (const _Float16*)f1, ncls, fx0, fx1, tf0, tf1, gx, gy, gz, flags,
          rho, u, pops, fib);
      break;
  }
  return hipGetLastError();
}

hipError_t launch_interp(int prec, const Grid& g, const void* f0, const void* f1,
                         const uint8_t* ncls, const long long* fx0, const long long* fx1,
                         const uint8_t* tf0, const uint8_t* tf1, double gx, double gy, double gz,
                         const DevFlags* flags, long long n, const double* pts,
                         const double* field, double* out, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const unsigned grid = cdiv(n * 32, 256);
  switch (prec) {
    case 0:
      k_interp<double><<<grid, 256, 0, s>>>(g, (const double*)f0, (const double*)f1, ncls, fx0, fx1,
                                            tf0, tf1, gx, gy, gz, flags, n, pts, field, out);
      break;
    case 1:
      k_interp<float><<<grid, 256, 0, s>>>(g, (const float*)f0, (const float*)f1, ncls, fx0, fx1,
                                           tf0, tf1, gx, gy, gz, flags, n, pts, field, out);
      break;
    default:
      k_interp<_Float16><<<grid, 256, 0, s>>>(g, (const _Float16*)f0, (const _Float16*)f1, ncls, fx0,
                                              fx1, tf0, tf1, gx, gy, gz, flags, n, pts, field, out);
      break;
  }
  return hipGetLastError();
}

hipError_t launch_spread_api(const Grid& g, const uint8_t* ncls, long long n, const double* pts,
                             const double* F, const double* c, long long* fx, DevFlags* flags,
                             hipStream_t s) {
  if (n == 0) return hipSuccess;
  k_spread_api<<<cdiv(n * 32, 256), 256, 0, s>>>(g, ncls, n, pts, F, c, fx, flags);
  return hipGetLastError();
}

hipError_t launch_flush_fx(const Grid& g, long long* fx, double* fib, hipStream_t s) {
  const long long N = (long long)g.nx * g.ny * g.nz;
  k_flush_fx<<<cdiv(N, 256), 256, 0, s>>>(g, fx, fib);
  return hipGetLastError();
}

}  // namespace lbm
