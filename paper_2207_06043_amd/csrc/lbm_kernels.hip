// gfx950 kernels of the coupled lattice-Boltzmann / dynamic immersed-boundary
// step (Coclite, de Tullio, Pascazio, Politi, arXiv 2207.06043, section
// "Numerical method and computational procedure").
//
// One coupled step is four launches on one stream (a step without bodies:
// the fluid launch and k_close):
//   k_ib_force   marker blocks: MLS interpolation of the streamed (pre-force)
//                velocity at the face centroids, direct forcing and spreading
//                (fixed-point atomics, deterministic); element blocks:
//                stretching and bending forces; diagnostics blocks: volume,
//                area, bounding box and damage check of the positions;
//   k_fluid_all  (k_fluid_bulk and k_fluid_rec on two streams for large
//                grids) fused pull-stream + wall links (interpolated
//                bounce-back) + Zou-He + moments + forced BGK collision; bulk
//                nodes as SoA loads/stores of V consecutive nodes (or one node
//                per thread from a list), boundary nodes from compact records;
//   k_mls_post   hydrodynamic probes (pressure and viscous stress from MLS
//                fits at +-1.2 dx), repulsion, MLS velocity at the vertices,
//                clearing of the previous step's spread buffer;
//   k_body_post  vertex forces and Verlet (soft) / Newton-Euler (rigid); its
//                last block closes the step (with many bodies a k_close
//                launch follows instead).
// Populations are stored as deviations g_i = f_i - w_i from the rest
// equilibrium; the collision is written for g (algebraically identical to the
// BGK rule on f, with smaller rounding).
#include <float.h>
#include <limits.h>
#include <math.h>

#include <mutex>

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
};
template <>
struct Store<float> {
  typedef float C;
};
template <>
struct Store<_Float16> {
  typedef float C;
};
// V consecutive populations of one plane: aligned and element-aligned forms.
template <class S, int V>
struct Vec {
  typedef S a __attribute__((ext_vector_type(V)));
  typedef S u __attribute__((ext_vector_type(V), aligned(sizeof(S))));
};
template <int V>
struct ClsWord;
template <>
struct ClsWord<1> { typedef uint8_t T; };
template <>
struct ClsWord<2> { typedef uint16_t T; };
template <>
struct ClsWord<4> { typedef uint32_t T; };
template <>
struct ClsWord<8> { typedef uint64_t T; };

// ------------------------------------------------------------ index helpers
__device__ __forceinline__ int wrap2(int c, int n) {  // |c| excursion <= 2 cells
  c = c < 0 ? c + n : (c >= n ? c - n : c);
  return c < 0 ? c + n : (c >= n ? c - n : c);
}
__device__ __forceinline__ long long nbr(const Grid& G, int x, int y, int z, int dx, int dy,
                                         int dz) {
  x = wrap2(x + dx, G.nx);
  y = wrap2(y + dy, G.ny);
  z = wrap2(z + dz, G.nz);
  return x + (long long)G.px * (y + (long long)G.ny * z);
}

__device__ __forceinline__ unsigned int udiv31(unsigned int u, unsigned int m, int s) {
  return (unsigned int)(((unsigned long long)u * m) >> s);
}
__device__ __forceinline__ void coords(const Grid& G, long long n, int& x, int& y, int& z) {
  const unsigned int u = (unsigned int)n;  // padded index < 2^31
  const unsigned int t = u / (unsigned int)G.px;
  x = (int)(u - t * (unsigned int)G.px);
  z = (int)(t / (unsigned int)G.ny);
  y = (int)(t - (unsigned int)z * (unsigned int)G.ny);
}
// The same with the divisions as multiply-shifts (fewer instructions; the
// fluid kernels, where the instruction count bounds the FP16S sweep).
__device__ __forceinline__ void coords_ms(const Grid& G, long long n, int& x, int& y, int& z) {
  const unsigned int u = (unsigned int)n;
  const unsigned int t = udiv31(u, G.mpx, G.spx);
  x = (int)(u - t * (unsigned int)G.px);
  z = (int)udiv31(t, G.mny, G.sny);
  y = (int)(t - (unsigned int)z * (unsigned int)G.ny);
}

// The wrapped neighbourhood of a node for offsets -2..2 on each axis, as the
// three terms of a padded index (x, px y, px ny z): at() gives the same index
// as nbr(), with the wraps done once per node instead of once per neighbour.
struct Hood {
  int tx[5], ty[5], tz[5];
  __device__ __forceinline__ int at(int dx, int dy, int dz) const {
    return tx[dx + 2] + ty[dy + 2] + tz[dz + 2];
  }
};
__device__ __forceinline__ Hood hood(const Grid& G, int x, int y, int z) {
  Hood h;
#pragma unroll
  for (int d = 0; d < 5; d++) {
    h.tx[d] = wrap2(x + d - 2, G.nx);
    h.ty[d] = G.px * wrap2(y + d - 2, G.ny);
    h.tz[d] = G.px * G.ny * wrap2(z + d - 2, G.nz);
  }
  return h;
}

// Blocks are dispatched round-robin over the 8 XCDs; give every XCD a
// contiguous run of tiles so that neighbouring rows share its L2.
__device__ __forceinline__ int xcd_remap(int b, int n) {
  int full = n & ~7;
  if (b >= full) return b;
  return (b & 7) * (full >> 3) + (b >> 3);
}

__device__ __forceinline__ void fx_add(long long* p, double v, DevFlags* fl) {
  if (!(fabs(v) <= 1.0)) {
    // out of the fixed-point range: dropped and flagged
    atomicOr(&fl->overflow, 1u);
    atomicOr(&fl->pending, ST_UNSTABLE);
    v = 0.0;
  }
  long long q = __double2ll_rn(v * FX_SCALE);
  atomicAdd((unsigned long long*)p, (unsigned long long)q);
}

// ---------------------------------------------------------------- collision
// Sum of the 19 deviations (the density deviation rho - 1).  The deviations
// of a direction and its opposite are close to +-3 w e.u and nearly cancel,
// so they are added pairwise first: those sums are exact or nearly so, and
// the density deviation keeps its relative precision in float as well,
// instead of carrying rounding of the size of the large terms.
template <class C>
__device__ __forceinline__ C dev_sum(const C (&g)[19]) {
  const C ax = ((g[1] + g[2]) + (g[3] + g[4])) + (g[5] + g[6]);
  const C d1 = ((g[7] + g[12]) + (g[8] + g[11])) + ((g[9] + g[14]) + (g[10] + g[13]));
  const C d2 = (g[15] + g[18]) + (g[16] + g[17]);
  return g[0] + ((ax + d1) + d2);
}

// e v for a lattice velocity component e in {-1, 0, 1}.  The zero term is
// -0, which an addition drops exactly, so the unrolled dot products below
// keep only their non-zero terms: the same values as the full products
// (0 v + w = w), without the multiplications by zero that IEEE arithmetic
// would otherwise have to carry out.
template <class C>
__device__ __forceinline__ C eterm(int e, C v) {
  return e == 0 ? C(-0.0) : (e > 0 ? v : -v);
}

// BGK with the forcing term on deviations g = f - w (Eqs. evoleq, eqfunc,
// forcing): rho = 1 + sum g, rho u = sum g e + F/2,
// g^eq_i = w_i (drho + rho (3 e.u + 9/2 (e.u)^2 - 3/2 u.u)),
// F_i = (1 - 1/(2 tau)) w_i (3 (e_i - u) + 9 (e_i.u) e_i).F.
template <class C>
__device__ __forceinline__ void collide(C (&g)[19], C Fx, C Fy, C Fz, C omega, C& drho_out, C& ux,
                                        C& uy, C& uz) {
  const C drho = dev_sum(g);
  drho_out = drho;
  C mx = (g[1] - g[2]) + (g[7] + g[8]) + (g[9] + g[10]) - (g[11] + g[12]) - (g[13] + g[14]);
  C my = (g[3] - g[4]) + (g[7] - g[8]) + (g[11] - g[12]) + (g[15] + g[16]) - (g[17] + g[18]);
  C mz = (g[5] - g[6]) + (g[9] - g[10]) + (g[13] - g[14]) + (g[15] - g[16]) + (g[17] - g[18]);
  const C rho = C(1) + drho;
  C ir = C(1) / rho;
  ux = (mx + C(0.5) * Fx) * ir;
  uy = (my + C(0.5) * Fy) * ir;
  uz = (mz + C(0.5) * Fz) * ir;
  C usq = ux * ux + uy * uy + uz * uz;
  C uF = ux * Fx + uy * Fy + uz * Fz;
  C kf = C(1) - C(0.5) * omega;
#pragma unroll
  for (int i = 0; i < 19; i++) {
    C eu = eterm(EX[i], ux) + eterm(EY[i], uy) + eterm(EZ[i], uz);
    C eF = eterm(EX[i], Fx) + eterm(EY[i], Fy) + eterm(EZ[i], Fz);
    C w = C(WD[i]);
    C geq = w * (drho + rho * (C(3) * eu + C(4.5) * eu * eu - C(1.5) * usq));
    C Gi = kf * w * (C(3) * (eF - uF) + C(9) * eu * eF);
    g[i] = g[i] - omega * (g[i] - geq) + Gi;
  }
  if constexpr (sizeof(C) < sizeof(double)) {
    // The collision keeps the mass (rho - 1) and turns the momentum m into
    // m + F exactly; with the weights rounded to float it does not (their
    // sums are off by ~1e-8, the same sign at every node and step), so the
    // residuals are put back: mass on the rest population, momentum on the
    // axis pairs.
    const C mx1 = (g[1] - g[2]) + (g[7] + g[8]) + (g[9] + g[10]) - (g[11] + g[12]) - (g[13] + g[14]);
    const C my1 = (g[3] - g[4]) + (g[7] - g[8]) + (g[11] - g[12]) + (g[15] + g[16]) - (g[17] + g[18]);
    const C mz1 = (g[5] - g[6]) + (g[9] - g[10]) + (g[13] - g[14]) + (g[15] - g[16]) + (g[17] - g[18]);
    const C rx = C(0.5) * ((mx + Fx) - mx1), ry = C(0.5) * ((my + Fy) - my1), rz = C(0.5) * ((mz + Fz) - mz1);
    g[1] += rx;
    g[2] -= rx;
    g[3] += ry;
    g[4] -= ry;
    g[5] += rz;
    g[6] -= rz;
    g[0] += drho - dev_sum(g);
  }
}

// ----------------------------------------------------- boundary nodes (S1/S2)
template <class S>
__device__ __forceinline__ typename Store<S>::C ldA(const FluidArgs& a, int j, long long node) {
  return to_c(((const S*)a.A)[(long long)j * a.g.plane + node]);
}

// Zou-He on an open face (Eq. extbound, general inward normal n = s e_ax),
// on deviations: rho_w = (1 + G0 + 2 Gout)/(1 - u_n) for a velocity face,
// u_n = (rho_w - 1 - G0 - 2 Gout)/rho_w for a density face (tangential u = 0);
// unknowns (e.n = +1): axis  g = g_opp + rho_w/3 u_n,
// diagonal e = n + t: g = g_opp + rho_w/6 (u_n + u.t) - N_t with
// N_t = 1/2 sum_{e.n = 0} g (e.t) - rho_w/3 u.t.  Written with selects on the
// runtime face so that the code stays small.
template <class C>
__device__ void zouhe(C (&g)[19], int face, int kind, C bx, C by, C bz, C brho) {
  const int ax = face >> 1;
  const int s = (face & 1) ? -1 : 1;
  C G0 = 0, Gout = 0, T[3] = {0, 0, 0};
#pragma unroll
  for (int j = 0; j < 19; j++) {
    const int e_ax = ax == 0 ? EX[j] : (ax == 1 ? EY[j] : EZ[j]);
    const int en = s * e_ax;
    G0 += en == 0 ? g[j] : C(0);
    Gout += en == -1 ? g[j] : C(0);
    if (EX[j]) T[0] += en == 0 ? C(EX[j]) * g[j] : C(0);
    if (EY[j]) T[1] += en == 0 ? C(EY[j]) * g[j] : C(0);
    if (EZ[j]) T[2] += en == 0 ? C(EZ[j]) * g[j] : C(0);
  }
  C u[3] = {bx, by, bz};
  C rho, un;
  if (kind == 0) {
    un = C(s) * (ax == 0 ? u[0] : (ax == 1 ? u[1] : u[2]));
    rho = (C(1) + G0 + C(2) * Gout) / (C(1) - un);
  } else {
    rho = brho;
    un = (rho - C(1) - G0 - C(2) * Gout) / rho;
    u[0] = ax == 0 ? C(s) * un : C(0);
    u[1] = ax == 1 ? C(s) * un : C(0);
    u[2] = ax == 2 ? C(s) * un : C(0);
  }
  C N[3];
#pragma unroll
  for (int k = 0; k < 3; k++) N[k] = C(0.5) * T[k] - rho / C(3) * u[k];
  C out[19];
#pragma unroll
  for (int j = 0; j < 19; j++) {
    const int e_ax = ax == 0 ? EX[j] : (ax == 1 ? EY[j] : EZ[j]);
    // tangential part t = e_j - n (zero on the normal axis)
    const C tx = ax == 0 ? C(0) : C(EX[j]), ty = ax == 1 ? C(0) : C(EY[j]), tz = ax == 2 ? C(0) : C(EZ[j]);
    const C ut = u[0] * tx + u[1] * ty + u[2] * tz;
    const C Nt = N[0] * tx + N[1] * ty + N[2] * tz;
    const bool axis = tx == C(0) && ty == C(0) && tz == C(0);
    const C fill = axis ? g[OPP[j]] + rho / C(3) * un : g[OPP[j]] + rho / C(6) * (un + ut) - Nt;
    out[j] = (s * e_ax == 1) ? fill : g[j];
  }
#pragma unroll
  for (int j = 0; j < 19; j++) g[j] = out[j];
}

// Interpolated bounce-back of the linked direction j at node x (Eq.
// bbouzidi): k0 f*_i(x) + k1 t1 + k2 t2 with i the opposite of j and, by the
// link's branch, t1 = f*_i(x - e_i), t2 = f*_i(x - 2e_i) (q < 1/2) or
// t1 = f*_j(x), t2 = f*_j(x - e_i) (q >= 1/2); k1, k2 are zero where the
// fluid neighbours are missing.  The loads carry no branch (they go out in
// one batch with the rest of the node's loads); for a direction without a
// link they read the node's own values (no traffic) and the caller drops
// the result.
template <class S>
struct Bfl {
  typename Store<S>::C k0, k1, k2, s, t1, t2;
};

template <class S>
__device__ __forceinline__ Bfl<S> bfl_load(const FluidArgs& a, int j, bool linked, int lk, bool hq,
                                           int node, const Hood& h) {
  typedef typename Store<S>::C C;
  const Grid& G = a.g;
  const C* lc = (const C*)a.lk_c;
  const S* A = (const S*)a.A;
  const long long nl = a.nlinks;
  const int i = OPP[j];
  const int l = linked ? lk : 0;
  const int n1 = linked ? h.at(EX[j], EY[j], EZ[j]) : node;  // x - e_i
  const int n2 = linked ? h.at(2 * EX[j], 2 * EY[j], 2 * EZ[j]) : node;
  Bfl<S> r;
  r.k0 = lc[l];
  r.k1 = lc[nl + l];
  r.k2 = lc[2 * nl + l];
  r.s = ldA<S>(a, i, node);
  r.t1 = to_c(A[hq ? (long long)j * G.plane + node : (long long)i * G.plane + n1]);
  r.t2 = to_c(A[hq ? (long long)j * G.plane + n1 : (long long)i * G.plane + n2]);
  return r;
}

// The same loads with each neighbour index formed on its own (fewer values
// live at once: used where registers are scarce, in the IB kernels).
template <class S>
__device__ __forceinline__ Bfl<S> bfl_load_nb(const FluidArgs& a, int j, bool linked, int lk, bool hq,
                                              long long node, int x, int y, int z) {
  typedef typename Store<S>::C C;
  const Grid& G = a.g;
  const C* lc = (const C*)a.lk_c;
  const long long nl = a.nlinks;
  const int i = OPP[j];
  const int l = linked ? lk : 0;
  const long long n1 = linked ? nbr(G, x, y, z, EX[j], EY[j], EZ[j]) : node;  // x - e_i
  const long long n2 = linked ? nbr(G, x, y, z, 2 * EX[j], 2 * EY[j], 2 * EZ[j]) : node;
  Bfl<S> r;
  r.k0 = lc[l];
  r.k1 = lc[nl + l];
  r.k2 = lc[2 * nl + l];
  r.s = ldA<S>(a, i, node);
  r.t1 = ldA<S>(a, hq ? j : i, hq ? node : n1);
  r.t2 = ldA<S>(a, hq ? j : i, hq ? n1 : n2);
  return r;
}

template <class S>
__device__ __forceinline__ typename Store<S>::C bfl_value(const Bfl<S>& b) {
  return b.k0 * b.s + b.k1 * b.t1 + b.k2 * b.t2;
}

// Streamed populations of a boundary record: plain pulls (periodic wrap),
// interpolated bounce-back on wall links, and Zou-He for the populations
// entering through an open face.  Addresses are formed with periodic wrap,
// so they lie in the box; after the record's header every load is issued
// in one batch, then the arithmetic follows.  A pull from a solid node or
// from outside the box reads the node's own rest value (no traffic) and is
// not used.
template <class S>
__device__ void pull_general(const FluidArgs& a, int r, typename Store<S>::C (&g)[19], bool zh = true) {
  typedef typename Store<S>::C C;
  const Grid& G = a.g;
  const S* A = (const S*)a.A;
  const int node = a.rec_node[r];
  const uint32_t mask = a.rec_mask[r];
  const uint32_t hqm = a.rec_mb[r];
  const int lk0 = a.rec_link0[r];
  const int fc = a.rec_face[r];
  int x, y, z;
  coords(G, node, x, y, z);
  const Hood h = hood(G, x, y, z);
  const int face = fc & 7, kind = (fc >> 4) & 1;
  const int ax = face >> 1, s = (face & 1) ? -1 : 1;
  C pl[19];
  Bfl<S> bb[19];
  pl[0] = ldA<S>(a, 0, node);
#pragma unroll
  for (int j = 1; j < 19; j++) {
    const int e[3] = {EX[j], EY[j], EZ[j]};
    const bool linked = (mask >> j) & 1u;
    const bool unknown = fc != 0xff && s * (ax == 0 ? e[0] : (ax == 1 ? e[1] : e[2])) == 1;
    const bool plain = !linked && !unknown;
    pl[j] = to_c(A[plain ? (long long)j * G.plane + h.at(-EX[j], -EY[j], -EZ[j]) : (long long)node]);
    bb[j] = bfl_load<S>(a, j, linked, lk0 + __popc(mask & ((1u << j) - 1u)), (hqm >> j) & 1u, node, h);
  }
  g[0] = pl[0];
#pragma unroll
  for (int j = 1; j < 19; j++) {
    const int e[3] = {EX[j], EY[j], EZ[j]};
    const bool linked = (mask >> j) & 1u;
    const bool unknown = fc != 0xff && s * (ax == 0 ? e[0] : (ax == 1 ? e[1] : e[2])) == 1;
    g[j] = linked ? bfl_value<S>(bb[j]) : (unknown ? C(0) : pl[j]);
  }
  if (fc != 0xff && zh) {
    zouhe<C>(g, face, kind, (C)a.rec_bc[r], (C)a.rec_bc[a.nrec + r], (C)a.rec_bc[2 * a.nrec + r],
             (C)a.rec_bc[3 * a.nrec + r]);
  }
}

struct Moments {
  double drho, m[3];
};

template <class S>
__device__ __forceinline__ Moments streamed_moments(const FluidArgs& a, long long node) {
  Moments out;
  double& drho = out.drho;
  double (&m)[3] = out.m;
  const Grid& G = a.g;
  int x, y, z;
  coords(G, node, x, y, z);
  double g[19];
  if (a.ncls[node] == CLS_BULK) {
#pragma unroll
    for (int j = 0; j < 19; j++) g[j] = (double)ldA<S>(a, j, nbr(G, x, y, z, -EX[j], -EY[j], -EZ[j]));
  } else {
    const int r = a.rec_of[node];
    const uint32_t mask = a.rec_mask[r];
    const uint32_t hqm = a.rec_mb[r];
    const int lk0 = a.rec_link0[r];
    const int fc = a.rec_face[r];
    const int face = fc & 7, ax = face >> 1, sgn = (face & 1) ? -1 : 1;
    typedef typename Store<S>::C C;
    C pl[19];
    Bfl<S> bb[19];
    pl[0] = ldA<S>(a, 0, node);
#pragma unroll
    for (int j = 1; j < 19; j++) {
      const int en = sgn * (ax == 0 ? EX[j] : (ax == 1 ? EY[j] : EZ[j]));
      const bool linked = (mask >> j) & 1u;
      const bool plain = !linked && !(fc != 0xff && en == 1);
      pl[j] = ldA<S>(a, plain ? j : 0, plain ? nbr(G, x, y, z, -EX[j], -EY[j], -EZ[j]) : node);
      bb[j] = bfl_load_nb<S>(a, j, linked, lk0 + __popc(mask & ((1u << j) - 1u)), (hqm >> j) & 1u, node, x, y, z);
    }
    g[0] = (double)pl[0];
#pragma unroll
    for (int j = 1; j < 19; j++) {
      const int en = sgn * (ax == 0 ? EX[j] : (ax == 1 ? EY[j] : EZ[j]));
      const bool linked = (mask >> j) & 1u;
      const bool unknown = fc != 0xff && en == 1;  // the Zou-He rule fills it
      g[j] = linked ? (double)bfl_value<S>(bb[j]) : (unknown ? 0.0 : (double)pl[j]);
    }
    if (fc != 0xff) {
      double G0 = 0.0, Gout = 0.0;
#pragma unroll
      for (int j = 0; j < 19; j++) {
        const int en = sgn * (ax == 0 ? EX[j] : (ax == 1 ? EY[j] : EZ[j]));
        G0 += en == 0 ? g[j] : 0.0;
        Gout += en == -1 ? g[j] : 0.0;
      }
      const int kind = (fc >> 4) & 1;
      double rw, un, ut[3] = {0.0, 0.0, 0.0};
      if (kind == 0) {
        const double bu[3] = {a.rec_bc[r], a.rec_bc[a.nrec + r], a.rec_bc[2 * a.nrec + r]};
        un = sgn * bu[ax];
        rw = (1.0 + G0 + 2.0 * Gout) / (1.0 - un);
#pragma unroll
        for (int k = 0; k < 3; k++) ut[k] = k == ax ? 0.0 : bu[k];
      } else {
        rw = a.rec_bc[3 * a.nrec + r];
        un = (rw - 1.0 - G0 - 2.0 * Gout) / rw;
      }
      drho = rw - 1.0;
#pragma unroll
      for (int k = 0; k < 3; k++) m[k] = rw * (k == ax ? sgn * un : ut[k]);
      return out;
    }
  }
  drho = dev_sum(g);
  m[0] = (g[1] - g[2]) + (g[7] + g[8]) + (g[9] + g[10]) - (g[11] + g[12]) - (g[13] + g[14]);
  m[1] = (g[3] - g[4]) + (g[7] - g[8]) + (g[11] - g[12]) + (g[15] + g[16]) - (g[17] + g[18]);
  m[2] = (g[5] - g[6]) + (g[9] - g[10]) + (g[13] - g[14]) + (g[15] - g[16]) + (g[17] - g[18]);
  return out;
}

// Streamed populations at any non-solid node.
template <class S>
__device__ __forceinline__ void pull_node(const FluidArgs& a, long long node,
                                          typename Store<S>::C (&g)[19]) {
  if (a.ncls[node] == CLS_BULK) {
    const Grid& G = a.g;
    int x, y, z;
    coords(G, node, x, y, z);
    const Hood h = hood(G, x, y, z);
#pragma unroll
    for (int j = 0; j < 19; j++) g[j] = ldA<S>(a, j, h.at(-EX[j], -EY[j], -EZ[j]));
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

// ------------------------------------------------------------ step closing
// Blocks of a kernel that closes a piece of work count themselves on a
// device counter; the last one to arrive combines the kernel's results.
// No agent-scope fence (on gfx950 that writes back the whole L2): the few
// values the last block reads are written with device-coherent atomic
// stores or read-modify-writes, and each writing wave waits for them to
// complete before its block is counted.
__device__ __forceinline__ void wait_mem() { __builtin_amdgcn_s_waitcnt(0); }

__device__ __forceinline__ void store_coherent(double* p, double v) {
  __hip_atomic_store((unsigned long long*)p, (unsigned long long)__double_as_longlong(v),
                     __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double load_coherent(const double* p) {
  return __longlong_as_double((long long)__hip_atomic_load((unsigned long long*)p, __ATOMIC_RELAXED,
                                                           __HIP_MEMORY_SCOPE_AGENT));
}

__device__ __forceinline__ void raise_pending(DevFlags* flags, unsigned int bits) {
  atomicOr(&flags->pending, bits);
  wait_mem();
}

__device__ __forceinline__ bool last_block(unsigned int* counter, unsigned int nblocks) {
  __shared__ int is_last;
  wait_mem();
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned int done = atomicAdd(counter, 1u);
    is_last = (done == nblocks - 1);
  }
  __syncthreads();
  return is_last != 0;
}

// ------------------------------------------------------------- k_fluid
// One thread = V consecutive nodes of a row.  The populations carry guard
// regions of one z-plane plus one row on both sides, so the 19 vector loads
// stay inside the allocation for any group; values pulled for solid or
// boundary-record nodes are computed and discarded.
template <class S, int V, bool PERX>
__device__ void fluid_bulk(const FluidArgs& a, int blk) {
  typedef typename Store<S>::C C;
  typedef typename Vec<S, V>::a vec;
  typedef typename Vec<S, V>::u vecu;
  const Grid& G = a.g;
  long long base;
  if (V == 1 && a.bulk_list) {
    // list form: one bulk node per thread from the sorted list of bulk
    // nodes (no idle lanes on sparse geometries; runs along x stay coalesced)
    const long long i = (long long)blk * blockDim.x + threadIdx.x;
    if (i >= a.nbulk_nodes) return;
    base = a.bulk_list[i];
  } else {
    const long long tile = a.tile_list[blk];
    base = tile * ((long long)blockDim.x * V) + (long long)threadIdx.x * V;
  }
  if (base >= G.Np) return;
  const typename ClsWord<V>::T cw = *(const typename ClsWord<V>::T*)(a.ncls + base);
  bool isb[V];
  bool all = true, any = false;
#pragma unroll
  for (int k = 0; k < V; k++) {
    isb[k] = ((cw >> (8 * k)) & 0xff) == CLS_BULK;
    all = all && isb[k];
    any = any || isb[k];
  }
  if (!any) return;
  const bool flagged = a.tflag && a.tflag[base >> TILE_SHIFT];
  const S* A = (const S*)a.A;
  S* B = (S*)a.B;
  const C omega = (C)a.omega;
  int x0, y, z;
  coords_ms(G, base, x0, y, z);
  // The nine source rows (y - e_y, z - e_z), wrapped once on periodic axes
  // (on closed ones the guard rows take the discarded pulls), as element
  // offsets from the start of a plane: padded indices, guards included,
  // stay inside int range (checked when the lattice is created).
  int rows[3][3];
  {
    const int pxy = G.px * G.ny;
    int ty[3], tz[3];
#pragma unroll
    for (int d = 0; d < 3; d++) {
      ty[d] = G.px * (G.per[1] ? wrap2(y + d - 1, G.ny) : y + d - 1);
      tz[d] = pxy * (G.per[2] ? wrap2(z + d - 1, G.nz) : z + d - 1);
    }
#pragma unroll
    for (int dz = 0; dz < 3; dz++)
#pragma unroll
      for (int dy = 0; dy < 3; dy++) rows[dz][dy] = (ty[dy] + x0) + tz[dz];
  }
  // periodic x: groups touching x = 0 or x = nx-1 gather element by element
  const bool xedge = PERX && (x0 == 0 || x0 + V > G.nx - 1);
  vec in[19];
  if (!PERX || !xedge) {
#pragma unroll
    for (int j = 0; j < 19; j++) {
      const S* pl = A + (long long)j * G.plane;
      const int o = rows[1 - EZ[j]][1 - EY[j]];
      if (EX[j] == 0)
        in[j] = *(const vec*)(pl + o);
      else
        in[j] = *(const vecu*)(pl + (o - EX[j]));
    }
  } else {
#pragma unroll
    for (int j = 0; j < 19; j++) {
      const S* pl = A + (long long)j * G.plane + (rows[1 - EZ[j]][1 - EY[j]] - x0);
#pragma unroll
      for (int k = 0; k < V; k++) in[j][k] = pl[wrap2(x0 + k - EX[j], G.nx)];
    }
  }
  bool bad = false;
#pragma unroll
  for (int k = 0; k < V; k++) {
    C g[19];
#pragma unroll
    for (int j = 0; j < 19; j++) g[j] = to_c(in[j][k]);
    C Fx, Fy, Fz, drho, ux, uy, uz;
    node_force<C>(a, base + k, flagged && isb[k], Fx, Fy, Fz);
    collide<C>(g, Fx, Fy, Fz, omega, drho, ux, uy, uz);
    if (a.mac && isb[k]) store_mac<C>(a, base + k, drho, ux, uy, uz);
    bad = bad || (isb[k] && !(ux * ux + uy * uy + uz * uz <= C(0.09)));
#pragma unroll
    for (int j = 0; j < 19; j++) in[j][k] = (S)g[j];
  }
  const int b32 = (int)base;
  if (all) {
#pragma unroll
    for (int j = 0; j < 19; j++) *(vec*)(B + (long long)j * G.plane + b32) = in[j];
  } else {
#pragma unroll
    for (int j = 0; j < 19; j++)
#pragma unroll
      for (int k = 0; k < V; k++)
        if (isb[k]) B[(long long)j * G.plane + (b32 + k)] = in[j][k];
  }
  if (bad) raise_pending(a.flags, ST_UNSTABLE);
}

// This step's rho - 1 and u at a node (what the probes and the vertex
// velocities interpolate), [Np][4] in the compute type.
template <class C>
__device__ __forceinline__ void store_mac(const FluidArgs& a, long long node, C drho, C ux, C uy, C uz) {
  typedef C C4 __attribute__((ext_vector_type(4)));
  C4 v;
  v.x = drho;
  v.y = ux;
  v.z = uy;
  v.w = uz;
  ((C4*)a.mac)[node] = v;
}

template <class S>
__device__ __forceinline__ void load_mac(const FluidArgs& a, long long node, double& drho, double& ux,
                                         double& uy, double& uz) {
  typedef typename Store<S>::C C;
  typedef C C4 __attribute__((ext_vector_type(4)));
  const C4 v = ((const C4*)a.mac)[node];
  drho = (double)v.x;
  ux = (double)v.y;
  uy = (double)v.z;
  uz = (double)v.w;
}

// Boundary record, one thread: all loads in one batch (pull_general), then
// the forced collision; consecutive records are consecutive nodes, so the
// loads of a wave are coalesced along x.
template <class S>
__device__ void fluid_record_thread(const FluidArgs& a, int r) {
  typedef typename Store<S>::C C;
  C g[19];
  pull_general<S>(a, r, g);
  const long long node = a.rec_node[r];
  const bool flagged = a.tflag && a.tflag[node >> TILE_SHIFT];
  C Fx, Fy, Fz, drho, ux, uy, uz;
  node_force<C>(a, node, flagged, Fx, Fy, Fz);
  collide<C>(g, Fx, Fy, Fz, (C)a.omega, drho, ux, uy, uz);
  if (a.mac) store_mac<C>(a, node, drho, ux, uy, uz);
  S* B = (S*)a.B;
#pragma unroll
  for (int j = 0; j < 19; j++) B[(long long)j * a.g.plane + node] = (S)g[j];
  if (!(ux * ux + uy * uy + uz * uz <= C(0.09))) raise_pending(a.flags, ST_UNSTABLE);
}

// The bulk tiles and the boundary records are two kernels: the records
// need several times the registers of the bulk path, and sharing one kernel
// would cap the occupancy of the bandwidth-bound part.  The two launches
// read A and write disjoint nodes of B and may run concurrently.
template <class S, int V, bool PERX>
__global__ __launch_bounds__(256) void k_fluid_bulk(FluidArgs a) {
  if (a.flags->stop) return;
  fluid_bulk<S, V, PERX>(a, xcd_remap(blockIdx.x, a.nbulk_blocks));
}

template <class S>
__global__ __launch_bounds__(256) void k_fluid_rec(FluidArgs a) {
  if (a.flags->stop) return;
  const int r = xcd_remap(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (r < a.nrec) fluid_record_thread<S>(a, r);
}

// Small (cache-resident, latency-bound) grids: records and bulk tiles in one
// launch, the record blocks first (they take longest), so that a step has
// no fork and join between two streams.  Both parts use blocks of the same
// size.
template <class S, int V, bool PERX>
__device__ __forceinline__ void fluid_unit(const FluidArgs& a, int nrb, int u) {
  if (u < nrb) {
    const int r = u * blockDim.x + threadIdx.x;
    if (r < a.nrec) fluid_record_thread<S>(a, r);
  } else {
    fluid_bulk<S, V, PERX>(a, u - nrb);
  }
}

template <class S, int V, bool PERX>
__global__ __launch_bounds__(256) void k_fluid_all(FluidArgs a, int nrb) {
  if (a.flags->stop) return;
  const int b = blockIdx.x;
  fluid_unit<S, V, PERX>(a, nrb, b < nrb ? xcd_remap(b, nrb) : nrb + xcd_remap(b - nrb, a.nbulk_blocks));
}

// Closes a fluid-only step (one thread).
__global__ void k_close(DevFlags* flags) {
  if (flags->stop) return;
  const unsigned int pend =
      __hip_atomic_load(&flags->pending, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  flags->steps_done += 1;
  flags->stop |= pend;
  flags->pending = 0u;
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
  int cx, cy, cz;  // node coordinates before periodic wrap
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
  s.cx = c[0];
  s.cy = c[1];
  s.cz = c[2];
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
  // moments in double whatever the storage (off the bandwidth-bound path)
  double g[19];
#pragma unroll
  for (int j = 0; j < 19; j++) g[j] = (double)to_c(f[(long long)j * G.plane + node]);
  const double drho = dev_sum(g);
  const double mx = (g[1] - g[2]) + (g[7] + g[8]) + (g[9] + g[10]) - (g[11] + g[12]) - (g[13] + g[14]);
  const double my = (g[3] - g[4]) + (g[7] - g[8]) + (g[11] - g[12]) + (g[15] + g[16]) - (g[17] + g[18]);
  const double mz = (g[5] - g[6]) + (g[9] - g[10]) + (g[13] - g[14]) + (g[15] - g[16]) + (g[17] - g[18]);
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

__device__ __forceinline__ void face_geom_pts(const double (&pa)[3], const double (&pb)[3],
                                              const double (&pd)[3], double (&c)[3], double (&n)[3],
                                              double& area) {
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
  face_geom_pts(pa, pb, pd, c, n, area);
}

__device__ __forceinline__ void cross3(const double* a, const double* b, double* c) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}

// Signed dihedral angle of hinge (a, b, c, d) (faces (a,b,c) and (b,a,d),
// outward normals, positive for a convex fold) and its gradient with
// respect to the four vertices: the wing gradients are -|e| n/|n|^2; the
// edge-end gradients follow from translation and rotation invariance.
__device__ void hinge_all(const double* X, const int32_t* h, double& theta, double (&gr)[4][3]) {
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
    gr[0][k] = -((1.0 - al_c) * gc + (1.0 - al_d) * gd);
    gr[1][k] = -(al_c * gc + al_d * gd);
    gr[2][k] = gc;
    gr[3][k] = gd;
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

// ------------------------------------------------------------ diagnostics
// One block of one body (one face, vertex and edge per thread): partial
// volume sum a.(b x c)/6, area, bounding box, NaN and largest stretch
// l/l0 of the positions X, written to diag_part[dblk].
__device__ void diag_block(const BodyArgs& b, const double* X, int dblk) {
  __shared__ double sh[8];
  __shared__ double shm[4][9];
  const int body = b.dblk_body[dblk];
  const int i = (dblk - b.b_dblk0[body]) * 256 + threadIdx.x;
  // reference centre of the bounding sphere (the previous box centre)
  const double* cref = b.b_diag + 16 * body + 13;
  double V = 0.0, S = 0.0, strain = 0.0, nan = 0.0, r2 = 0.0;
  double lo[3] = {DBL_MAX, DBL_MAX, DBL_MAX}, hi[3] = {-DBL_MAX, -DBL_MAX, -DBL_MAX};
  if (i < b.b_nf[body]) {
    const int f = b.b_face0[body] + i;
    const int* F = b.faces + 3 * f;
    double bc[3];
    cross3(X + 3 * F[1], X + 3 * F[2], bc);
    const double* pa = X + 3 * F[0];
    V = (pa[0] * bc[0] + pa[1] * bc[1] + pa[2] * bc[2]) / 6.0;
    double c[3], n[3];
    face_geom(X, b.faces, f, c, n, S);
  }
  if (i < b.b_nv[body]) {
    const int v = b.b_vert0[body] + i;
    for (int k = 0; k < 3; k++) {
      const double c = X[3 * v + k];
      if (!(c == c)) nan = 1.0;
      lo[k] = c;
      hi[k] = c;
      r2 += (c - cref[k]) * (c - cref[k]);
    }
  }
  if (i < b.b_ne[body]) {
    const int e = b.b_edge0[body] + i;
    const int p = b.edges[2 * e], c = b.edges[2 * e + 1];
    const double r[3] = {X[3 * p] - X[3 * c], X[3 * p + 1] - X[3 * c + 1], X[3 * p + 2] - X[3 * c + 2]};
    strain = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]) / b.l0[e];
  }
  V = block_sum(V, sh);
  S = block_sum(S, sh);
  for (int k = 0; k < 3; k++)
    for (int m = 32; m >= 1; m >>= 1) {
      lo[k] = fmin(lo[k], __shfl_xor(lo[k], m, 64));
      hi[k] = fmax(hi[k], __shfl_xor(hi[k], m, 64));
    }
  for (int m = 32; m >= 1; m >>= 1) {
    strain = fmax(strain, __shfl_xor(strain, m, 64));
    nan = fmax(nan, __shfl_xor(nan, m, 64));
    r2 = fmax(r2, __shfl_xor(r2, m, 64));
  }
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    for (int k = 0; k < 3; k++) {
      shm[w][k] = lo[k];
      shm[w][3 + k] = hi[k];
    }
    shm[w][6] = strain;
    shm[w][7] = nan;
    shm[w][8] = r2;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double* P = b.diag_part + 12 * (long long)dblk;
    store_coherent(P, V);
    store_coherent(P + 1, S);
    for (int k = 0; k < 9; k++) {
      double m = shm[0][k];
      for (int q = 1; q < (int)(blockDim.x >> 6); q++) m = (k < 3) ? fmin(m, shm[q][k]) : fmax(m, shm[q][k]);
      store_coherent(P + 2 + k, m);
    }
  }
}

// Combine the partials of every body in block order (run by the last
// block); returns the DAMAGED / UNSTABLE bits found by this thread.
__device__ unsigned int diag_finalize(const BodyArgs& b) {
  unsigned int raised = 0u;
  // one wave per body; its lanes take the partial blocks (all loads in
  // flight at once), then a fixed-order xor reduction
  const int wv = threadIdx.x >> 6, ln = threadIdx.x & 63, nw = blockDim.x >> 6;
  for (int body = wv; body < b.nbody; body += nw) {
    double V = 0.0, S = 0.0, lo[3], hi[3], strain = 0.0, nan = 0.0, r2 = 0.0;
    for (int k = 0; k < 3; k++) {
      lo[k] = DBL_MAX;
      hi[k] = -DBL_MAX;
    }
    for (int q = b.b_dblk0[body] + ln; q < b.b_dblk0[body + 1]; q += 64) {
      const double* P = b.diag_part + 12 * (long long)q;
      double p[11];
#pragma unroll
      for (int k = 0; k < 11; k++) p[k] = load_coherent(P + k);
      V += p[0];
      S += p[1];
      for (int k = 0; k < 3; k++) {
        lo[k] = fmin(lo[k], p[2 + k]);
        hi[k] = fmax(hi[k], p[5 + k]);
      }
      strain = fmax(strain, p[8]);
      nan = fmax(nan, p[9]);
      r2 = fmax(r2, p[10]);
    }
    V = red64(V);
    S = red64(S);
    for (int m = 32; m >= 1; m >>= 1) {
      for (int k = 0; k < 3; k++) {
        lo[k] = fmin(lo[k], __shfl_xor(lo[k], m, 64));
        hi[k] = fmax(hi[k], __shfl_xor(hi[k], m, 64));
      }
      strain = fmax(strain, __shfl_xor(strain, m, 64));
      nan = fmax(nan, __shfl_xor(nan, m, 64));
      r2 = fmax(r2, __shfl_xor(r2, m, 64));
    }
    if (ln != 0) continue;
    double* d = b.b_diag + 16 * body;
    d[0] = V;
    d[1] = S;
    for (int k = 0; k < 3; k++) {
      d[2 + k] = lo[k];
      d[5 + k] = hi[k];
    }
    d[8] = strain;
    // bounding sphere of the vertices (and so of the face centroids): the
    // reference centre the blocks measured from, and the largest distance;
    // the next reference is this box's centre
    for (int k = 0; k < 3; k++) {
      d[9 + k] = d[13 + k];
      d[13 + k] = 0.5 * (lo[k] + hi[k]);
    }
    d[12] = sqrt(r2);
    // a link whose length doubles its rest length is damaged (computation stops)
    if (!b.b_rigid[body] && strain >= 2.0) raised |= ST_DAMAGED;
    if (nan > 0.0) raised |= ST_UNSTABLE;
  }
  return raised;
}

// ---------------------------------------------------------- k_ib_force
// First launch of a coupled step, three kinds of blocks:
//  markers   direct forcing at the face centroids (Eqs. uLag, the direct
//            forcing equation, bodyforce): U = sum phi u* with u* = sum f e
//            / rho of the streamed populations (no force), F_l = U_b - U,
//            spread of c_l phi_k F_l (c_l = face area) in fixed point;
//  elements  stretching force per edge (Eq. strainFor) and bending force per
//            hinge, F = -k_b sin(theta - theta0) dtheta/dx (soft bodies);
//  diag      volume, area, bounding box and stretch of x^n; the last block
//            combines them and stops the computation before anything of
//            this step is written when x^n is damaged or not finite.
__device__ __forceinline__ long long fx_quant(double v, DevFlags* fl) {
  if (!(fabs(v) <= 1.0)) {
    // out of the fixed-point range: the step ends as unstable
    atomicOr(&fl->overflow, 1u);
    atomicOr(&fl->pending, ST_UNSTABLE);
    v = 0.0;
  }
  return __double2ll_rn(v * FX_SCALE);
}

// ---------------------------------------------- MLS, one point per lane
// Support k (0..26) of a point with stencil base bs = floor(p + 1/2) is the
// node bs + (k%3-1, (k/3)%3-1, k/9-1); it is used when it lies in the box
// (periodic faces wrap) and is not solid.
__device__ __forceinline__ bool support_node(const Grid& G, const uint8_t* ncls, int cx, int cy,
                                             int cz, long long& node) {
  int c[3] = {cx, cy, cz};
  const int dim[3] = {G.nx, G.ny, G.nz};
#pragma unroll
  for (int k = 0; k < 3; k++) {
    if (c[k] < 0 || c[k] >= dim[k]) {
      if (!G.per[k]) return false;
      c[k] = ((c[k] % dim[k]) + dim[k]) % dim[k];
    }
  }
  node = c[0] + (long long)G.px * (c[1] + (long long)G.ny * c[2]);
  return ncls[node] != CLS_SOLID;
}

// W = exp(-(r/0.3)^2), r = |x_k - p| / 2.6 (Eqs. l2norm, intKernel).  On
// the 3x3x3 stencil around floor(p + 1/2) every |x_k - p| <= 1.5 sqrt(3)
// < 2.6, so r <= 1 always holds and W factors into one term per axis:
// W = w(dx) w(dy) w(dz) with w(d) = exp(-d^2 / (2.6^2 0.09)); the nine
// per-axis terms of a point are computed once.
constexpr double MLS_K = 1.0 / (2.6 * 2.6 * 0.09);

__device__ __forceinline__ void axis_weights(double p, int base, double (&w)[3]) {
#pragma unroll
  for (int i = 0; i < 3; i++) {
    const double d = (double)(base + i - 1) - p;
    w[i] = exp(-(d * d) * MLS_K);
  }
}

// A += W p p^T with p = (1, dx, dy, dz); A packed a00 a01 a02 a03 a11 a12
// a13 a22 a23 a33.
__device__ __forceinline__ void mls_add(double (&A)[10], double W, double dx, double dy, double dz) {
  const double wx = W * dx, wy = W * dy, wz = W * dz;
  A[0] += W;
  A[1] += wx;
  A[2] += wy;
  A[3] += wz;
  A[4] += wx * dx;
  A[5] += wx * dy;
  A[6] += wx * dz;
  A[7] += wy * dy;
  A[8] += wy * dz;
  A[9] += wz * dz;
}

// b += W p f
__device__ __forceinline__ void mls_rhs(double (&bf)[4], double W, double dx, double dy, double dz,
                                        double f) {
  const double wf = W * f;
  bf[0] += wf;
  bf[1] += wf * dx;
  bf[2] += wf * dy;
  bf[3] += wf * dz;
}

// Cholesky A = L L^T; singular (a pivot below 1e-10 of the largest
// diagonal) returns false.  r holds 1/L_ii.
struct Chol4 {
  double L[4][4];
  double r[4];
};

__device__ __forceinline__ bool chol4(const double (&A)[10], Chol4& c) {
  const double M[4][4] = {{A[0], A[1], A[2], A[3]},
                          {A[1], A[4], A[5], A[6]},
                          {A[2], A[5], A[7], A[8]},
                          {A[3], A[6], A[8], A[9]}};
  const double dmax = fmax(fmax(A[0], A[4]), fmax(A[7], A[9]));
  bool ok = dmax > 0.0;
#pragma unroll
  for (int j = 0; j < 4; j++) {
    double d = M[j][j];
#pragma unroll
    for (int k = 0; k < j; k++) d -= c.L[j][k] * c.L[j][k];
    if (!(d > 1e-10 * dmax)) ok = false;
    c.L[j][j] = ok ? sqrt(d) : 1.0;
    c.r[j] = 1.0 / c.L[j][j];
#pragma unroll
    for (int i = j + 1; i < 4; i++) {
      double v = M[i][j];
#pragma unroll
      for (int k = 0; k < j; k++) v -= c.L[i][k] * c.L[j][k];
      c.L[i][j] = v * c.r[j];
    }
  }
  return ok;
}

// x = A^{-1} b
__device__ __forceinline__ void chol_solve(const Chol4& c, const double (&b)[4], double (&x)[4]) {
  double y[4];
#pragma unroll
  for (int i = 0; i < 4; i++) {
    double v = b[i];
#pragma unroll
    for (int k = 0; k < i; k++) v -= c.L[i][k] * y[k];
    y[i] = v * c.r[i];
  }
#pragma unroll
  for (int i = 3; i >= 0; i--) {
    double v = y[i];
#pragma unroll
    for (int k = i + 1; k < 4; k++) v -= c.L[k][i] * x[k];
    x[i] = v * c.r[i];
  }
}

// ------------------------------------------------ forcing markers (S4)
// A block takes MARKERS_PER_BLOCK consecutive faces (neighbouring faces of
// the mesh); four lanes (a quad) serve each marker:
//  1. centroid, area and marker velocity U_b of the face;
//  2. the block's bounding box of support nodes; all its threads compute
//     u* = sum f e / rho of the streamed populations (no force) at every
//     node of the box into LDS;
//  3. per marker: A = sum W p p^T and sum W p u* over the 27 supports, split
//     over the quad (lane q takes supports q, q+4, ...) and combined by a
//     fixed xor tree, one Cholesky, U = e0 . A^{-1} sum W p u*,
//     F_l = U_b - U (Eqs. uLag and the direct-forcing equation);
//  4. spreading (Eq. bodyforce): c_l phi_k F_l with c_l = face area and
//     phi_k = W_k p_k . A^{-1} e0, in fixed point, summed per node in LDS,
//     then one device atomic per node and component (integer sums: the
//     result does not depend on the order).
// A box larger than BOX_CELLS takes the direct path: u* per support from
// global memory and one device atomic per contribution.
__device__ __forceinline__ double sel3(int i, const double (&w)[3]) {
  return i == 0 ? w[0] : (i == 1 ? w[1] : w[2]);
}

__device__ __forceinline__ double quad_sum(double v) {
  v += __shfl_xor(v, 1, 4);
  v += __shfl_xor(v, 2, 4);
  return v;
}

template <class S>
__device__ void marker_block(const FluidArgs& a, const BodyArgs& b, int blk, long long* fxc,
                             uint8_t* tfc) {
  __shared__ double s_u[3][BOX_CELLS];
  __shared__ long long s_acc[3][BOX_CELLS];
  __shared__ int s_node[BOX_CELLS];  // padded node index (< 2^31) or -1
  __shared__ int s_box[6];
  const Grid& G = a.g;
  const int t = threadIdx.x, sub = t & 3;
  const int nchunk = b.chunk_n[blk];
  if (nchunk == 0) {
    // an unused chunk: its box stays empty (the repulsion and the owner
    // pass skip it), and nothing else is done
    if (t < 6) b.chunk_box[6 * blk + t] = t < 3 ? INT_MAX : INT_MIN;
    return;
  }
  const int m = b.chunk_s0[blk] + (t >> 2);  // slot
  const bool mk = (t >> 2) < nchunk;
  if (t < 6) s_box[t] = t < 3 ? INT_MAX : INT_MIN;
  __syncthreads();
  double cen[3] = {0.0, 0.0, 0.0}, Ub[3] = {0.0, 0.0, 0.0}, area = 0.0;
  int bs[3] = {0, 0, 0};
  if (mk) {
    // two rounds of loads: the slot's vertex ids and body, then everything
    // that depends on them at once (positions, vertex velocities, rigid
    // state; the unused of the last two are discarded)
    const int4 sf = *(const int4*)(b.slot_f + 4 * (long long)m);
    const int v0 = sf.x, v1 = sf.y, v2 = sf.z;
    const int body = sf.w;
    double pa[3], pb[3], pd[3], va[3], vb[3], vd[3], rs[12];
#pragma unroll
    for (int k = 0; k < 3; k++) {
      pa[k] = b.Xcur[3 * v0 + k];
      pb[k] = b.Xcur[3 * v1 + k];
      pd[k] = b.Xcur[3 * v2 + k];
      va[k] = b.Vel[3 * v0 + k];
      vb[k] = b.Vel[3 * v1 + k];
      vd[k] = b.Vel[3 * v2 + k];
    }
#pragma unroll
    for (int k = 0; k < 12; k++) rs[k] = b.b_rig[32 * body + k];
    const int rigid = b.b_rigid[body];
    double nrm[3];
    face_geom_pts(pa, pb, pd, cen, nrm, area);
    if (rigid) {
      const double r[3] = {cen[0] - rs[0], cen[1] - rs[1], cen[2] - rs[2]};
      const double* w = rs + 9;
      Ub[0] = rs[3] + (w[1] * r[2] - w[2] * r[1]);
      Ub[1] = rs[4] + (w[2] * r[0] - w[0] * r[2]);
      Ub[2] = rs[5] + (w[0] * r[1] - w[1] * r[0]);
    } else {
#pragma unroll
      for (int k = 0; k < 3; k++) Ub[k] = (va[k] + vb[k] + vd[k]) / 3.0;
    }
#pragma unroll
    for (int k = 0; k < 3; k++) bs[k] = (int)floor(cen[k] + 0.5);
    if (sub == 0) {
#pragma unroll
      for (int k = 0; k < 3; k++) b.centroid[3 * m + k] = cen[k];
      atomicMin(&s_box[0], bs[0]);
      atomicMin(&s_box[1], bs[1]);
      atomicMin(&s_box[2], bs[2]);
      atomicMax(&s_box[3], bs[0]);
      atomicMax(&s_box[4], bs[1]);
      atomicMax(&s_box[5], bs[2]);
    }
  }
  __syncthreads();
  // this block's slots form one chunk: its box of stencil bases lets the
  // repulsion skip the chunk when a face is farther than dx from it (an
  // unused chunk keeps the empty box)
  if (t < 6) b.chunk_box[6 * blk + t] = s_box[t];
  const int x0 = s_box[0] - 1, y0 = s_box[1] - 1, z0 = s_box[2] - 1;
  const int ex = s_box[3] - s_box[0] + 3, ey = s_box[4] - s_box[1] + 3, ez = s_box[5] - s_box[2] + 3;
  const bool fits = s_box[3] >= s_box[0] && (long long)ex * ey * ez <= BOX_CELLS;
  const int ncell = fits ? ex * ey * ez : 0;
  for (int c = t; c < ncell; c += blockDim.x) {
    long long node = -1;
    double u3[3] = {0.0, 0.0, 0.0};
    if (support_node(G, a.ncls, x0 + c % ex, y0 + (c / ex) % ey, z0 + c / (ex * ey), node)) {
      const Moments mo = streamed_moments<S>(a, node);
      const double rho = 1.0 + mo.drho;
#pragma unroll
      for (int k = 0; k < 3; k++) u3[k] = mo.m[k] / rho;
    } else {
      node = -1;
    }
#pragma unroll
    for (int k = 0; k < 3; k++) {
      s_u[k][c] = u3[k];
      s_acc[k][c] = 0;
    }
    s_node[c] = (int)node;
  }
  __syncthreads();
  // a quad always holds one marker (or none), so the quad sums below see
  // four lanes that agree on mk
  double wx[3], wy[3], wz[3];
  axis_weights(cen[0], bs[0], wx);
  axis_weights(cen[1], bs[1], wy);
  axis_weights(cen[2], bs[2], wz);
  double A[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0}, bu[3][4] = {{0, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}};
  // The support loops run rolled: each marker block runs this code once per
  // step on its CU, so its length costs instruction fetch (measured: the
  // seven-fold unrolled loops took longer than their arithmetic).
  if (mk && fits) {
#pragma unroll 1
    for (int k = sub; k < 27; k += 4) {
      const int kx = k % 3, ky = (k / 3) % 3, kz = k / 9;
      const int cx = bs[0] + kx - 1, cy = bs[1] + ky - 1, cz = bs[2] + kz - 1;
      const double dx = cx - cen[0], dy = cy - cen[1], dz = cz - cen[2];
      const int c = (cx - x0) + ex * ((cy - y0) + ey * (cz - z0));
      const double W = s_node[c] >= 0 ? sel3(kx, wx) * sel3(ky, wy) * sel3(kz, wz) : 0.0;
      mls_add(A, W, dx, dy, dz);
#pragma unroll
      for (int q = 0; q < 3; q++) mls_rhs(bu[q], W, dx, dy, dz, s_u[q][c]);
    }
  } else if (mk) {
#pragma unroll 1
    for (int k = sub; k < 27; k += 4) {
      const int kx = k % 3, ky = (k / 3) % 3, kz = k / 9;
      const int cx = bs[0] + kx - 1, cy = bs[1] + ky - 1, cz = bs[2] + kz - 1;
      const double dx = cx - cen[0], dy = cy - cen[1], dz = cz - cen[2];
      long long node;
      double u3[3] = {0.0, 0.0, 0.0};
      const bool ok = support_node(G, a.ncls, cx, cy, cz, node);
      if (ok) {
        const Moments mo = streamed_moments<S>(a, node);
#pragma unroll
        for (int q = 0; q < 3; q++) u3[q] = mo.m[q] / (1.0 + mo.drho);
      }
      const double W = ok ? sel3(kx, wx) * sel3(ky, wy) * sel3(kz, wz) : 0.0;
      mls_add(A, W, dx, dy, dz);
#pragma unroll
      for (int q = 0; q < 3; q++) mls_rhs(bu[q], W, dx, dy, dz, u3[q]);
    }
  }
#pragma unroll
  for (int k = 0; k < 10; k++) A[k] = quad_sum(A[k]);
#pragma unroll
  for (int q = 0; q < 3; q++)
#pragma unroll
    for (int k = 0; k < 4; k++) bu[q][k] = quad_sum(bu[q][k]);
  if (mk) {
    Chol4 ch;
    double cc[4] = {0.0, 0.0, 0.0, 0.0};
    if (chol4(A, ch)) {
      const double e0[4] = {1.0, 0.0, 0.0, 0.0};
      chol_solve(ch, e0, cc);
    } else if (sub == 0) {
      atomicAdd(&a.flags->mls_singular, 1);
    }
    double F[3];
#pragma unroll
    for (int q = 0; q < 3; q++)
      F[q] = Ub[q] - (cc[0] * bu[q][0] + cc[1] * bu[q][1] + cc[2] * bu[q][2] + cc[3] * bu[q][3]);
    if (fits) {
#pragma unroll 1
      for (int k = sub; k < 27; k += 4) {
        const int kx = k % 3, ky = (k / 3) % 3, kz = k / 9;
        const int cx = bs[0] + kx - 1, cy = bs[1] + ky - 1, cz = bs[2] + kz - 1;
        const double dx = cx - cen[0], dy = cy - cen[1], dz = cz - cen[2];
        const int c = (cx - x0) + ex * ((cy - y0) + ey * (cz - z0));
        const double phi = sel3(kx, wx) * sel3(ky, wy) * sel3(kz, wz) * (cc[0] + cc[1] * dx + cc[2] * dy + cc[3] * dz);
        if (s_node[c] >= 0 && phi != 0.0) {
          const double cp = area * phi;
#pragma unroll
          for (int q = 0; q < 3; q++)
            atomicAdd((unsigned long long*)&s_acc[q][c], (unsigned long long)fx_quant(cp * F[q], a.flags));
        }
      }
    } else {
#pragma unroll 1
      for (int k = sub; k < 27; k += 4) {
        const int kx = k % 3, ky = (k / 3) % 3, kz = k / 9;
        const int cx = bs[0] + kx - 1, cy = bs[1] + ky - 1, cz = bs[2] + kz - 1;
        const double dx = cx - cen[0], dy = cy - cen[1], dz = cz - cen[2];
        long long node;
        const bool ok = support_node(G, a.ncls, cx, cy, cz, node);
        const double phi = sel3(kx, wx) * sel3(ky, wy) * sel3(kz, wz) * (cc[0] + cc[1] * dx + cc[2] * dy + cc[3] * dz);
        if (ok && phi != 0.0) {
          const double cp = area * phi;
#pragma unroll
          for (int q = 0; q < 3; q++)
            atomicAdd((unsigned long long*)(fxc + q * G.Np + node), (unsigned long long)fx_quant(cp * F[q], a.flags));
          tfc[node >> TILE_SHIFT] = 1;
        }
      }
    }
  }
  __syncthreads();
  if (b.stage) {
    // two-pass spread: the block's sums go to its staging box; the owner
    // pass (k_spread_owner) adds them up across blocks without atomics
    long long* st = b.stage + (long long)blk * BOX_CELLS * 3;
    int* sn = b.stage_node + (long long)blk * BOX_CELLS;
    for (int c = t; c < ncell; c += blockDim.x) {
      sn[c] = s_node[c];
#pragma unroll
      for (int q = 0; q < 3; q++) st[3 * c + q] = s_acc[q][c];
    }
    return;
  }
  for (int c = t; c < ncell; c += blockDim.x) {
    const long long node = s_node[c];
    if (node < 0) continue;
    bool any = false;
#pragma unroll
    for (int q = 0; q < 3; q++) {
      const long long v = s_acc[q][c];
      if (v != 0) {
        atomicAdd((unsigned long long*)(fxc + q * G.Np + node), (unsigned long long)v);
        any = true;
      }
    }
    if (any) tfc[node >> TILE_SHIFT] = 1;
  }
}

// Cell of node (x, y, z) in a chunk's box (origin o, extents e), trying the
// periodic images one period away; -1 if outside.
__device__ __forceinline__ int box_cell(const Grid& G, const int (&o)[3], const int (&e)[3], int x, int y, int z) {
  const int p[3] = {x, y, z}, n[3] = {G.nx, G.ny, G.nz};
  int c[3];
#pragma unroll
  for (int a = 0; a < 3; a++) {
    int d = p[a] - o[a];
    if (G.per[a] && (d < 0 || d >= e[a])) d = d < 0 ? d + n[a] : d - n[a];
    if (d < 0 || d >= e[a]) return -1;
    c[a] = d;
  }
  return c[0] + e[0] * (c[1] + e[1] * c[2]);
}

// The box of chunk k from its bases (cb: its six ints); false when the chunk
// did not fit LDS (its block added its sums with atomics) or is empty.
__device__ __forceinline__ bool chunk_geom(const int* cb, int (&o)[3], int (&e)[3]) {
  if (cb[3] < cb[0]) return false;
#pragma unroll
  for (int a = 0; a < 3; a++) {
    o[a] = cb[a] - 1;
    e[a] = cb[3 + a] - cb[a] + 3;
  }
  return (long long)e[0] * e[1] * e[2] <= BOX_CELLS;
}

// Owner pass of the two-pass spread: thread (chunk c, cell i) holds node n;
// it is the owner when no lower chunk's box holds n, and then adds the
// staged sums of every chunk that holds n, in chunk order, into the force
// field (plain stores: one owner per node), and flags the tile.
__global__ __launch_bounds__(256) void k_spread_owner(Grid G, BodyArgs b, long long* fxc, uint8_t* tfc,
                                                      const DevFlags* flags) {
  if (flags->stop) return;
  const int nch = b.n_marker_blocks, c = blockIdx.y;
  int o[3], e[3];
  if (!chunk_geom(b.chunk_box + 6 * c, o, e)) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= e[0] * e[1] * e[2]) return;
  const int node = b.stage_node[(long long)c * BOX_CELLS + i];
  if (node < 0) return;
  int x, y, z;
  coords(G, node, x, y, z);
  for (int k = 0; k < c; k++) {
    int ok[3], ek[3];
    if (!chunk_geom(b.chunk_box + 6 * k, ok, ek)) continue;
    const int j = box_cell(G, ok, ek, x, y, z);
    if (j >= 0 && b.stage_node[(long long)k * BOX_CELLS + j] == node) return;  // not the owner
  }
  long long acc[3] = {0, 0, 0};
  for (int k = c; k < nch; k++) {
    int ok[3], ek[3];
    if (!chunk_geom(b.chunk_box + 6 * k, ok, ek)) continue;
    const int j = box_cell(G, ok, ek, x, y, z);
    if (j < 0 || b.stage_node[(long long)k * BOX_CELLS + j] != node) continue;
    const long long* st = b.stage + ((long long)k * BOX_CELLS + j) * 3;
#pragma unroll
    for (int q = 0; q < 3; q++) acc[q] += st[q];
  }
  if (acc[0] == 0 && acc[1] == 0 && acc[2] == 0) return;
#pragma unroll
  for (int q = 0; q < 3; q++) fxc[q * G.Np + node] += acc[q];
  tfc[node >> TILE_SHIFT] = 1;
}

// ------------------------------------------------------------ face binning
// The marker order.  One block per body: each face's key is the position of
// its stencil base floor(c + 1/2) (relative to the body's smallest base, 10
// bits per axis) along the 3-D Hilbert curve, above the face's index within
// the body; the keys are bitonic-sorted (in LDS up to BIN_LDS_KEYS faces,
// else in the body's part of bin_keys) and slot f0 + r takes the face of
// rank r.  The keys are distinct, so the order is a function of the
// positions alone.  The Hilbert curve (unlike the Morton order) has no
// jumps, so 64 consecutive faces stay one compact patch of the membrane.
__device__ __forceinline__ unsigned int spread_bits10(unsigned int x) {
  x &= 1023u;
  x = (x | (x << 16)) & 0x030000FFu;
  x = (x | (x << 8)) & 0x0300F00Fu;
  x = (x | (x << 4)) & 0x030C30C3u;
  x = (x | (x << 2)) & 0x09249249u;
  return x;
}

// Hilbert index of a point of [0, 1024)^3, by Skilling's transpose method
// (J. Skilling, "Programming the Hilbert curve", AIP Conf. Proc. 707, 2004):
// the coordinates are turned, level by level from the top, into the
// transposed index, whose bits interleaved give the distance along the
// curve.
__device__ __forceinline__ unsigned int hilbert10(int a, int b, int c) {
  unsigned int X[3] = {(unsigned int)min(max(a, 0), 1023), (unsigned int)min(max(b, 0), 1023),
                       (unsigned int)min(max(c, 0), 1023)};
  for (unsigned int Q = 512u; Q > 1u; Q >>= 1) {
    const unsigned int P = Q - 1u;
#pragma unroll
    for (int i = 0; i < 3; i++) {
      if (X[i] & Q) {
        X[0] ^= P;  // invert the low bits of the first axis
      } else {      // exchange the low bits of axes 0 and i
        const unsigned int t = (X[0] ^ X[i]) & P;
        X[0] ^= t;
        X[i] ^= t;
      }
    }
  }
  X[1] ^= X[0];  // Gray encode
  X[2] ^= X[1];
  unsigned int t = 0u;
  for (unsigned int Q = 512u; Q > 1u; Q >>= 1)
    if (X[2] & Q) t ^= Q - 1u;
  X[0] ^= t;
  X[1] ^= t;
  X[2] ^= t;
  return (spread_bits10(X[0]) << 2) | (spread_bits10(X[1]) << 1) | spread_bits10(X[2]);
}

__device__ __forceinline__ void face_base(const double* X, const int32_t* faces, int f, int (&bs)[3]) {
  const int v0 = faces[3 * f], v1 = faces[3 * f + 1], v2 = faces[3 * f + 2];
#pragma unroll
  for (int k = 0; k < 3; k++) bs[k] = (int)floor((X[3 * v0 + k] + X[3 * v1 + k] + X[3 * v2 + k]) / 3.0 + 0.5);
}

// Keys and sort of one body; K is LDS or global memory (inlined separately
// for each, so that LDS accesses stay LDS instructions).  On return K[0..nf)
// holds the body's keys in increasing order.
__device__ __forceinline__ void hilbert_sort(const BodyArgs& b, int f0, int nf, int n2, const int (&lo)[3],
                                             unsigned long long* K) {
  const int t = threadIdx.x;
  for (int i = t; i < n2; i += blockDim.x) {
    unsigned long long key = ~0ull;  // padding sorts last
    if (i < nf) {
      int bs[3];
      face_base(b.Xcur, b.faces, f0 + i, bs);
      key = ((unsigned long long)hilbert10(bs[0] - lo[0], bs[1] - lo[1], bs[2] - lo[2]) << 32) | (unsigned int)i;
    }
    K[i] = key;
  }
  __syncthreads();
  for (int k = 2; k <= n2; k <<= 1)
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = t; i < n2; i += blockDim.x) {
        const int p = i ^ j;
        if (p > i) {
          const unsigned long long x = K[i], y = K[p];
          if ((x > y) == ((i & k) == 0)) {
            K[i] = y;
            K[p] = x;
          }
        }
      }
      __syncthreads();
    }
}

__device__ __forceinline__ unsigned int compact_bits10(unsigned int x) {
  x &= 0x09249249u;
  x = (x | (x >> 2)) & 0x030C30C3u;
  x = (x | (x >> 4)) & 0x0300F00Fu;
  x = (x | (x >> 8)) & 0x030000FFu;
  x = (x | (x >> 16)) & 0x000003FFu;
  return x;
}

// The point of [0, 1024)^3 at Hilbert index h (the inverse of hilbert10:
// Gray decode, then the exchanges and inversions undone from the bottom
// level up).
__device__ __forceinline__ void hilbert10_point(unsigned int h, int (&c)[3]) {
  unsigned int X[3] = {compact_bits10(h >> 2), compact_bits10(h >> 1), compact_bits10(h)};
  const unsigned int t = X[2] >> 1;
  X[2] ^= X[1];
  X[1] ^= X[0];
  X[0] ^= t;
  for (unsigned int Q = 2u; Q != 1024u; Q <<= 1) {
    const unsigned int P = Q - 1u;
#pragma unroll
    for (int i = 2; i >= 0; i--) {
      if (X[i] & Q) {
        X[0] ^= P;
      } else {
        const unsigned int u = (X[0] ^ X[i]) & P;
        X[0] ^= u;
        X[i] ^= u;
      }
    }
  }
  c[0] = (int)X[0];
  c[1] = (int)X[1];
  c[2] = (int)X[2];
}

// Exclusive prefix sum over the block's threads in thread order; total gets
// the sum.  s_tmp holds BIN_THREADS / 64 + 1 values.
template <class T>
__device__ __forceinline__ T block_scan(T v, T* s_tmp, T& total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  T x = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const T y = __shfl_up(x, d, 64);
    if (lane >= d) x += y;
  }
  if (lane == 63) s_tmp[w] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    T acc = 0;
    for (int k = 0; k < nw; k++) {
      const T c = s_tmp[k];
      s_tmp[k] = acc;
      acc += c;
    }
    s_tmp[nw] = acc;
  }
  __syncthreads();
  const T ex = s_tmp[w] + x - v;
  total = s_tmp[nw];
  __syncthreads();
  return ex;
}

// Chunks of at most 64 consecutive slots, in order: nrun runs of 64 (the
// last one shorter), the rest of the body's chunks unused.
// Slot s takes face f: the permutation and the face's vertex ids and body.
__device__ __forceinline__ void set_slot(const BodyArgs& b, int s, int f) {
  b.perm[s] = f;
  const int4 v = make_int4(b.faces[3 * f], b.faces[3 * f + 1], b.faces[3 * f + 2], b.face_body[f]);
  *(int4*)(b.slot_f + 4 * (long long)s) = v;
}

__device__ __forceinline__ void fixed_chunks(const BodyArgs& b, int f0, int nf, int c0, int cap) {
  const int nrun = (nf + MARKERS_PER_BLOCK - 1) / MARKERS_PER_BLOCK;
  for (int c = threadIdx.x; c < cap; c += blockDim.x) {
    b.chunk_s0[c0 + c] = f0 + min(c, nrun) * MARKERS_PER_BLOCK;
    b.chunk_n[c0 + c] = c < nrun ? min(MARKERS_PER_BLOCK, nf - c * MARKERS_PER_BLOCK) : 0;
  }
}

__global__ __launch_bounds__(BIN_THREADS) void k_bin_faces(BodyArgs b) {
  __shared__ unsigned long long s_keys[BIN_LDS_KEYS];
  __shared__ unsigned long long s_tmp[BIN_THREADS / 64 + 1];
  __shared__ int s_min[3];
  const int body = blockIdx.x, t = threadIdx.x;
  const int f0 = b.b_face0[body], nf = b.b_nf[body];
  const int c0 = b.b_chunk0[body], cap = b.b_chunk0[body + 1] - c0;
  int n2 = 1;
  while (n2 < nf) n2 <<= 1;
  if (t < 3) s_min[t] = INT_MAX;
  __syncthreads();
  int lo[3] = {INT_MAX, INT_MAX, INT_MAX};
  for (int i = t; i < nf; i += blockDim.x) {
    int bs[3];
    face_base(b.Xcur, b.faces, f0 + i, bs);
#pragma unroll
    for (int k = 0; k < 3; k++) lo[k] = min(lo[k], bs[k]);
  }
#pragma unroll
  for (int k = 0; k < 3; k++) atomicMin(&s_min[k], lo[k]);
  __syncthreads();
  const int mn[3] = {s_min[0], s_min[1], s_min[2]};
  if (n2 > BIN_LDS_KEYS) {
    // large body: sorted in global memory, cut in runs of 64
    unsigned long long* K = b.bin_keys + b.b_key0[body];
    hilbert_sort(b, f0, nf, n2, mn, K);
    for (int i = t; i < nf; i += blockDim.x) set_slot(b, f0 + i, f0 + (int)(K[i] & 0xffffffffull));
    fixed_chunks(b, f0, nf, c0, cap);
    return;
  }
  hilbert_sort(b, f0, nf, n2, mn, s_keys);
  // Chunks: thread t owns the sorted positions t R .. t R + R - 1.  A
  // position starts a segment where its base is more than J (Chebyshev)
  // from the previous one's; each segment of length L is cut into
  // ceil(L / 64) near-equal chunks.  J is the smallest of 1..4 whose
  // segments fit the body's chunks (else plain runs of 64).
  const int R = (nf + BIN_THREADS - 1) / BIN_THREADS;  // <= 8
  unsigned int jm[4] = {0u, 0u, 0u, 0u};
  {
    int prev[3] = {0, 0, 0};
    const int i0 = t * R;
    if (i0 >= 1 && i0 - 1 < nf) hilbert10_point((unsigned int)(s_keys[i0 - 1] >> 32), prev);
    for (int r = 0; r < R; r++) {
      const int i = i0 + r;
      if (i >= nf) break;
      const unsigned long long key = s_keys[i];
      set_slot(b, f0 + i, f0 + (int)(key & 0xffffffffull));
      int c[3];
      hilbert10_point((unsigned int)(key >> 32), c);
      const int d = max(abs(c[0] - prev[0]), max(abs(c[1] - prev[1]), abs(c[2] - prev[2])));
#pragma unroll
      for (int J = 0; J < 4; J++)
        if (i == 0 || d > J + 1) jm[J] |= 1u << r;
      prev[0] = c[0];
      prev[1] = c[1];
      prev[2] = c[2];
    }
  }
  unsigned long long packed = 0ull;
#pragma unroll
  for (int J = 0; J < 4; J++) packed |= (unsigned long long)__popc(jm[J]) << (16 * J);
  unsigned long long tot;
  const unsigned long long ex = block_scan(packed, s_tmp, tot);  // syncs: the keys are free after
  const int nrun = (nf + MARKERS_PER_BLOCK - 1) / MARKERS_PER_BLOCK;
  int J = -1;
  for (int q = 3; q >= 0; q--)
    if ((int)((tot >> (16 * q)) & 0xffffull) + nrun <= cap) J = q;
  if (J < 0) {
    fixed_chunks(b, f0, nf, c0, cap);
    return;
  }
  const int S = (int)((tot >> (16 * J)) & 0xffffull);
  int* SS = reinterpret_cast<int*>(s_keys);  // segment starts [S + 1]
  {
    int o = (int)((ex >> (16 * J)) & 0xffffull);
    for (int r = 0; r < R; r++)
      if (jm[J] & (1u << r)) SS[o++] = t * R + r;
    if (t == 0) SS[S] = nf;
  }
  __syncthreads();
  // chunks of thread t's segments t Rs .. t Rs + Rs - 1
  const int Rs = (S + BIN_THREADS - 1) / BIN_THREADS;
  int nk = 0;
  for (int s = t * Rs; s < min(S, t * Rs + Rs); s++) nk += (SS[s + 1] - SS[s] + MARKERS_PER_BLOCK - 1) / MARKERS_PER_BLOCK;
  unsigned long long ntot;
  int cc = c0 + (int)block_scan((unsigned long long)nk, s_tmp, ntot);
  for (int s = t * Rs; s < min(S, t * Rs + Rs); s++) {
    const int a = SS[s], L = SS[s + 1] - a;
    const int k = (L + MARKERS_PER_BLOCK - 1) / MARKERS_PER_BLOCK;
    for (int q = 0; q < k; q++, cc++) {
      const int lo_q = (L * q) / k, hi_q = (L * (q + 1)) / k;
      b.chunk_s0[cc] = f0 + a + lo_q;
      b.chunk_n[cc] = hi_q - lo_q;
    }
  }
  for (int c = (int)ntot + t; c < cap; c += blockDim.x) {
    b.chunk_s0[c0 + c] = f0 + nf;
    b.chunk_n[c0 + c] = 0;
  }
}

// Zeroes the spread force of the previous step in the tiles it flagged, and
// the flags.  That buffer is not read again once this step has started, and
// the next step adds into it.  Block cb of ncb reads the flags of its tiles
// cb, cb + ncb, ... all at once (one per thread), lists the set ones in LDS,
// then clears them one after the other with all its threads.
__device__ void clear_tiles(const Grid& G, long long* fxp, uint8_t* tfp, int cb, int ncb) {
  __shared__ int s_n;
  __shared__ int s_list[256];
  const long long ntiles = (G.Np >> TILE_SHIFT) + 1;
  for (long long first = cb; first < ntiles; first += (long long)ncb * blockDim.x) {
    if (threadIdx.x == 0) s_n = 0;
    __syncthreads();
    const long long tl = first + (long long)threadIdx.x * ncb;
    if (tl < ntiles && tfp[tl]) s_list[atomicAdd(&s_n, 1)] = (int)tl;
    __syncthreads();
    const int n = s_n;
    // the listed tiles' nodes, all threads at once
    for (int k = threadIdx.x; k < (n << TILE_SHIFT); k += blockDim.x) {
      const long long q = ((long long)s_list[k >> TILE_SHIFT] << TILE_SHIFT) + (k & ((1 << TILE_SHIFT) - 1));
      if (q < G.Np) {
        fxp[q] = 0;
        fxp[G.Np + q] = 0;
        fxp[2 * G.Np + q] = 0;
      }
    }
    if ((int)threadIdx.x < n) tfp[s_list[threadIdx.x]] = 0;
    __syncthreads();
  }
}

__device__ void membrane_element(const BodyArgs& b, int idx) {
  if (idx < b.ne) {
    const int e = idx;
    const int va = b.edges[2 * e], vb = b.edges[2 * e + 1];
    if (b.b_rigid[b.vert_body[va]]) return;
    // F_a = -k (l - l0) (x_a - x_b) / l
    const double r[3] = {b.Xcur[3 * va] - b.Xcur[3 * vb], b.Xcur[3 * va + 1] - b.Xcur[3 * vb + 1],
                         b.Xcur[3 * va + 2] - b.Xcur[3 * vb + 2]};
    const double l = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
    const double c = -b.kl[e] * (l - b.l0[e]) / l;
    const int sa = b.sl_edge[2 * e], sb = b.sl_edge[2 * e + 1];
#pragma unroll
    for (int k = 0; k < 3; k++) {
      b.f_slot[((long long)sa * 3 + k) * b.nv + va] = c * r[k];
      b.f_slot[((long long)sb * 3 + k) * b.nv + vb] = -(c * r[k]);
    }
  } else if (idx < b.ne + b.nh) {
    const int h = idx - b.ne;
    const int32_t* H = b.hinges + 4 * h;
    if (b.b_rigid[b.vert_body[H[0]]]) return;
    double th, gr[4][3];
    hinge_all(b.Xcur, H, th, gr);
    const double amp = -b.kb[h] * sin(th - b.theta0[h]);
#pragma unroll
    for (int r = 0; r < 4; r++) {
      const long long sl = b.sl_hinge[4 * h + r];
#pragma unroll
      for (int k = 0; k < 3; k++) b.f_slot[(sl * 3 + k) * b.nv + H[r]] = amp * gr[r][k];
    }
  }
}

template <class S>
__device__ __forceinline__ void ib_force_block(const FluidArgs& a, const BodyArgs& b, long long* fxc,
                                               uint8_t* tfc, long long* fxp, uint8_t* tfp,
                                               unsigned int* counter, int blk) {
  const int nmk = b.n_marker_blocks, nel = b.n_elem_blocks;
  (void)fxp;
  (void)tfp;
  if (blk < nmk) {
    marker_block<S>(a, b, blk, fxc, tfc);
  } else if (blk < nmk + nel) {
    membrane_element(b, (blk - nmk) * 256 + threadIdx.x);
  } else {
    diag_block(b, b.Xcur, blk - nmk - nel);
    // the diagnostics blocks count themselves; the last one combines them
    if (last_block(counter, b.n_diag_blocks)) {
      const unsigned int raised = diag_finalize(b);
      if (raised) atomicOr(&a.flags->stop, raised);
      __syncthreads();
      if (threadIdx.x == 0) *counter = 0u;
    }
  }
}

// Two blocks per CU (two waves per SIMD) in FP32 and FP16S: the marker
// blocks are latency-bound chains, and a second resident block hides them.
// (FP64 would spill to scratch at that register budget.)
template <class S>
__global__ __launch_bounds__(256, sizeof(S) == 8 ? 1 : 2) void k_ib_force(FluidArgs a, BodyArgs b, long long* fxc,
                                                  uint8_t* tfc, long long* fxp, uint8_t* tfp,
                                                  unsigned int* counter) {
  if (a.flags->stop) return;
  ib_force_block<S>(a, b, fxc, tfc, fxp, tfp, counter, blockIdx.x);
}

// Diagnostics of the current positions only (set-up and synchronisation
// points): fills the body table and stops on damage or non-finite values.
__global__ __launch_bounds__(256) void k_check(BodyArgs b, const double* X0, const double* X1,
                                               DevFlags* flags, unsigned int* counter) {
  if (flags->stop) return;
  const double* X = (flags->steps_done & 1) ? X1 : X0;
  if ((int)blockIdx.x < b.n_diag_blocks) diag_block(b, X, blockIdx.x);
  if (last_block(counter, gridDim.x)) {
    const unsigned int raised = diag_finalize(b);
    if (raised) atomicOr(&flags->stop, raised);
    __syncthreads();
    if (threadIdx.x == 0) *counter = 0u;
  }
}

// ---------------------------------------------------------- k_mls_post
// One MLS point per lane, supports read from this step's rho - 1 and u.
// Face waves (32 faces each): lanes 0-31 take the probe 1.2 dx outside
// their face, lanes 32-63 the probe inside the same face; each fits rho
// (value) and u (gradient) by moving least squares (the linear-fit
// coefficients), then the outer lane forms the traction: pressure p = rho/3
// and viscous stress rho nu (grad u + grad u^T) (Eqs. hydroForP,
// hydroForNu), the repulsion of centroids of other bodies closer than dx
// (Eq. collision) and, for soft bodies, the volume penalty
// k_v (1 - V/V0) A n (Eq. volFor, outward n).  A singular fit gives 0.
// Vertex waves (64 soft vertices each): the MLS velocity u_v,0 at x_v^n.
template <class S>
__device__ __forceinline__ void fit_point(const FluidArgs& a, int sub, double px, double py, double pz,
                                          bool want_grad, double& rfit, double (&val)[3],
                                          double (&grad)[3][3]) {
  typedef typename Store<S>::C C;
  typedef C C4 __attribute__((ext_vector_type(4)));
  const Grid& G = a.g;
  const int bx = (int)floor(px + 0.5), by = (int)floor(py + 0.5), bz = (int)floor(pz + 0.5);
  // this lane's supports k = sub, sub + 4, ... : loads first, all together
  // (out-of-box supports read node 0 and are not used; solid nodes hold
  // zeros and get W = 0)
  bool use[7];
  C4 mv[7];
  uint8_t cls[7];
#pragma unroll
  for (int i = 0; i < 7; i++) {
    const int k = sub + 4 * i;
    long long node = 0;
    int c[3] = {bx + k % 3 - 1, by + (k / 3) % 3 - 1, bz + k / 9 - 1};
    const int dim[3] = {G.nx, G.ny, G.nz};
    bool in = k < 27;
#pragma unroll
    for (int q = 0; q < 3; q++)
      if (c[q] < 0 || c[q] >= dim[q]) {
        if (G.per[q]) c[q] = ((c[q] % dim[q]) + dim[q]) % dim[q];
        else in = false;
      }
    if (in) node = c[0] + (long long)G.px * (c[1] + (long long)G.ny * c[2]);
    use[i] = in;
    cls[i] = a.ncls[node];
    mv[i] = ((const C4*)a.mac)[node];
  }
  double wx[3], wy[3], wz[3];
  axis_weights(px, bx, wx);
  axis_weights(py, by, wy);
  axis_weights(pz, bz, wz);
  double A[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0}, br[4] = {0, 0, 0, 0};
  double bu[3][4] = {{0, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}};
#pragma unroll
  for (int i = 0; i < 7; i++) {
    const int k = sub + 4 * i;
    const int kx = k % 3, ky = (k / 3) % 3, kz = k / 9;
    const double dx = (bx + kx - 1) - px, dy = (by + ky - 1) - py, dz = (bz + kz - 1) - pz;
    const bool u = use[i] && cls[i] != CLS_SOLID;
    const double W = u ? sel3(kx, wx) * sel3(ky, wy) * sel3(kz, wz) : 0.0;
    const double dr = u ? (double)mv[i].x : 0.0;
    const double u3[3] = {u ? (double)mv[i].y : 0.0, u ? (double)mv[i].z : 0.0, u ? (double)mv[i].w : 0.0};
    mls_add(A, W, dx, dy, dz);
    mls_rhs(br, W, dx, dy, dz, dr);
#pragma unroll
    for (int q = 0; q < 3; q++) mls_rhs(bu[q], W, dx, dy, dz, u3[q]);
  }
  // the quad's four partial sums, in a fixed order
#pragma unroll
  for (int k = 0; k < 10; k++) A[k] = quad_sum(A[k]);
#pragma unroll
  for (int k = 0; k < 4; k++) br[k] = quad_sum(br[k]);
#pragma unroll
  for (int q = 0; q < 3; q++)
#pragma unroll
    for (int k = 0; k < 4; k++) bu[q][k] = quad_sum(bu[q][k]);
  Chol4 ch;
  const bool ok = chol4(A, ch);
  if (!ok && sub == 0) atomicAdd(&a.flags->mls_singular, 1);
  double cc[4] = {0.0, 0.0, 0.0, 0.0};
  if (ok) {
    const double e0[4] = {1.0, 0.0, 0.0, 0.0};
    chol_solve(ch, e0, cc);
  }
  // the weights add up to 1, so the fit of rho is 1 + the fit of rho - 1
  rfit = ok ? 1.0 + (cc[0] * br[0] + cc[1] * br[1] + cc[2] * br[2] + cc[3] * br[3]) : 0.0;
#pragma unroll
  for (int q = 0; q < 3; q++) {
    val[q] = cc[0] * bu[q][0] + cc[1] * bu[q][1] + cc[2] * bu[q][2] + cc[3] * bu[q][3];
    double x[4] = {0.0, 0.0, 0.0, 0.0};
    if (ok && want_grad) chol_solve(ch, bu[q], x);
#pragma unroll
    for (int c = 0; c < 3; c++) grad[q][c] = x[1 + c];
  }
}

// Face waves take 8 faces: the quad of lanes 4f..4f+3 (f < 8) fits the probe
// outside face f, lanes 32 + 4f.. the probe inside; vertex waves take 16
// soft vertices, one quad each.

template <class S>
__device__ __forceinline__ void mls_post_block(const FluidArgs& a, const BodyArgs& b, int blk) {
  const int gw = (blk * 256 + threadIdx.x) >> 6;
  const int l = threadIdx.x & 63, sub = l & 3;
  const int nfw = (b.nf + MLS_FACES_PER_WAVE - 1) / MLS_FACES_PER_WAVE;
  if (gw < nfw) {
    const int f = gw * MLS_FACES_PER_WAVE + ((l & 31) >> 2);
    const bool valid = f < b.nf;
    const int fv = valid ? f : b.nf - 1;  // spare lanes repeat a face and write nothing
    double cen[3], nrm[3], area;
    face_geom(b.Xcur, b.faces, fv, cen, nrm, area);
    const double sg = l < 32 ? 1.2 : -1.2;
    double rfit, val[3], G[3][3];
    fit_point<S>(a, sub, cen[0] + sg * nrm[0], cen[1] + sg * nrm[1], cen[2] + sg * nrm[2], true, rfit,
                 val, G);
    // the inner probe of this lane's face
    const double r_in = __shfl(rfit, l + 32, 64);
    double Gin[3][3];
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
      for (int c = 0; c < 3; c++) Gin[i][c] = __shfl(G[i][c], l + 32, 64);
    const int body = b.face_body[fv];
    double acc = 0.0;
    if (b.nbody > 1) {
      // repulsion.  First the lanes test the (face q of the wave, other body
      // o) pairs in parallel: o's box must come within dx of q's body's box
      // and of the face itself, and its bounding sphere within dx of the
      // face.  Then, for each surviving pair in (q, o) order, all lanes scan
      // o's centroids.
      const int npair = MLS_FACES_PER_WAVE * b.nbody;
      int cur_q = -1;
      double part = 0.0;
      for (int base = 0; base < npair; base += 64) {
        const int pi = base + l < npair ? base + l : npair - 1;
        const int pq = pi / b.nbody, po = pi - pq * b.nbody;
        const double px = __shfl(cen[0], 4 * pq, 64), py = __shfl(cen[1], 4 * pq, 64),
                     pz = __shfl(cen[2], 4 * pq, 64);
        const int pb = __shfl(body, 4 * pq, 64);
        bool cand = base + l < npair && po != pb;
        {
          const double* bb = b.b_diag + 16 * pb + 2;
          const double* ob = b.b_diag + 16 * po + 2;
          const double* os = b.b_diag + 16 * po + 9;
#pragma unroll
          for (int k = 0; k < 3; k++)
            if (bb[k] > ob[3 + k] + 1.0 || ob[k] > bb[3 + k] + 1.0) cand = false;
          if (px < ob[0] - 1.0 || px > ob[3] + 1.0 || py < ob[1] - 1.0 || py > ob[4] + 1.0 ||
              pz < ob[2] - 1.0 || pz > ob[5] + 1.0)
            cand = false;
          const double sx = px - os[0], sy = py - os[1], sz = pz - os[2];
          if (sx * sx + sy * sy + sz * sz > (os[3] + 1.0) * (os[3] + 1.0)) cand = false;
        }
        unsigned long long m = __ballot(cand);
        while (m) {
          const int bit = __ffsll((unsigned long long)m) - 1;
          m &= m - 1;
          const int q = (base + bit) / b.nbody, o = base + bit - q * b.nbody;
          if (q != cur_q) {
            if (cur_q >= 0) {
              const double tot = red64(part);
              if ((l >> 2) == cur_q) acc = tot;
            }
            cur_q = q;
            part = 0.0;
          }
          const double qx = __shfl(cen[0], 4 * q, 64), qy = __shfl(cen[1], 4 * q, 64),
                       qz = __shfl(cen[2], 4 * q, 64);
          // the lanes test o's chunks in parallel (a centroid c of a chunk
          // has floor(c + 1/2) inside the chunk's box of bases, so a face
          // farther than 1.5 from that box has no partner there); the
          // surviving chunks are scanned one centroid per lane (centroids
          // are stored by slot)
          const int c0 = b.b_chunk0[o], c1 = b.b_chunk0[o + 1] - 1;
          for (int cb0 = c0; cb0 <= c1; cb0 += 64) {
            bool near = false;
            if (cb0 + l <= c1) {
              const int* cb = b.chunk_box + 6 * (cb0 + l);
              near = !(qx < cb[0] - 1.5 || qx > cb[3] + 1.5 || qy < cb[1] - 1.5 || qy > cb[4] + 1.5 ||
                       qz < cb[2] - 1.5 || qz > cb[5] + 1.5);
            }
            unsigned long long mc = __ballot(near);
            while (mc) {
              const int cbit = __ffsll((unsigned long long)mc) - 1;
              mc &= mc - 1;
              const int cb = cb0 + cbit;
              if (l < b.chunk_n[cb]) {
                const int g = b.chunk_s0[cb] + l;
                const double* cj = b.centroid + 3 * g;
                const double ddx = qx - cj[0], ddy = qy - cj[1], ddz = qz - cj[2];
                const double d = sqrt(ddx * ddx + ddy * ddy + ddz * ddz);
                if (d < 1.0 && d > 0.0) part += 1.0 / sqrt(d * d * d * d * d);
              }
            }
          }
        }
      }
      if (cur_q >= 0) {
        const double tot = red64(part);
        if ((l >> 2) == cur_q) acc = tot;
      }
    }
    if (l < 32 && sub == 0 && valid) {
      const double nu = b.nu;
      const double dp = (rfit - r_in) / 3.0;
      double F[3];
#pragma unroll
      for (int i = 0; i < 3; i++) {
        double tn = 0.0;
#pragma unroll
        for (int c = 0; c < 3; c++) {
          const double tp = rfit * nu * (G[i][c] + G[c][i]);
          const double tm = r_in * nu * (Gin[i][c] + Gin[c][i]);
          tn += (tp - tm) * nrm[c];
        }
        F[i] = (-dp * nrm[i] + tn) * area;
      }
      const double pref = b.umax / (8.0 * sqrt(2.0));
      double cv = 0.0;
      if (!b.b_rigid[body]) {
        const double V0 = b.b_param[8 * body], kv = b.b_param[8 * body + 2];
        cv = kv * (1.0 - b.b_diag[16 * body] / V0) * area;
      }
      double Ft[3];
#pragma unroll
      for (int i = 0; i < 3; i++) {
        Ft[i] = F[i] - pref * acc * nrm[i] + cv * nrm[i];
        b.fext[3 * f + i] = Ft[i];
      }
      // a third of the face force at each of its vertices
#pragma unroll
      for (int r = 0; r < 3; r++) {
        const long long sl = b.sl_face[3 * f + r];
        const int vr = b.faces[3 * f + r];
#pragma unroll
        for (int i = 0; i < 3; i++) b.f_slot[(sl * 3 + i) * b.nv + vr] = Ft[i] / 3.0;
      }
    }
    return;
  }
  if (b.nsoft_v == 0) return;
  const int idx = (gw - nfw) * MLS_VERTS_PER_WAVE + (l >> 2);
  const bool valid = idx < b.nsoft_v;
  const int v = b.soft_vlist[valid ? idx : b.nsoft_v - 1];
  double rfit, U[3], G[3][3];
  fit_point<S>(a, sub, b.Xcur[3 * v], b.Xcur[3 * v + 1], b.Xcur[3 * v + 2], false, rfit, U, G);
  if (valid && sub == 0) {
    b.u0v[3 * v] = U[0];
    b.u0v[3 * v + 1] = U[1];
    b.u0v[3 * v + 2] = U[2];
  }
}

// Blocks of the probe / vertex-velocity part of the launch.
__host__ __device__ __forceinline__ int mls_post_blocks(const BodyArgs& b) {
  const long long waves = (long long)(b.nf + MLS_FACES_PER_WAVE - 1) / MLS_FACES_PER_WAVE +
                          (b.nsoft_v + MLS_VERTS_PER_WAVE - 1) / MLS_VERTS_PER_WAVE;
  return (int)((waves * 64 + 255) / 256);
}

// The launch also clears the force tiles of the previous step (the buffer
// the next step spreads into).  It runs after the forcing launch has checked
// the positions: a damage stop raised there skips this launch, so the force
// of the last completed step survives the stop.
template <class S>
__device__ __forceinline__ void mls_post_unit(const FluidArgs& a, const BodyArgs& b, long long* fxp,
                                              uint8_t* tfp, int blk) {
  const int nm = mls_post_blocks(b);
  if (blk < nm) mls_post_block<S>(a, b, blk);
  else clear_tiles(a.g, fxp, tfp, blk - nm, b.n_clear_blocks);
}

template <class S>
__global__ __launch_bounds__(256) void k_mls_post(FluidArgs a, BodyArgs b, long long* fxp, uint8_t* tfp) {
  if (a.flags->stop) return;
  mls_post_unit<S>(a, b, fxp, tfp, blockIdx.x);
}

// ----------------------------------------------------------- k_body_post
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

// Rigid body (one block): total force and moment about the centre of mass
// from one third of each face force at its vertices, second-order backward
// update of u and omega (Eq. angularVelRig with the Newton-Euler system,
// inertia rotated with the body), x_c += u, rotation by omega (Rodrigues).
__device__ void rigid_block(const BodyArgs& b, int body) {
  __shared__ double sh[8];
  __shared__ double rs[32];
  const int v0 = b.b_vert0[body], nv = b.b_nv[body];
  double* st = b.b_rig + 32 * body;
  if (b.b_fixed[body]) {
    for (int v = threadIdx.x; v < nv; v += blockDim.x)
      for (int k = 0; k < 3; k++) {
        b.Xnext[3 * (v0 + v) + k] = b.Xcur[3 * (v0 + v) + k];
        b.Vel[3 * (v0 + v) + k] = 0.0;
      }
    return;
  }
  const int f0 = b.b_face0[body], nf = b.b_nf[body];
  double F[3] = {0, 0, 0}, M[3] = {0, 0, 0};
  const double xc[3] = {st[0], st[1], st[2]};
  for (int f = threadIdx.x; f < nf; f += blockDim.x) {
    const double* Ff = b.fext + 3 * (f0 + f);
    for (int k = 0; k < 3; k++) F[k] += Ff[k];
    const double Fv[3] = {Ff[0] / 3.0, Ff[1] / 3.0, Ff[2] / 3.0};
    for (int c = 0; c < 3; c++) {
      const int v = b.faces[3 * (f0 + f) + c];
      const double r[3] = {b.Xcur[3 * v] - xc[0], b.Xcur[3 * v + 1] - xc[1], b.Xcur[3 * v + 2] - xc[2]};
      double t[3];
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
    const double mass = b.b_param[8 * body + 4];
    double Ibm[9];  // body-frame inertia tensor, stored after the [nbody][8] parameters
    for (int k = 0; k < 9; k++) Ibm[k] = b.b_param[8 * b.nbody + 9 * body + k];
    double RI[9], Iw[9];
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
}

// Soft vertex: gather the element forces (stretching per edge, bending per
// hinge, one third of each face's volume + hydrodynamic + repulsion force),
// then the Verlet update with the MLS tentative velocity (Eqs. verletPos,
// verletVel, verletPosC, dt = 1).
__device__ void soft_vertex(const BodyArgs& b, int idx) {
  const int v = b.soft_vlist[idx];
  const int body = b.vert_body[v];
  const double* x = b.Xcur;
  const double xv[3] = {x[3 * v], x[3 * v + 1], x[3 * v + 2]};
  // sum of the element forces written into this vertex's slots (stretching,
  // bending, a third of each incident face's force), in slot order; the
  // slot-major layout makes every load coalesced across the wave
  double F[3] = {0.0, 0.0, 0.0};
  double val[VT_SLOTS][3];
#pragma unroll
  for (int k = 0; k < VT_SLOTS; k++)
#pragma unroll
    for (int c = 0; c < 3; c++) val[k][c] = b.f_slot[((long long)k * 3 + c) * b.nv + v];
#pragma unroll
  for (int k = 0; k < VT_SLOTS; k++)
#pragma unroll
    for (int c = 0; c < 3; c++) F[c] += val[k][c];
  const double mv = b.b_param[8 * body + 3];
  for (int k = 0; k < 3; k++) {
    const double acc = 0.5 * F[k] / mv;
    const double xt = xv[k] + b.u0v[3 * v + k] + acc;                  // predictor
    const double un = 1.5 * xt - 2.0 * xv[k] + 0.5 * b.Xnext[3 * v + k];  // velocity
    b.Xnext[3 * v + k] = xv[k] + un + acc;                             // corrector
    b.Vel[3 * v + k] = un;
  }
}

// Last IB launch of a coupled step: rigid blocks, then soft-vertex blocks
// (one vertex per thread, 64-thread blocks).  With a counter, the last block
// to finish closes the step (what k_close does), so that a coupled step is
// four launches: worth it for a few tens of blocks (one capsule: 42 blocks,
// 4 us saved per step); with hundreds, each block's wait for its stores
// before it is counted costs more than the k_close launch (16 capsules:
// +5.8 us against 4.6 us), and k_close follows instead.
__device__ __forceinline__ void body_post_block(const BodyArgs& b, int blk) {
  if (blk < b.nbody) {
    if (b.b_rigid[blk]) rigid_block(b, blk);
  } else {
    const int idx = (blk - b.nbody) * (int)blockDim.x + threadIdx.x;
    if (idx < b.nsoft_v) soft_vertex(b, idx);
  }
}

__global__ __launch_bounds__(256) void k_body_post(BodyArgs b, DevFlags* flags, unsigned int* counter) {
  if (flags->stop) return;  // read before any block closes: every block returns here, or none
  body_post_block(b, blockIdx.x);
  if (counter && last_block(counter, gridDim.x) && threadIdx.x == 0) {
    const unsigned int pend =
        __hip_atomic_load(&flags->pending, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    flags->steps_done += 1;
    flags->stop |= pend;
    flags->pending = 0u;
    *counter = 0u;
  }
}

// ------------------------------------------------------------ batches
// A batch advances independent contexts together: each phase of a coupled
// step is one launch over the work units of all of them.  Block g of a
// phase takes unit map[g] = (instance, block of that instance's own launch);
// the instance's arguments are read from a device table (per step parity).
// The tables are read through the constant address space: with a uniform
// address such a load is a scalar load into SGPRs, and the compiler may
// reload a field where it is used instead of holding it (a plain global
// pointer gets vector loads, and every field then held in a VGPR).
typedef const __attribute__((address_space(4))) BatchItem CBatchItem;
typedef const __attribute__((address_space(4))) int CInt;
__device__ __forceinline__ int2 batch_unit_at(const int2* map, int u) {
  const CInt* p = (const CInt*)map;
  return make_int2(p[2 * u], p[2 * u + 1]);
}
__device__ __forceinline__ int2 batch_unit(const int2* map) { return batch_unit_at(map, blockIdx.x); }
__device__ __forceinline__ const BatchItem& batch_item(const BatchItem* items, int k) {
  return *(const BatchItem*)&((CBatchItem*)items)[k];
}

template <class S>
__global__ __launch_bounds__(256, sizeof(S) == 8 ? 1 : 2) void kb_ib_force(const BatchItem* items,
                                                                          const int2* map) {
  const int2 m = batch_unit(map);
  const BatchItem& it = batch_item(items, m.x);
  if (it.a.flags->stop) return;
  ib_force_block<S>(it.a, it.b, it.fxc, it.tfc, it.fxp, it.tfp, it.counter, m.y);
}

// Fluid phase.  Merged form: records and bulk tiles of every instance in
// one launch (unit = record block or bulk tile).  Split form: the record
// blocks of all instances, then the bulk tiles of all instances, each
// kernel with its own register budget (the bulk kernel keeps the occupancy
// that the bandwidth-bound part needs).  The host orders every map so that
// each XCD takes a contiguous run of units (whole instances where possible).
template <class S, int V, bool PERX>
__global__ __launch_bounds__(256) void kb_fluid_all(const BatchItem* items, const int2* map) {
  const int2 m = batch_unit(map);
  const FluidArgs a = batch_item(items, m.x).a;
  if (a.flags->stop) return;
  fluid_unit<S, V, PERX>(a, batch_item(items, m.x).nrb, m.y);
}

// Persistent form (its own kernel: holding an instance's arguments across
// units takes registers the one-unit form does not need): per_xcd blocks on
// each of the 8 XCDs walk the XCD's contiguous share of the units; an
// instance's arguments are loaded once per run of its units.
template <class S, int V, bool PERX>
__global__ __launch_bounds__(256) void kb_fluid_all_persist(const BatchItem* items, const int2* map,
                                                            int nunits, int per_xcd) {
  const int x = blockIdx.x & 7, j = blockIdx.x >> 3;
  const int u0 = (int)(((long long)nunits * x) >> 3), u1 = (int)(((long long)nunits * (x + 1)) >> 3);
  int cur = -1, nrb = 0;
  bool stop = true;
  FluidArgs a;
  for (int u = u0 + j; u < u1; u += per_xcd) {
    const int2 m = batch_unit_at(map, u);
    if (m.x != cur) {
      cur = m.x;
      a = batch_item(items, m.x).a;
      nrb = batch_item(items, m.x).nrb;
      stop = a.flags->stop != 0u;
    }
    if (!stop) fluid_unit<S, V, PERX>(a, nrb, m.y);
  }
}

template <class S>
__global__ __launch_bounds__(256) void kb_fluid_rec(const BatchItem* items, const int2* map) {
  const int2 m = batch_unit(map);
  const FluidArgs a = batch_item(items, m.x).a;
  if (a.flags->stop) return;
  const int r = m.y * blockDim.x + threadIdx.x;
  if (r < a.nrec) fluid_record_thread<S>(a, r);
}

// Bulk tiles; per_xcd > 0 is the persistent form: per_xcd blocks on each of
// the 8 XCDs walk the XCD's contiguous share of the units in strides of
// per_xcd.
template <class S, int V, bool PERX>
__global__ __launch_bounds__(256) void kb_fluid_bulk(const BatchItem* items, const int2* map) {
  const int2 m = batch_unit(map);
  const FluidArgs a = batch_item(items, m.x).a;
  if (a.flags->stop) return;
  fluid_bulk<S, V, PERX>(a, m.y);
}

template <class S, int V, bool PERX>
__global__ __launch_bounds__(256) void kb_fluid_bulk_persist(const BatchItem* items, const int2* map,
                                                             int nunits, int per_xcd) {
  const int x = blockIdx.x & 7, j = blockIdx.x >> 3;
  const int u0 = (int)(((long long)nunits * x) >> 3), u1 = (int)(((long long)nunits * (x + 1)) >> 3);
  int cur = -1;
  bool stop = true;
  FluidArgs a;
  for (int u = u0 + j; u < u1; u += per_xcd) {
    const int2 m = batch_unit_at(map, u);
    if (m.x != cur) {  // an instance's arguments once per run of its units
      cur = m.x;
      a = batch_item(items, m.x).a;
      stop = a.flags->stop != 0u;
    }
    if (!stop) fluid_bulk<S, V, PERX>(a, m.y);
  }
}

template <class S>
__global__ __launch_bounds__(256) void kb_mls_post(const BatchItem* items, const int2* map) {
  const int2 m = batch_unit(map);
  const BatchItem& it = batch_item(items, m.x);
  if (it.a.flags->stop) return;
  mls_post_unit<S>(it.a, it.b, it.fxp, it.tfp, m.y);
}

__global__ __launch_bounds__(256) void kb_body_post(const BatchItem* items, const int2* map) {
  const int2 m = batch_unit(map);
  const BatchItem& it = batch_item(items, m.x);
  if (it.a.flags->stop) return;
  body_post_block(it.b, m.y);
}

// Closes a step of every instance (one thread each).
__global__ void kb_close(const BatchItem* items, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  DevFlags* flags = items[i].a.flags;
  if (flags->stop) return;
  const unsigned int pend =
      __hip_atomic_load(&flags->pending, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  flags->steps_done += 1;
  flags->stop |= pend;
  flags->pending = 0u;
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

template <class S, int V>
static void bulk_launch(const FluidArgs& a, unsigned grid, hipStream_t s) {
  if (a.g.per[0]) k_fluid_bulk<S, V, true><<<grid, a.bulk_block, 0, s>>>(a);
  else k_fluid_bulk<S, V, false><<<grid, a.bulk_block, 0, s>>>(a);
}

hipError_t launch_fluid_bulk(int prec, const FluidArgs& a, hipStream_t s) {
  if (a.nbulk_blocks == 0) return hipSuccess;
  const unsigned grid = (unsigned)a.nbulk_blocks;
  switch (prec * 16 + (a.bulk_v == 0 ? 1 : a.bulk_v)) {  // 0: list form, one node per thread
    case 0 * 16 + 1: bulk_launch<double, 1>(a, grid, s); break;
    case 0 * 16 + 2: bulk_launch<double, 2>(a, grid, s); break;
    case 1 * 16 + 1: bulk_launch<float, 1>(a, grid, s); break;
    case 1 * 16 + 2: bulk_launch<float, 2>(a, grid, s); break;
    case 1 * 16 + 4: bulk_launch<float, 4>(a, grid, s); break;
    case 2 * 16 + 1: bulk_launch<_Float16, 1>(a, grid, s); break;
    case 2 * 16 + 2: bulk_launch<_Float16, 2>(a, grid, s); break;
    case 2 * 16 + 4: bulk_launch<_Float16, 4>(a, grid, s); break;
    case 2 * 16 + 8: bulk_launch<_Float16, 8>(a, grid, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_fluid_rec(int prec, const FluidArgs& a, hipStream_t s) {
  if (a.nrec == 0) return hipSuccess;
  const unsigned grid = cdiv(a.nrec, a.rec_block);
  const unsigned blk = (unsigned)a.rec_block;
  switch (prec) {
    case 0: k_fluid_rec<double><<<grid, blk, 0, s>>>(a); break;
    case 1: k_fluid_rec<float><<<grid, blk, 0, s>>>(a); break;
    default: k_fluid_rec<_Float16><<<grid, blk, 0, s>>>(a); break;
  }
  return hipGetLastError();
}

template <class S, int V>
static void all_launch(const FluidArgs& a, int nrb, unsigned grid, hipStream_t s) {
  if (a.g.per[0]) k_fluid_all<S, V, true><<<grid, a.bulk_block, 0, s>>>(a, nrb);
  else k_fluid_all<S, V, false><<<grid, a.bulk_block, 0, s>>>(a, nrb);
}

hipError_t launch_fluid_all(int prec, const FluidArgs& a, hipStream_t s) {
  const int nrb = a.nrec > 0 ? (int)cdiv(a.nrec, a.bulk_block) : 0;
  const unsigned grid = (unsigned)(nrb + a.nbulk_blocks);
  if (grid == 0) return hipSuccess;
  switch (prec * 16 + (a.bulk_v == 0 ? 1 : a.bulk_v)) {  // 0: list form
    case 0 * 16 + 1: all_launch<double, 1>(a, nrb, grid, s); break;
    case 0 * 16 + 2: all_launch<double, 2>(a, nrb, grid, s); break;
    case 1 * 16 + 1: all_launch<float, 1>(a, nrb, grid, s); break;
    case 1 * 16 + 2: all_launch<float, 2>(a, nrb, grid, s); break;
    case 1 * 16 + 4: all_launch<float, 4>(a, nrb, grid, s); break;
    case 2 * 16 + 1: all_launch<_Float16, 1>(a, nrb, grid, s); break;
    case 2 * 16 + 2: all_launch<_Float16, 2>(a, nrb, grid, s); break;
    case 2 * 16 + 4: all_launch<_Float16, 4>(a, nrb, grid, s); break;
    case 2 * 16 + 8: all_launch<_Float16, 8>(a, nrb, grid, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_close(DevFlags* flags, hipStream_t s) {
  k_close<<<1, 1, 0, s>>>(flags);
  return hipGetLastError();
}

hipError_t launch_ib_force(int prec, const FluidArgs& a, const BodyArgs& b, long long* fxc,
                           uint8_t* tfc, long long* fxp, uint8_t* tfp, unsigned int* counter,
                           hipStream_t s) {
  const unsigned grid = (unsigned)(b.n_marker_blocks + b.n_elem_blocks + b.n_diag_blocks);
  if (grid == 0) return hipSuccess;
  switch (prec) {
    case 0: k_ib_force<double><<<grid, 256, 0, s>>>(a, b, fxc, tfc, fxp, tfp, counter); break;
    case 1: k_ib_force<float><<<grid, 256, 0, s>>>(a, b, fxc, tfc, fxp, tfp, counter); break;
    default: k_ib_force<_Float16><<<grid, 256, 0, s>>>(a, b, fxc, tfc, fxp, tfp, counter); break;
  }
  return hipGetLastError();
}

hipError_t launch_mls_post(int prec, const FluidArgs& a, const BodyArgs& b, long long* fxp, uint8_t* tfp,
                           hipStream_t s) {
  if (b.nf == 0) return hipSuccess;
  const unsigned grid = (unsigned)(mls_post_blocks(b) + b.n_clear_blocks);
  switch (prec) {
    case 0: k_mls_post<double><<<grid, 256, 0, s>>>(a, b, fxp, tfp); break;
    case 1: k_mls_post<float><<<grid, 256, 0, s>>>(a, b, fxp, tfp); break;
    default: k_mls_post<_Float16><<<grid, 256, 0, s>>>(a, b, fxp, tfp); break;
  }
  return hipGetLastError();
}

hipError_t launch_body_post(const BodyArgs& b, DevFlags* flags, unsigned int* counter, hipStream_t s) {
  // small blocks: the vertex gathers are spread over many CUs' load pipelines
  k_body_post<<<body_post_blocks(b), 64, 0, s>>>(b, flags, counter);
  return hipGetLastError();
}

hipError_t launch_batch_ib_force(int prec, const BatchItem* items, const int2* map, int n,
                                 hipStream_t s) {
  if (n == 0) return hipSuccess;
  switch (prec) {
    case 0: kb_ib_force<double><<<n, 256, 0, s>>>(items, map); break;
    case 1: kb_ib_force<float><<<n, 256, 0, s>>>(items, map); break;
    default: kb_ib_force<_Float16><<<n, 256, 0, s>>>(items, map); break;
  }
  return hipGetLastError();
}

template <class S, int V>
static void batch_fluid_launch(const BatchFluid& f, const BatchItem* items, hipStream_t s) {
  if (f.mode == 0) {
    if (f.n_all && f.per_xcd > 0)
      kb_fluid_all_persist<S, V, false><<<8u * f.per_xcd, f.block, 0, s>>>(items, f.map_all, f.n_all, f.per_xcd);
    else if (f.n_all)
      kb_fluid_all<S, V, false><<<f.n_all, f.block, 0, s>>>(items, f.map_all);
    return;
  }
  if (f.n_rec) kb_fluid_rec<S><<<f.n_rec, f.block, 0, s>>>(items, f.map_rec);
  if (f.n_bulk && f.per_xcd > 0)
    kb_fluid_bulk_persist<S, V, false><<<8u * f.per_xcd, f.block, 0, s>>>(items, f.map_bulk, f.n_bulk, f.per_xcd);
  else if (f.n_bulk)
    kb_fluid_bulk<S, V, false><<<f.n_bulk, f.block, 0, s>>>(items, f.map_bulk);
}

hipError_t launch_batch_fluid(int prec, const BatchFluid& f, const BatchItem* items, hipStream_t s) {
  switch (prec * 16 + (f.V == 0 ? 1 : f.V)) {  // 0: list form
    case 0 * 16 + 1: batch_fluid_launch<double, 1>(f, items, s); break;
    case 0 * 16 + 2: batch_fluid_launch<double, 2>(f, items, s); break;
    case 1 * 16 + 1: batch_fluid_launch<float, 1>(f, items, s); break;
    case 1 * 16 + 2: batch_fluid_launch<float, 2>(f, items, s); break;
    case 1 * 16 + 4: batch_fluid_launch<float, 4>(f, items, s); break;
    case 2 * 16 + 1: batch_fluid_launch<_Float16, 1>(f, items, s); break;
    case 2 * 16 + 2: batch_fluid_launch<_Float16, 2>(f, items, s); break;
    case 2 * 16 + 4: batch_fluid_launch<_Float16, 4>(f, items, s); break;
    case 2 * 16 + 8: batch_fluid_launch<_Float16, 8>(f, items, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_batch_mls_post(int prec, const BatchItem* items, const int2* map, int n,
                                 hipStream_t s) {
  if (n == 0) return hipSuccess;
  switch (prec) {
    case 0: kb_mls_post<double><<<n, 256, 0, s>>>(items, map); break;
    case 1: kb_mls_post<float><<<n, 256, 0, s>>>(items, map); break;
    default: kb_mls_post<_Float16><<<n, 256, 0, s>>>(items, map); break;
  }
  return hipGetLastError();
}

hipError_t launch_batch_body_post(const BatchItem* items, const int2* map, int n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  kb_body_post<<<n, 64, 0, s>>>(items, map);
  return hipGetLastError();
}

hipError_t launch_batch_close(const BatchItem* items, int n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  kb_close<<<cdiv(n, 64), 64, 0, s>>>(items, n);
  return hipGetLastError();
}

// Global FP64 mass and momentum of the populations of the last completed
// step: per block, each thread sums its nodes in index order, then a fixed
// tree; k_diag_final sums the blocks in a fixed order (bitwise reproducible).
constexpr int DIAG_SUM_BLOCKS = 1024;

template <class S>
__global__ __launch_bounds__(256) void k_diag_sum(Grid G, const S* f0, const S* f1, const uint8_t* ncls,
                                                  const DevFlags* flags, double* part) {
  __shared__ double sh[8];
  const S* f = (flags->steps_done & 1) ? f1 : f0;
  double v[5] = {0.0, 0.0, 0.0, 0.0, 0.0};  // non-solid nodes, sum of deviations, momentum
  for (long long p = blockIdx.x * 256LL + threadIdx.x; p < G.Np; p += (long long)gridDim.x * 256) {
    if (ncls[p] == CLS_SOLID) continue;
    v[0] += 1.0;
#pragma unroll
    for (int i = 0; i < 19; i++) {
      const double g = (double)to_c(f[(long long)i * G.plane + p]);
      v[1] += g;
      v[2] += EX[i] * g;
      v[3] += EY[i] * g;
      v[4] += EZ[i] * g;
    }
  }
#pragma unroll
  for (int k = 0; k < 5; k++) {
    const double t = block_sum(v[k], sh);
    if (threadIdx.x == 0) part[5 * blockIdx.x + k] = t;
  }
}

__global__ __launch_bounds__(256) void k_diag_final(const double* part, int nblk, double* out) {
  __shared__ double sh[8];
  for (int k = 0; k < 5; k++) {
    double v = 0.0;
    for (int j = threadIdx.x; j < nblk; j += blockDim.x) v += part[5 * j + k];
    v = block_sum(v, sh);
    if (threadIdx.x == 0) out[k] = v;
  }
}

hipError_t launch_diag_sums(int prec, const Grid& g, const void* f0, const void* f1, const uint8_t* ncls,
                            const DevFlags* flags, double* part, double* out, hipStream_t s) {
  switch (prec) {
    case 0: k_diag_sum<double><<<DIAG_SUM_BLOCKS, 256, 0, s>>>(g, (const double*)f0, (const double*)f1, ncls, flags, part); break;
    case 1: k_diag_sum<float><<<DIAG_SUM_BLOCKS, 256, 0, s>>>(g, (const float*)f0, (const float*)f1, ncls, flags, part); break;
    default: k_diag_sum<_Float16><<<DIAG_SUM_BLOCKS, 256, 0, s>>>(g, (const _Float16*)f0, (const _Float16*)f1, ncls, flags, part); break;
  }
  k_diag_final<<<1, 256, 0, s>>>(part, DIAG_SUM_BLOCKS, out);
  return hipGetLastError();
}

// ------------------------------------------------------------- adjoint
// Discrete adjoint of the fluid step (FP64, no bodies).  One step maps the
// post-collision deviations g^k to g^{k+1} = C(P(g^k)): P is the streaming
// (plain pulls, interpolated bounce-back, Zou-He -- affine in g^k) and C
// the forced BGK collision of each node.  Given lam = dJ/dg^{k+1}, the step
// back is mu = (dC/dh)^T lam node by node, then lam' = P^T mu.
__device__ __forceinline__ bool zh_unknown(int fc, int j) {
  const int face = fc & 7, ax = face >> 1, sg = (face & 1) ? -1 : 1;
  return fc != 0xff && sg * (ax == 0 ? EX[j] : (ax == 1 ? EY[j] : EZ[j])) == 1;
}

// One forward step of the fluid in the context's precision (storage S, the
// same pull and collision as the stream-collide kernels) from a.A into a.B:
// bulk node t of a.bulk_list, or
// boundary record r.  Solid nodes are not written (they hold zero in every
// buffer of the sweep).  hrec (may be null): [19][nrec], the records'
// populations entering the collision (after Zou-He), kept for the step back.
template <class S>
__device__ __forceinline__ void adj_fwd_bulk_one(const FluidArgs& a, int t) {
  typedef typename Store<S>::C C;
  const Grid& G = a.g;
  const long long n = a.bulk_list[t];
  S* B = (S*)a.B;
  int x, y, z;
  coords(G, n, x, y, z);
  C g[19], dr, ux, uy, uz, Fx, Fy, Fz;
  const Hood h = hood(G, x, y, z);
#pragma unroll
  for (int j = 0; j < 19; j++) g[j] = ldA<S>(a, j, h.at(-EX[j], -EY[j], -EZ[j]));
  node_force<C>(a, n, a.tflag && a.tflag[n >> TILE_SHIFT], Fx, Fy, Fz);
  collide<C>(g, Fx, Fy, Fz, (C)a.omega, dr, ux, uy, uz);
  if (a.mac) store_mac<C>(a, n, dr, ux, uy, uz);
#pragma unroll
  for (int j = 0; j < 19; j++) B[(long long)j * G.plane + n] = (S)g[j];
}

template <class S>
__device__ __forceinline__ void adj_fwd_rec_one(const FluidArgs& a, double* hrec, int r) {
  typedef typename Store<S>::C C;
  C g[19], dr, ux, uy, uz, Fx, Fy, Fz;
  pull_general<S>(a, r, g);
  if (hrec) {
#pragma unroll
    for (int j = 0; j < 19; j++) hrec[(long long)j * a.nrec + r] = (double)g[j];
  }
  const long long n = a.rec_node[r];
  node_force<C>(a, n, a.tflag && a.tflag[n >> TILE_SHIFT], Fx, Fy, Fz);
  collide<C>(g, Fx, Fy, Fz, (C)a.omega, dr, ux, uy, uz);
  if (a.mac) store_mac<C>(a, n, dr, ux, uy, uz);
  S* B = (S*)a.B;
#pragma unroll
  for (int j = 0; j < 19; j++) B[(long long)j * a.g.plane + n] = (S)g[j];
}

// Split form: the bulk kernel keeps the small register budget of the plain
// pull; merged form (small grids): the records' latency-bound blocks run
// alongside the bulk blocks in one launch (blocks below rec_blocks take
// records).
template <class S>
__global__ __launch_bounds__(256) void k_adj_fwd_bulk(FluidArgs a) {
  const int t = blockIdx.x * 256 + threadIdx.x;
  if (t < a.nbulk_nodes) adj_fwd_bulk_one<S>(a, t);
}

template <class S>
__global__ __launch_bounds__(256) void k_adj_fwd_rec(FluidArgs a, double* hrec) {
  const int r = blockIdx.x * 256 + threadIdx.x;
  if (r < a.nrec) adj_fwd_rec_one<S>(a, hrec, r);
}

// Block b of a merged launch -> record block or bulk block, each part's
// blocks remapped so that every XCD takes a contiguous run (neighbouring
// rows share its L2).
__device__ __forceinline__ int adj_unit(int b, int rec_blocks, int nblocks) {
  return b < rec_blocks ? xcd_remap(b, rec_blocks) : rec_blocks + xcd_remap(b - rec_blocks, nblocks - rec_blocks);
}

template <class S>
__global__ __launch_bounds__(256) void k_adj_fwd_all(FluidArgs a, double* hrec, int rec_blocks) {
  const int u = adj_unit(blockIdx.x, rec_blocks, gridDim.x);
  if (u < rec_blocks) {
    const int r = u * 256 + threadIdx.x;
    if (r < a.nrec) adj_fwd_rec_one<S>(a, hrec, r);
  } else {
    const int t = (u - rec_blocks) * 256 + threadIdx.x;
    if (t < a.nbulk_nodes) adj_fwd_bulk_one<S>(a, t);
  }
}

// The transpose of the collision's Jacobian, written out: with
// Phi = sum_i l_i (omega g^eq_i + G_i) as a function of (rho - 1, u, F),
//   P   = dPhi/d(rho - 1) at fixed u,  U_a = dPhi/du_a,  Q_a = dPhi/dF_a at fixed u,
// and du_a/dh_j = (e_ja - u_a)/rho, d(rho - 1)/dh_j = 1, du_a/dF_a = 1/(2 rho):
//   mu_j = (1 - omega) l_j + P + sum_a U_a (e_ja - u_a)/rho,
//   dJ/dF_a += Q_a + U_a/(2 rho).
// With the sums over i of w_i l_i times 1, (1 + 3 e.u + 9/2 (e.u)^2 - 3/2 u.u),
// (3 + 9 e.u) e_a and (e.F) e_a (SL, P', V_a, Z_a):
//   P = omega P',  U_a = omega rho V_a + 9 kf Z_a - 3 (omega rho u_a + kf F_a) SL,
//   Q_a = kf (V_a - 3 u_a SL),  kf = 1 - omega/2.
// dF[3] += dJ/d(omega) at fixed h: sum_i l_i (g^eq_i - h_i - G_i / (2 kf)).
// With bodies, x7 adds adjoint sources at the node: x7[0] = dJ/drho and
// x7[1..3] = dJ/du of the step's fields (read by the probes and the vertex
// velocities; u depends on F, so they enter dJ/dF too), x7[4..6] = dJ/du*
// of the pre-force velocity u* = m / rho that the forcing markers read
// (mu_j += dJ/du* . (e_j - u*) / rho).  dFn: this node's dJ/dF, dw: dJ/d(omega).
__device__ __forceinline__ void collide_vjp(const double (&h)[19], const double (&l)[19], double Fx, double Fy,
                                            double Fz, double omega, const double (&x7)[7], double (&mu)[19],
                                            double (&dFn)[3], double& dw) {
  const double drho = dev_sum(h);
  const double mx = (h[1] - h[2]) + (h[7] + h[8]) + (h[9] + h[10]) - (h[11] + h[12]) - (h[13] + h[14]);
  const double my = (h[3] - h[4]) + (h[7] - h[8]) + (h[11] - h[12]) + (h[15] + h[16]) - (h[17] + h[18]);
  const double mz = (h[5] - h[6]) + (h[9] - h[10]) + (h[13] - h[14]) + (h[15] - h[16]) + (h[17] - h[18]);
  const double rho = 1.0 + drho, ir = 1.0 / rho;
  const double ux = (mx + 0.5 * Fx) * ir, uy = (my + 0.5 * Fy) * ir, uz = (mz + 0.5 * Fz) * ir;
  const double usq = ux * ux + uy * uy + uz * uz;
  const double kf = 1.0 - 0.5 * omega;
  const double uF = ux * Fx + uy * Fy + uz * Fz;
  double SL = 0.0, Pp = 0.0, V0 = 0.0, V1 = 0.0, V2 = 0.0, Z0 = 0.0, Z1 = 0.0, Z2 = 0.0, Dw = 0.0;
#pragma unroll
  for (int i = 0; i < 19; i++) {
    const double eu = EX[i] * ux + EY[i] * uy + EZ[i] * uz;
    const double eF = EX[i] * Fx + EY[i] * Fy + EZ[i] * Fz;
    const double wl = WD[i] * l[i];
    SL += wl;
    Pp += wl * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * usq);
    // d(out_i)/d(omega) = -(h_i - g^eq_i) - 1/2 w_i (3 (e.F - u.F) + 9 (e.u)(e.F))
    Dw += wl * (drho + rho * (3.0 * eu + 4.5 * eu * eu - 1.5 * usq) - 0.5 * (3.0 * (eF - uF) + 9.0 * eu * eF)) -
          l[i] * h[i];
    const double v = wl * (3.0 + 9.0 * eu), zz = wl * eF;
    if (EX[i]) { V0 += EX[i] * v; Z0 += EX[i] * zz; }
    if (EY[i]) { V1 += EY[i] * v; Z1 += EY[i] * zz; }
    if (EZ[i]) { V2 += EZ[i] * v; Z2 += EZ[i] * zz; }
  }
  const double orho = omega * rho;
  const double U0 = orho * V0 + 9.0 * kf * Z0 - 3.0 * (orho * ux + kf * Fx) * SL + x7[1];
  const double U1 = orho * V1 + 9.0 * kf * Z1 - 3.0 * (orho * uy + kf * Fy) * SL + x7[2];
  const double U2 = orho * V2 + 9.0 * kf * Z2 - 3.0 * (orho * uz + kf * Fz) * SL + x7[3];
  double A0 = omega * Pp + x7[0] - (U0 * ux + U1 * uy + U2 * uz) * ir;
  double a0 = U0 * ir, a1 = U1 * ir, a2 = U2 * ir;
  dFn[0] = kf * (V0 - 3.0 * ux * SL) + 0.5 * a0;
  dFn[1] = kf * (V1 - 3.0 * uy * SL) + 0.5 * a1;
  dFn[2] = kf * (V2 - 3.0 * uz * SL) + 0.5 * a2;
  dw = Dw;
  // u* = m / rho (no force): mu_j += x7[4..6] . (e_j - u*) / rho
  A0 -= (x7[4] * mx + x7[5] * my + x7[6] * mz) * ir * ir;
  a0 += x7[4] * ir;
  a1 += x7[5] * ir;
  a2 += x7[6] * ir;
#pragma unroll
  for (int j = 0; j < 19; j++) mu[j] = (1.0 - omega) * l[j] + A0 + (EX[j] * a0 + EY[j] * a1 + EZ[j] * a2);
}

// Zou-He's transpose (the rule of zouhe(), affine in the known populations
// for a fixed wall velocity or density): m = dJ/d(populations after the
// rule) -> dJ/d(populations before it), in place; gs += dJ/ds with s the
// scale of the wall velocity of a velocity face.  hz: the populations after
// the rule (its known entries are the ones before).  With c_i = 1, 2, 0 for
// e_i.n = 0, -1, +1, rho_w depends on g_i through c_i / (1 - u_n) (velocity
// face) and u_n through -c_i / rho_w (density face); the tangential sums T
// through e_i (e_i.n = 0); each unknown j adds m_j to its opposite input.
__device__ __forceinline__ void zouhe_vjp(const double (&hz)[19], double (&m)[19], int face, int kind,
                                          const double* bc, double& gs) {
  const int ax = face >> 1;
  const int sg = (face & 1) ? -1 : 1;
  double G0 = 0.0, Gout = 0.0;
#pragma unroll
  for (int j = 0; j < 19; j++) {
    const int en = sg * (ax == 0 ? EX[j] : (ax == 1 ? EY[j] : EZ[j]));
    G0 += en == 0 ? hz[j] : 0.0;
    Gout += en == -1 ? hz[j] : 0.0;
  }
  double u[3] = {bc[0], bc[1], bc[2]};
  double rho, un;
  if (kind == 0) {
    un = sg * u[ax];
    rho = (1.0 + G0 + 2.0 * Gout) / (1.0 - un);
  } else {
    rho = bc[3];
    un = (rho - 1.0 - G0 - 2.0 * Gout) / rho;
    u[0] = ax == 0 ? sg * un : 0.0;
    u[1] = ax == 1 ? sg * un : 0.0;
    u[2] = ax == 2 ? sg * un : 0.0;
  }
  // R = sum over unknowns of m_j d(fill_j)/d(rho_w) (velocity face) or
  // d(fill_j)/d(u_n) (density face); W = sum over diagonal unknowns of m_j t_j
  double R = 0.0, W[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int j = 0; j < 19; j++) {
    const int en = sg * (ax == 0 ? EX[j] : (ax == 1 ? EY[j] : EZ[j]));
    if (en != 1) continue;
    const double t[3] = {ax == 0 ? 0.0 : (double)EX[j], ax == 1 ? 0.0 : (double)EY[j], ax == 2 ? 0.0 : (double)EZ[j]};
    const bool axis = t[0] == 0.0 && t[1] == 0.0 && t[2] == 0.0;
    const double ut = u[0] * t[0] + u[1] * t[1] + u[2] * t[2];
    const double coef = kind == 0 ? (axis ? un / 3.0 : (un + ut) / 6.0 + ut / 3.0) : (axis ? rho / 3.0 : rho / 6.0);
    R += m[j] * coef;
    if (!axis) {
      W[0] += m[j] * t[0];
      W[1] += m[j] * t[1];
      W[2] += m[j] * t[2];
    }
  }
  double out[19];
#pragma unroll
  for (int i = 0; i < 19; i++) {
    const int en = sg * (ax == 0 ? EX[i] : (ax == 1 ? EY[i] : EZ[i]));
    const double c = en == 0 ? 1.0 : (en == -1 ? 2.0 : 0.0);
    double v = en != 1 ? m[i] : 0.0;
    if (en == -1) v += m[OPP[i]];  // the unknown opposite copies this input
    v += R * (kind == 0 ? c / (1.0 - un) : -c / rho);
    if (en == 0) v -= 0.5 * (W[0] * EX[i] + W[1] * EY[i] + W[2] * EZ[i]);
    out[i] = v;
  }
#pragma unroll
  for (int i = 0; i < 19; i++) m[i] = out[i];
  if (kind == 0) gs += (rho * un / (1.0 - un) + rho) * R;
}


// The bounce-back transpose of record r's links: the mu m of each linked
// direction goes back, with the rule's coefficients, to the three
// populations the rule read (FP64 atomics: several links may feed one).
template <class S>
__device__ __forceinline__ void adj_links_one(const FluidArgs& a, int r, long long node, const double (&m)[19],
                                              double* acc) {
  const uint32_t mask = a.rec_mask[r];
  if (!mask) return;
  const Grid& G = a.g;
  const uint32_t hqm = a.rec_mb[r];
  const int lk0 = a.rec_link0[r];
  const typename Store<S>::C* lc = (const typename Store<S>::C*)a.lk_c;
  const long long nl = a.nlinks;
  int x, y, z;
  coords(G, node, x, y, z);
  const Hood hd = hood(G, x, y, z);
#pragma unroll
  for (int j = 1; j < 19; j++) {
    if (!((mask >> j) & 1u)) continue;
    const int l = lk0 + __popc(mask & ((1u << j) - 1u));
    const int i = OPP[j];
    const bool hq = (hqm >> j) & 1u;
    const long long n1 = hd.at(EX[j], EY[j], EZ[j]);  // x - e_i
    const long long n2 = hd.at(2 * EX[j], 2 * EY[j], 2 * EZ[j]);
    const double k0 = (double)lc[l], k1 = (double)lc[nl + l], k2 = (double)lc[2 * nl + l];
    if (k0 != 0.0) atomicAdd(acc + (long long)i * G.plane + node, k0 * m[j]);
    if (k1 != 0.0) atomicAdd(acc + (long long)(hq ? j : i) * G.plane + (hq ? node : n1), k1 * m[j]);
    if (k2 != 0.0) atomicAdd(acc + (long long)(hq ? j : i) * G.plane + (hq ? n1 : n2), k2 * m[j]);
  }
}

// One node of the reverse step: lam = P^T mu_next at the node (plain pulls
// transposed: mu_next of direction j at the node that pulled j from here;
// plus the bounce-back transposes gathered in acc_in), then mu = (dC/dh)^T
// (lam + w) for bulk node t of a.bulk_list (REC false) or boundary record t
// (REC true; h: the populations that entered the collision, Zou-He applied,
// as the recompute kept them in hrec; at open-face records mu is then taken
// back through Zou-He and the links' transposes go to acc_out).  dF, gs += the node's derivatives of the body force and
// of the inlet-velocity scale.
template <bool REC, class S>
__device__ __forceinline__ void adj_reverse_one(const FluidArgs& a, const AdjStep& st, int t, double (&dF)[4],
                                                double& gs) {
  const Grid& G = a.g;
  double h[19], l[19], m[19];
  long long n;
  if (REC) {
    n = a.rec_node[t];
#pragma unroll
    for (int j = 0; j < 19; j++) h[j] = st.hrec[(long long)j * a.nrec + t];
  } else {
    n = a.bulk_list[t];
  }
  // with bodies: the IB force at the node, and whether the force-adjoint
  // pass (mode 1) has anything to do here
  // (mode 1 also visits the tiles of every marker's supports, flagged in etf
  // beforehand: dJ/dF is needed there even where the step's force is zero)
  const bool fflag = st.ftf && st.ftf[n >> TILE_SHIFT];
  if (st.mode == 1 && !fflag && !(st.etf && st.etf[n >> TILE_SHIFT])) return;
  int x, y, z;
  coords(G, n, x, y, z);
  const Hood hd = hood(G, x, y, z);
  if (!REC) {
#pragma unroll
    for (int j = 0; j < 19; j++) h[j] = (double)ldA<S>(a, j, hd.at(-EX[j], -EY[j], -EZ[j]));
  }
  const int q = REC ? a.nbulk_nodes + t : t;
  const uint32_t am = st.amask[q];
  if (st.lam) {
#pragma unroll
    for (int j = 0; j < 19; j++) l[j] = st.lam[(long long)j * G.plane + n];
  } else {
    const uint32_t pm = st.pmask[q];
#pragma unroll
    for (int j = 0; j < 19; j++) {
      const long long src = j == 0 ? n : hd.at(EX[j], EY[j], EZ[j]);
      double v = ((pm >> j) & 1u) ? st.mu_next[(long long)j * G.plane + src] : 0.0;
      if ((am >> j) & 1u) {
        double* pa = st.acc_in + (long long)j * G.plane + n;
        v += *pa;
        if (st.mode == 0) *pa = 0.0;
      }
      l[j] = v;
    }
  }
  if (st.w && (am >> 31)) {  // w is non-zero at this node
#pragma unroll
    for (int j = 0; j < 19; j++) l[j] += st.w[(long long)j * G.plane + n];
  }
  double Fx = a.gx, Fy = a.gy, Fz = a.gz;
  if (fflag) {
    Fx += (double)st.fx[n] * FX_INV;
    Fy += (double)st.fx[G.Np + n] * FX_INV;
    Fz += (double)st.fx[2 * G.Np + n] * FX_INV;
  }
  double x7[7] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  if (st.etf && st.etf[n >> TILE_SHIFT]) {
#pragma unroll
    for (int k = 0; k < 7; k++) x7[k] = st.ext[(long long)k * G.Np + n];
  }
  double dFn[3], dw;
  collide_vjp(h, l, Fx, Fy, Fz, a.omega, x7, m, dFn, dw);
  if (st.mode == 1) {
#pragma unroll
    for (int k = 0; k < 3; k++) st.fbar[(long long)k * G.Np + n] = dFn[k];
    return;
  }
  dF[0] += dFn[0];
  dF[1] += dFn[1];
  dF[2] += dFn[2];
  dF[3] += dw;
  if (REC) {
    const int fc = a.rec_face[t];
    if (fc != 0xff) {
      double bc[4];
      for (int q = 0; q < 4; q++) bc[q] = a.rec_bc[(long long)q * a.nrec + t];
      zouhe_vjp(h, m, fc & 7, (fc >> 4) & 1, bc, gs);
    }
  }
#pragma unroll
  for (int j = 0; j < 19; j++) st.mu[(long long)j * G.plane + n] = m[j];
  if (REC) adj_links_one<S>(a, t, n, m, st.acc_out);
}

// part[block][0..4] += the block's sums of dJ/ds, dJ/dF, dJ/d(omega)
// (fixed order: bitwise reproducible).
__device__ __forceinline__ void adj_part_add(double* part, double gs, const double (&dF)[4]) {
  __shared__ double sh[8];
  const double t0 = block_sum(gs, sh);
  const double t1 = block_sum(dF[0], sh);
  const double t2 = block_sum(dF[1], sh);
  const double t3 = block_sum(dF[2], sh);
  const double t4 = block_sum(dF[3], sh);
  if (threadIdx.x == 0) {
    double* p = part + ADJ_PART * blockIdx.x;
    p[0] += t0;
    p[1] += t1;
    p[2] += t2;
    p[3] += t3;
    p[4] += t4;
  }
}

// Split form: bulk (REC false) and records (REC true) in two launches,
// grid-stride over at most ADJ_BLOCKS blocks each (partials of the record
// launch in the second half of part).
template <bool REC, class S>
__global__ __launch_bounds__(256, REC ? 1 : 2) void k_adj_reverse(FluidArgs a, AdjStep st) {
  double dF[4] = {0.0, 0.0, 0.0, 0.0}, gs = 0.0;
  const int count = REC ? a.nrec : a.nbulk_nodes;
  for (int t = blockIdx.x * 256 + threadIdx.x; t < count; t += gridDim.x * 256)
    adj_reverse_one<REC, S>(a, st, t, dF, gs);
  adj_part_add(st.part + (REC ? ADJ_PART * ADJ_BLOCKS : 0), gs, dF);
}

// Merged form: blocks below rec_blocks take records, the rest bulk nodes.
template <class S>
__global__ __launch_bounds__(256) void k_adj_reverse_all(FluidArgs a, AdjStep st, int rec_blocks) {
  double dF[4] = {0.0, 0.0, 0.0, 0.0}, gs = 0.0;
  const int u = adj_unit(blockIdx.x, rec_blocks, gridDim.x);
  if (u < rec_blocks) {
    const int t = u * 256 + threadIdx.x;
    if (t < a.nrec) adj_reverse_one<true, S>(a, st, t, dF, gs);
  } else {
    const int t = (u - rec_blocks) * 256 + threadIdx.x;
    if (t < a.nbulk_nodes) adj_reverse_one<false, S>(a, st, t, dF, gs);
  }
  adj_part_add(st.part, gs, dF);
}

// Per non-solid node y (bulk list, then the records), once per sweep:
// pmask bit j: node y + e_j pulls direction j plainly from y; amask bit 31:
// the observable w is non-zero at y; amask bit d < 19:
// population d of y can receive a bounce-back transpose, i.e. some link
// reads it: the link of direction opp(d) or d at y, of opp(d) at y + e_d
// or y + 2 e_d, or of d at y - e_d (a superset: the coefficient and the
// branch of each link are not looked at).
__device__ __forceinline__ bool adj_linked(const FluidArgs& a, long long x, int j) {
  if (a.ncls[x] != CLS_GENERAL) return false;
  return (a.rec_mask[a.rec_of[x]] >> j) & 1u;
}

__global__ __launch_bounds__(256) void k_adj_mask(FluidArgs a, const double* w, uint32_t* pmask, uint32_t* amask) {
  const Grid& G = a.g;
  const int t = blockIdx.x * 256 + threadIdx.x;
  if (t >= a.nbulk_nodes + a.nrec) return;
  const long long y = t < a.nbulk_nodes ? (long long)a.bulk_list[t] : (long long)a.rec_node[t - a.nbulk_nodes];
  int px, py, pz;
  coords(G, y, px, py, pz);
  uint32_t m = 0, am = 0;
  for (int j = 0; j < 19; j++) {
    const long long x = j == 0 ? y : nbr(G, px, py, pz, EX[j], EY[j], EZ[j]);
    const uint8_t c = a.ncls[x];
    bool plain = c == CLS_BULK;
    if (c == CLS_GENERAL) {
      const int r = a.rec_of[x];
      plain = j == 0 || (!((a.rec_mask[r] >> j) & 1u) && !zh_unknown(a.rec_face[r], j));
    }
    m |= plain ? (1u << j) : 0u;
    if (j > 0) {
      const int o = OPP[j];
      const bool recv = adj_linked(a, y, o) || adj_linked(a, y, j) ||
                        adj_linked(a, nbr(G, px, py, pz, EX[j], EY[j], EZ[j]), o) ||
                        adj_linked(a, nbr(G, px, py, pz, 2 * EX[j], 2 * EY[j], 2 * EZ[j]), o) ||
                        adj_linked(a, nbr(G, px, py, pz, -EX[j], -EY[j], -EZ[j]), j);
      am |= recv ? (1u << j) : 0u;
    }
  }
  if (w) {
    bool nz = false;
    for (int j = 0; j < 19; j++) nz |= w[(long long)j * G.plane + y] != 0.0;
    am |= nz ? (1u << 31) : 0u;
  }
  pmask[t] = m;
  amask[t] = am;
}

// The last step of the sweep's transpose, lam = P^T mu: the plain pulls
// transposed plus the bounce-back transposes gathered in acc, at every
// non-solid node (bulk list, then the records).
__global__ __launch_bounds__(256) void k_adj_gather(FluidArgs a, const uint32_t* pmask, const uint32_t* amask,
                                                    const double* mu, const double* acc, double* lam) {
  const Grid& G = a.g;
  const int t = blockIdx.x * 256 + threadIdx.x;
  if (t >= a.nbulk_nodes + a.nrec) return;
  const long long y = t < a.nbulk_nodes ? (long long)a.bulk_list[t] : (long long)a.rec_node[t - a.nbulk_nodes];
  const uint32_t m = pmask[t], am = amask[t];
  int px, py, pz;
  coords(G, y, px, py, pz);
#pragma unroll
  for (int j = 0; j < 19; j++) {
    const long long x = j == 0 ? y : nbr(G, px, py, pz, EX[j], EY[j], EZ[j]);
    double v = ((m >> j) & 1u) ? mu[(long long)j * G.plane + x] : 0.0;
    if ((am >> j) & 1u) v += acc[(long long)j * G.plane + y];
    lam[(long long)j * G.plane + y] = v;
  }
}

// [19][N] with x fastest (N = nx ny nz) <-> the padded [19][plane] layout;
// towards the padded side only the non-solid nodes are written.
__global__ void k_adj_layout(Grid G, const uint8_t* ncls, const double* in, double* out, int to_padded) {
  const long long p = blockIdx.x * 256LL + threadIdx.x;
  if (p >= G.Np) return;
  const long long N = (long long)G.nx * G.ny * G.nz;
  const unsigned int t = (unsigned int)(p / G.px);
  const int x = (int)(p - (long long)t * G.px);
  const long long n = x + (long long)G.nx * t;
  const bool solid = ncls[p] == CLS_SOLID;  // padding included
  for (int j = 0; j < 19; j++) {
    if (to_padded) {
      if (!solid) out[(long long)j * G.plane + p] = in[(long long)j * N + n];
    } else if (x < G.nx) {
      out[(long long)j * N + n] = in[(long long)j * G.plane + p];
    }
  }
}

// grad[0..4] = dJ/ds, dJ/dF, dJ/dtau = -omega^2 dJ/d(omega), summed over the
// blocks in a fixed order.
__global__ void k_adj_grad_final(const double* part, int nblk, double omega, const double* ibsum, int nout,
                                 double* grad) {
  const int q = threadIdx.x;
  if (q >= nout) return;
  if (q == 5) {
    grad[5] = ibsum ? ibsum[1] : 0.0;
    return;
  }
  double t = 0.0;
  for (int b = 0; b < nblk; b++) t += part[ADJ_PART * b + q];
  grad[q] = q == 4 ? -omega * omega * t + (ibsum ? ibsum[0] : 0.0) : t;
}

template <class S>
static void adj_forward(const FluidArgs& a, double* hrec, int merged, hipStream_t s) {
  const int rb = (int)cdiv(a.nrec, 256), bb = (int)cdiv(a.nbulk_nodes, 256);
  if (merged) {
    if (rb + bb > 0) k_adj_fwd_all<S><<<rb + bb, 256, 0, s>>>(a, hrec, rb);
  } else {
    if (bb > 0) k_adj_fwd_bulk<S><<<bb, 256, 0, s>>>(a);
    if (rb > 0) k_adj_fwd_rec<S><<<rb, 256, 0, s>>>(a, hrec);
  }
}

hipError_t launch_adjoint_forward(int prec, const FluidArgs& a, double* hrec, int merged, hipStream_t s) {
  if (prec == 0) adj_forward<double>(a, hrec, merged, s);
  else if (prec == 1) adj_forward<float>(a, hrec, merged, s);
  else adj_forward<_Float16>(a, hrec, merged, s);
  return hipGetLastError();
}

hipError_t launch_adjoint_mask(const FluidArgs& a, const double* w, uint32_t* pmask, uint32_t* amask,
                               hipStream_t s) {
  if (a.nbulk_nodes + a.nrec > 0) k_adj_mask<<<cdiv(a.nbulk_nodes + a.nrec, 256), 256, 0, s>>>(a, w, pmask, amask);
  return hipGetLastError();
}

template <class S>
static void adj_reverse(const FluidArgs& a, const AdjStep& st, int merged, hipStream_t s) {
  const int rb = (int)cdiv(a.nrec, 256), bb = (int)cdiv(a.nbulk_nodes, 256);
  if (merged) {
    if (rb + bb > 0) k_adj_reverse_all<S><<<rb + bb, 256, 0, s>>>(a, st, rb);
  } else {
    if (bb > 0) k_adj_reverse<false, S><<<std::min(bb, ADJ_BLOCKS), 256, 0, s>>>(a, st);
    if (rb > 0) k_adj_reverse<true, S><<<std::min(rb, ADJ_BLOCKS), 256, 0, s>>>(a, st);
  }
}

hipError_t launch_adjoint_reverse(int prec, const FluidArgs& a, const AdjStep& st, int merged, hipStream_t s) {
  if (prec == 0) adj_reverse<double>(a, st, merged, s);
  else if (prec == 1) adj_reverse<float>(a, st, merged, s);
  else adj_reverse<_Float16>(a, st, merged, s);
  return hipGetLastError();
}

hipError_t launch_adjoint_gather(const FluidArgs& a, const uint32_t* pmask, const uint32_t* amask, const double* mu,
                                 const double* acc, double* lam, hipStream_t s) {
  if (a.nbulk_nodes + a.nrec > 0) {
    k_adj_gather<<<cdiv(a.nbulk_nodes + a.nrec, 256), 256, 0, s>>>(a, pmask, amask, mu, acc, lam);
  }
  return hipGetLastError();
}

hipError_t launch_adjoint_layout(const Grid& g, const uint8_t* ncls, const double* in, double* out, int to_padded,
                                 hipStream_t s) {
  k_adj_layout<<<cdiv(g.Np, 256), 256, 0, s>>>(g, ncls, in, out, to_padded);
  return hipGetLastError();
}

hipError_t launch_adjoint_grad(const double* part, int nblk, double omega, const double* ibsum, int nout,
                               double* grad, hipStream_t s) {
  k_adj_grad_final<<<1, 64, 0, s>>>(part, nblk, omega, ibsum, nout, grad);
  return hipGetLastError();
}

hipError_t launch_spread_owner(const Grid& g, const BodyArgs& b, long long* fxc, uint8_t* tfc,
                               const DevFlags* flags, hipStream_t s) {
  if (b.nbody == 0 || !b.stage) return hipSuccess;
  const dim3 grid((BOX_CELLS + 255) / 256, (unsigned)b.n_marker_blocks);
  k_spread_owner<<<grid, 256, 0, s>>>(g, b, fxc, tfc, flags);
  return hipGetLastError();
}

hipError_t launch_bin_faces(const BodyArgs& b, hipStream_t s) {
  if (b.nbody == 0) return hipSuccess;
  k_bin_faces<<<(unsigned)b.nbody, BIN_THREADS, 0, s>>>(b);
  return hipGetLastError();
}

hipError_t launch_check(const BodyArgs& b, const double* X0, const double* X1, DevFlags* flags,
                        unsigned int* counter, hipStream_t s) {
  if (b.nbody == 0) return hipSuccess;
  k_check<<<(unsigned)b.n_diag_blocks, 256, 0, s>>>(b, X0, X1, flags, counter);
  return hipGetLastError();
}

// The inverse of the populations output: the current state (the buffer of
// the completed step count's parity) takes f - w_i at every non-solid node,
// rounded to the storage type; solid nodes keep zero.
template <class S>
__global__ void k_set_pops(Grid G, S* f0, S* f1, const uint8_t* ncls, const DevFlags* flags, const double* pops) {
  const long long N = (long long)G.nx * G.ny * G.nz;
  const long long n = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (n >= N) return;
  S* f = (flags->steps_done & 1) ? f1 : f0;
  const int x = (int)(n % G.nx);
  const long long t = n / G.nx;
  const long long p = x + (long long)G.px * t;
  if (ncls[p] == CLS_SOLID) return;
  for (int i = 0; i < 19; i++) f[(long long)i * G.plane + p] = (S)(pops[(long long)i * N + n] - WD[i]);
}

hipError_t launch_set_populations(int prec, const Grid& g, void* f0, void* f1, const uint8_t* ncls,
                                  const DevFlags* flags, const double* pops, hipStream_t s) {
  const long long N = (long long)g.nx * g.ny * g.nz;
  switch (prec) {
    case 0: k_set_pops<double><<<cdiv(N, 256), 256, 0, s>>>(g, (double*)f0, (double*)f1, ncls, flags, pops); break;
    case 1: k_set_pops<float><<<cdiv(N, 256), 256, 0, s>>>(g, (float*)f0, (float*)f1, ncls, flags, pops); break;
    default:
      k_set_pops<_Float16><<<cdiv(N, 256), 256, 0, s>>>(g, (_Float16*)f0, (_Float16*)f1, ncls, flags, pops);
      break;
  }
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

// ------------------------------------------------- allocation-free spread
// Fixed-point force sums of the allocation-free spread, then its flags.  In
// host code the name stands for nothing on the device: the kernels get the
// address that hipGetSymbolAddress returned for the device in use.
static __device__ __align__(256) long long scratch[3 * NOALLOC_MAX_NODES + NOALLOC_FLAG_WORDS];

namespace {
std::mutex scratch_mu;
long long* scratch_dev[NOALLOC_MAX_DEVICES] = {};

__global__ void k_zero_words(long long* p, long long n) {
  const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}
}  // namespace

hipError_t noalloc_scratch(int device, long long** out) {
  if (device < 0 || device >= NOALLOC_MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(scratch_mu);
  if (!scratch_dev[device]) {
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device && (e = hipSetDevice(device)) != hipSuccess) return e;
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != device) {
      const hipError_t e2 = hipSetDevice(cur);
      if (e == hipSuccess) e = e2;
    }
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    scratch_dev[device] = (long long*)p;
  }
  *out = scratch_dev[device];
  return hipSuccess;
}

hipError_t launch_spread_noalloc(const Grid& g, const uint8_t* ncls, long long n, const double* pts,
                                 const double* F, const double* c, double* fib, long long* scr,
                                 hipStream_t s) {
  if (g.Np > NOALLOC_MAX_NODES) return hipErrorInvalidValue;
  long long* flag_words = scr + 3 * NOALLOC_MAX_NODES;
  // the last call's sums are normally flushed to zero already; clear anyway
  // (a fill kernel, not a memset, so that the sequence can be captured)
  k_zero_words<<<cdiv(3 * g.Np, 256), 256, 0, s>>>(scr, 3 * g.Np);
  k_zero_words<<<1, 64, 0, s>>>(flag_words, NOALLOC_FLAG_WORDS);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = launch_spread_api(g, ncls, n, pts, F, c, scr, (DevFlags*)flag_words, s);
  if (e != hipSuccess) return e;
  return launch_flush_fx(g, scr, fib, s);
}

// ====================================================== coupled adjoint (IB)
// The immersed-boundary part of the discrete adjoint of a coupled step, for
// soft bodies.  The step maps (g, P, Q, V) -> (g', P', Q', V'), with P the
// vertex positions x^n, Q = x^{n-1} and V the vertex velocities; going
// back, the transposes of the Verlet update (Eqs. verletPos, verletVel,
// verletPosC), the membrane forces (Eqs. strainFor, bendFor, volFor), the
// probe tractions (Eqs. hydroForP, hydroForNu), the MLS vertex velocities
// and the direct forcing with its spreading (Eqs. uLag, l2norm, intKernel,
// bodyforce) are applied, each with the derivative of its weights with
// respect to the moving points.  All in FP64.

// Forward-mode dual numbers (value and N partial derivatives), for the
// derivatives of the small per-point and per-element functions of the
// vertex positions.
template <int N>
struct Dual {
  double v;
  double d[N];
};

template <class T>
struct Scal;
template <>
struct Scal<double> {
  __device__ static double c(double v) { return v; }
};
template <int N>
struct Scal<Dual<N>> {
  __device__ static Dual<N> c(double v) {
    Dual<N> r;
    r.v = v;
#pragma unroll
    for (int i = 0; i < N; i++) r.d[i] = 0.0;
    return r;
  }
};

template <int N>
__device__ __forceinline__ Dual<N> dseed(double v, int k) {
  Dual<N> r = Scal<Dual<N>>::c(v);
  r.d[k] = 1.0;
  return r;
}
__device__ __forceinline__ double dval(double x) { return x; }
template <int N>
__device__ __forceinline__ double dval(const Dual<N>& x) {
  return x.v;
}

#define DUAL_BIN(OP, VEXPR, DEXPR)                                                           \
  template <int N>                                                                           \
  __device__ __forceinline__ Dual<N> operator OP(const Dual<N>& a, const Dual<N>& b) {       \
    Dual<N> r;                                                                               \
    r.v = VEXPR;                                                                             \
    _Pragma("unroll") for (int i = 0; i < N; i++) r.d[i] = DEXPR;                           \
    return r;                                                                                \
  }
DUAL_BIN(+, a.v + b.v, a.d[i] + b.d[i])
DUAL_BIN(-, a.v - b.v, a.d[i] - b.d[i])
DUAL_BIN(*, a.v * b.v, a.d[i] * b.v + a.v * b.d[i])
DUAL_BIN(/, a.v / b.v, (a.d[i] * b.v - a.v * b.d[i]) / (b.v * b.v))
#undef DUAL_BIN
template <int N>
__device__ __forceinline__ Dual<N> operator+(const Dual<N>& a, double b) {
  Dual<N> r = a;
  r.v += b;
  return r;
}
template <int N>
__device__ __forceinline__ Dual<N> operator+(double b, const Dual<N>& a) {
  return a + b;
}
template <int N>
__device__ __forceinline__ Dual<N> operator-(const Dual<N>& a, double b) {
  Dual<N> r = a;
  r.v -= b;
  return r;
}
template <int N>
__device__ __forceinline__ Dual<N> operator-(const Dual<N>& a) {
  Dual<N> r;
  r.v = -a.v;
#pragma unroll
  for (int i = 0; i < N; i++) r.d[i] = -a.d[i];
  return r;
}
template <int N>
__device__ __forceinline__ Dual<N> operator-(double b, const Dual<N>& a) {
  Dual<N> r = -a;
  r.v += b;
  return r;
}
template <int N>
__device__ __forceinline__ Dual<N> operator*(const Dual<N>& a, double b) {
  Dual<N> r;
  r.v = a.v * b;
#pragma unroll
  for (int i = 0; i < N; i++) r.d[i] = a.d[i] * b;
  return r;
}
template <int N>
__device__ __forceinline__ Dual<N> operator*(double b, const Dual<N>& a) {
  return a * b;
}
template <int N>
__device__ __forceinline__ Dual<N> operator/(const Dual<N>& a, double b) {
  return a * (1.0 / b);
}
template <int N>
__device__ __forceinline__ Dual<N>& operator+=(Dual<N>& a, const Dual<N>& b) {
  a = a + b;
  return a;
}
template <int N>
__device__ __forceinline__ Dual<N>& operator-=(Dual<N>& a, const Dual<N>& b) {
  a = a - b;
  return a;
}
// chain rule of a scalar function: value f, derivative df at a.v
template <int N>
__device__ __forceinline__ Dual<N> dchain(const Dual<N>& a, double f, double df) {
  Dual<N> r;
  r.v = f;
#pragma unroll
  for (int i = 0; i < N; i++) r.d[i] = df * a.d[i];
  return r;
}
__device__ __forceinline__ double dsqrt(double a) { return sqrt(a); }
__device__ __forceinline__ double dexp(double a) { return exp(a); }
__device__ __forceinline__ double dsin(double a) { return sin(a); }
__device__ __forceinline__ double dcos(double a) { return cos(a); }
__device__ __forceinline__ double datan2(double y, double x) { return atan2(y, x); }
template <int N>
__device__ __forceinline__ Dual<N> dsqrt(const Dual<N>& a) {
  const double r = sqrt(a.v);
  return dchain(a, r, 0.5 / r);
}
template <int N>
__device__ __forceinline__ Dual<N> dexp(const Dual<N>& a) {
  const double e = exp(a.v);
  return dchain(a, e, e);
}
template <int N>
__device__ __forceinline__ Dual<N> dsin(const Dual<N>& a) {
  return dchain(a, sin(a.v), cos(a.v));
}
template <int N>
__device__ __forceinline__ Dual<N> dcos(const Dual<N>& a) {
  return dchain(a, cos(a.v), -sin(a.v));
}
template <int N>
__device__ __forceinline__ Dual<N> datan2(const Dual<N>& y, const Dual<N>& x) {
  Dual<N> r;
  r.v = atan2(y.v, x.v);
  const double q = 1.0 / (x.v * x.v + y.v * y.v);
#pragma unroll
  for (int i = 0; i < N; i++) r.d[i] = (x.v * y.d[i] - y.v * x.d[i]) * q;
  return r;
}

template <class T>
__device__ __forceinline__ void cross_t(const T (&a)[3], const T (&b)[3], T (&c)[3]) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}
template <class T>
__device__ __forceinline__ T dot_t(const T (&a)[3], const T (&b)[3]) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

__device__ __forceinline__ double shfl_xor_t(double a, int m) { return __shfl_xor(a, m, 64); }
template <int N>
__device__ __forceinline__ Dual<N> shfl_xor_t(const Dual<N>& a, int m) {
  Dual<N> r;
  r.v = __shfl_xor(a.v, m, 64);
#pragma unroll
  for (int i = 0; i < N; i++) r.d[i] = __shfl_xor(a.d[i], m, 64);
  return r;
}

// Sum over the GS lanes of an aligned group inside one wave (xor tree:
// every lane ends with the same value, bit for bit).
template <int GS, class T>
__device__ __forceinline__ T group_sum(T v) {
#pragma unroll
  for (int m = GS / 2; m >= 1; m >>= 1) v = v + shfl_xor_t(v, m);
  return v;
}

// MLS at point p in any scalar type: the 27 supports of floor(p + 1/2)
// (solid and out-of-box nodes left out, as in the step), A = sum W P P^T
// with W = exp(-|d|^2 / (2.6^2 0.3^2)) and P = (1, d), d = x_k - p, then for
// each usable support fn(k, node, psi), psi = W A^{-1} P (psi[0] the
// interpolation weight phi_k, psi[1..3] the gradient weights of the linear
// fit).  A singular moment matrix (the step's rule) calls nothing and
// returns false.
// The work is split over a group of GS lanes (all of them call it, with the
// same p): lane l takes the supports l, l + GS, ...; the moment matrix is
// summed over the group, and fn runs for the lane's own supports.
template <int GS, class T, class Fn>
__device__ bool mls_each_g(const Grid& G, const uint8_t* ncls, const T (&p)[3], int lane, Fn&& fn) {
  const int bs[3] = {(int)floor(dval(p[0]) + 0.5), (int)floor(dval(p[1]) + 0.5), (int)floor(dval(p[2]) + 0.5)};
  T A[10];
#pragma unroll
  for (int k = 0; k < 10; k++) A[k] = Scal<T>::c(0.0);
  for (int k = lane; k < 27; k += GS) {
    long long node;
    const int c[3] = {bs[0] + k % 3 - 1, bs[1] + (k / 3) % 3 - 1, bs[2] + k / 9 - 1};
    if (!support_node(G, ncls, c[0], c[1], c[2], node)) continue;
    const T dx = (double)c[0] - p[0], dy = (double)c[1] - p[1], dz = (double)c[2] - p[2];
    const T W = dexp((dx * dx + dy * dy + dz * dz) * (-MLS_K));
    const T wx = W * dx, wy = W * dy, wz = W * dz;
    A[0] += W;
    A[1] += wx;
    A[2] += wy;
    A[3] += wz;
    A[4] += wx * dx;
    A[5] += wx * dy;
    A[6] += wx * dz;
    A[7] += wy * dy;
    A[8] += wy * dz;
    A[9] += wz * dz;
  }
  if (GS > 1) {
#pragma unroll
    for (int k = 0; k < 10; k++) A[k] = group_sum<GS>(A[k]);
  }
  const int ix[4][4] = {{0, 1, 2, 3}, {1, 4, 5, 6}, {2, 5, 7, 8}, {3, 6, 8, 9}};
  const double dmax = fmax(fmax(dval(A[0]), dval(A[4])), fmax(dval(A[7]), dval(A[9])));
  if (!(dmax > 0.0)) return false;
  // Cholesky factor, lower triangle packed row by row: L(i, j) = Lp[i (i + 1) / 2 + j]
  T Lp[10];
  for (int j = 0; j < 4; j++) {
    T d = A[ix[j][j]];
    for (int k = 0; k < j; k++) d -= Lp[j * (j + 1) / 2 + k] * Lp[j * (j + 1) / 2 + k];
    if (!(dval(d) > 1e-10 * dmax)) return false;
    Lp[j * (j + 1) / 2 + j] = dsqrt(d);
    for (int i = j + 1; i < 4; i++) {
      T v = A[ix[i][j]];
      for (int k = 0; k < j; k++) v -= Lp[i * (i + 1) / 2 + k] * Lp[j * (j + 1) / 2 + k];
      Lp[i * (i + 1) / 2 + j] = v / Lp[j * (j + 1) / 2 + j];
    }
  }
  for (int k = lane; k < 27; k += GS) {
    long long node;
    const int c[3] = {bs[0] + k % 3 - 1, bs[1] + (k / 3) % 3 - 1, bs[2] + k / 9 - 1};
    if (!support_node(G, ncls, c[0], c[1], c[2], node)) continue;
    const T P[4] = {Scal<T>::c(1.0), (double)c[0] - p[0], (double)c[1] - p[1], (double)c[2] - p[2]};
    const T W = dexp((P[1] * P[1] + P[2] * P[2] + P[3] * P[3]) * (-MLS_K));
    // psi = W A^{-1} P by the two triangular solves
    T y[4], psi[4];
    for (int i = 0; i < 4; i++) {
      T v = P[i];
      for (int j = 0; j < i; j++) v -= Lp[i * (i + 1) / 2 + j] * y[j];
      y[i] = v / Lp[i * (i + 1) / 2 + i];
    }
    for (int i = 3; i >= 0; i--) {
      T v = y[i];
      for (int j = i + 1; j < 4; j++) v -= Lp[j * (j + 1) / 2 + i] * psi[j];
      psi[i] = v / Lp[i * (i + 1) / 2 + i];
    }
    for (int i = 0; i < 4; i++) psi[i] = W * psi[i];
    fn(k, node, psi);
  }
  return true;
}

template <class T, class Fn>
__device__ bool mls_each(const Grid& G, const uint8_t* ncls, const T (&p)[3], Fn&& fn) {
  return mls_each_g<1>(G, ncls, p, 0, fn);
}

// Lanes per point in the IB transposes' MLS fits.
constexpr int ADJ_GS = 8;

// The bending force of a hinge (a, b, c, d) in any scalar type: the signed
// dihedral angle and F_r = -k_b sin(theta - theta0) dtheta/dx_r, with the
// closed-form angle gradient of the step.
template <class T>
__device__ void hinge_force_t(const T (&X)[4][3], double kb, double th0, T (&F)[4][3]) {
  T e[3], ca[3], da[3], ab[3], db[3], n1[3], n2[3];
  for (int k = 0; k < 3; k++) {
    e[k] = X[1][k] - X[0][k];
    ca[k] = X[2][k] - X[0][k];
    da[k] = X[3][k] - X[0][k];
    ab[k] = X[0][k] - X[1][k];
    db[k] = X[3][k] - X[1][k];
  }
  cross_t(e, ca, n1);
  cross_t(ab, db, n2);
  const T q1 = dot_t(n1, n1), q2 = dot_t(n2, n2), le2 = dot_t(e, e);
  const T le = dsqrt(le2), l1 = dsqrt(q1), l2 = dsqrt(q2);
  T m1[3], m2[3], t[3];
  for (int k = 0; k < 3; k++) {
    m1[k] = n1[k] / l1;
    m2[k] = n2[k] / l2;
  }
  cross_t(m1, m2, t);
  const T theta = datan2(dot_t(t, e) / le, dot_t(m1, m2));
  const T al_c = dot_t(ca, e) / le2, al_d = dot_t(da, e) / le2;
  const T amp = dsin(theta - th0) * (-kb);
  for (int k = 0; k < 3; k++) {
    const T gc = -(le * n1[k]) / q1;
    const T gd = -(le * n2[k]) / q2;
    F[0][k] = amp * (-((1.0 - al_c) * gc + (1.0 - al_d) * gd));
    F[1][k] = amp * (-(al_c * gc + al_d * gd));
    F[2][k] = amp * gc;
    F[3][k] = amp * gd;
  }
}

__device__ __forceinline__ void set_tile(uint8_t* tf, long long node) {
  if (!tf[node >> TILE_SHIFT]) tf[node >> TILE_SHIFT] = 1;
}

// The vertex update transposed.  With P' = P/2 + 3/2 u0 + 5/2 acc + Q/2,
// V' = -P/2 + 3/2 u0 + 3/2 acc + Q/2, Q' = P and acc = F / (2 m_v):
// dJ/du0 = 3/2 (aP + aV), dJ/dF = (5/2 aP + 3/2 aV) / (2 m_v),
// dJ/dQ = (aP + aV)/2, dJ/dP = aP/2 - aV/2 + aQ (more added by the later
// launches), dJ/dV = 0 (the forcing markers add theirs).
__global__ __launch_bounds__(256) void k_adjb_vertex(BodyArgs b, AdjIB ib) {
  const int idx = blockIdx.x * 256 + threadIdx.x;
  if (idx < b.nbody) ib.gsum[2 + idx] = 0.0;  // sum of A n . dJ/dFt per body (k_adjb_body adds it)
  if (idx >= b.nsoft_v) return;
  const int v = b.soft_vlist[idx];
  const double mv = b.b_param[8 * b.vert_body[v] + 3];
  for (int q = 0; q < 3; q++) {
    const int i = 3 * v + q;
    const double aX = ib.aP[i], aV = ib.aV[i], aQ = ib.aQ[i];
    ib.ub0[i] = 1.5 * (aX + aV);
    ib.Fb[i] = (2.5 * aX + 1.5 * aV) * 0.5 / mv;
    ib.Qn[i] = 0.5 * aX + 0.5 * aV;
    ib.LP[i] = 0.5 * aX - 0.5 * aV + aQ;
    ib.Vn[i] = 0.0;
  }
}

// Lift a function of a probe point (derivatives along its three
// coordinates) to the nine vertex coordinates the point depends on.
__device__ __forceinline__ Dual<9> lift9(const Dual<3>& f, const Dual<9> (&p)[3]) {
  Dual<9> r;
  r.v = f.v;
#pragma unroll
  for (int i = 0; i < 9; i++) r.d[i] = f.d[0] * p[0].d[i] + f.d[1] * p[1].d[i] + f.d[2] * p[2].d[i];
  return r;
}

// Elements, probes and vertex velocities transposed, one thread each:
// items [0, ne) edges, [ne, ne + nh) hinges, then faces, then soft vertices.
// Threads: one per edge and hinge, then (from the next multiple of 64) a
// group of ADJ_GS lanes per face and probe side, then per soft vertex; a
// group's MLS fits split the supports over its lanes.
__host__ __device__ __forceinline__ long long adjb_body_face0(const BodyArgs& b) {
  return ((long long)b.ne + b.nh + 63) / 64 * 64;
}

template <class S>
__global__ __launch_bounds__(128) void k_adjb_body(FluidArgs a, BodyArgs b, AdjIB ib) {
  const long long gt = blockIdx.x * 128LL + threadIdx.x;
  const Grid& G = a.g;
  const double* X = b.Xcur;
  const double ikap = 1.0 / ib.kappa;
  const long long g0 = adjb_body_face0(b);
  if (gt < g0) {
    // whole waves of elements (and padding lanes): dJ/dkappa summed over
    // the wave first, one atomic per wave
    const int it = gt < b.ne + b.nh ? (int)gt : -1;
    double fy = 0.0;
    if (it >= 0 && it < b.ne) {
      // stretching (Eq. strainFor): F_a = -k (l - l0) r / l, r = x_a - x_b; its
      // Jacobian K = -k [(1 - l0/l) 1 + l0 r r^T / l^3] is symmetric, and
      // dF_b = -dF_a
      const int e = it, va = b.edges[2 * e], vb = b.edges[2 * e + 1];
      double r[3], y[3];
      for (int k = 0; k < 3; k++) {
        r[k] = X[3 * va + k] - X[3 * vb + k];
        y[k] = ib.Fb[3 * va + k] - ib.Fb[3 * vb + k];
      }
      const double l = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
      const double kl = b.kl[e], l0 = b.l0[e];
      const double ry = r[0] * y[0] + r[1] * y[1] + r[2] * y[2];
      for (int k = 0; k < 3; k++) {
        const double g = -kl * ((1.0 - l0 / l) * y[k] + l0 * ry * r[k] / (l * l * l));
        atomicAdd(ib.LP + 3 * va + k, g);
        atomicAdd(ib.LP + 3 * vb + k, -g);
        fy += -kl * (l - l0) * r[k] / l * y[k];  // the force is linear in the modulus
      }
    } else if (it >= 0) {
      // bending: the force is minus the gradient of the hinge energy, so its
      // Jacobian is symmetric and the transposed product is the derivative
      // along the adjoint itself (one dual direction)
      const int h = it - b.ne;
      const int32_t* H = b.hinges + 4 * h;
      Dual<1> P[4][3], F[4][3];
      for (int r = 0; r < 4; r++)
        for (int k = 0; k < 3; k++) {
          P[r][k].v = X[3 * H[r] + k];
          P[r][k].d[0] = ib.Fb[3 * H[r] + k];
        }
      hinge_force_t(P, b.kb[h], b.theta0[h], F);
      for (int r = 0; r < 4; r++)
        for (int k = 0; k < 3; k++) {
          atomicAdd(ib.LP + 3 * H[r] + k, F[r][k].d[0]);
          fy += F[r][k].v * ib.Fb[3 * H[r] + k];
        }
    }
    fy = group_sum<64>(fy);
    if ((threadIdx.x & 63) == 0 && fy != 0.0) atomicAdd(ib.gsum + 1, fy * ikap);
    return;
  }
  const int lane = (int)((gt - g0) % ADJ_GS);
  const long long grp = (gt - g0) / ADJ_GS;
  const long long nfg = (2LL * b.nf * ADJ_GS + 63) / 64 * 64 / ADJ_GS;  // face groups, whole waves
  if (grp < nfg) {
    // face force Ft = A [-(r+ - r-)/3 n + nu (r+ (G+ + G+^T) - r- (G- + G-^T)) n]
    // + k_v (1 - V/V0) A n (probes at c +- 1.2 n: fitted density r and
    // velocity gradient G), a third at each vertex: dJ/dFt = the mean of
    // the vertices' dJ/dF.  Two groups per face: the outer probe's terms
    // with the volume term, and the inner probe's.
    const bool real = grp < 2LL * b.nf;  // groups past the faces pad the last wave
    const int f = real ? (int)(grp >> 1) : 0, side = (int)(grp & 1);
    const int body = b.face_body[f];
    const int vv[3] = {b.faces[3 * f], b.faces[3 * f + 1], b.faces[3 * f + 2]};
    double ab[3];
    for (int k = 0; k < 3; k++) ab[k] = (ib.Fb[3 * vv[0] + k] + ib.Fb[3 * vv[1] + k] + ib.Fb[3 * vv[2] + k]) / 3.0;
    // unit normal n and area A with their derivatives in the nine vertex
    // coordinates (j = 3 r + k), by dual numbers in this scope only
    double nv[3], Av, dn[3][9], dA[9], cen[3];
    {
      Dual<9> P[3][3];
      for (int r = 0; r < 3; r++)
        for (int k = 0; k < 3; k++) P[r][k] = dseed<9>(X[3 * vv[r] + k], 3 * r + k);
      Dual<9> u[3], w[3], N[3];
      for (int k = 0; k < 3; k++) {
        u[k] = P[1][k] - P[0][k];
        w[k] = P[2][k] - P[0][k];
      }
      cross_t(u, w, N);
      const Dual<9> ln = dsqrt(dot_t(N, N));
      for (int k = 0; k < 3; k++) {
        const Dual<9> nk = N[k] / ln;
        nv[k] = nk.v;
        for (int j = 0; j < 9; j++) dn[k][j] = nk.d[j];
        cen[k] = (P[0][k].v + P[1][k].v + P[2][k].v) / 3.0;
      }
      Av = 0.5 * ln.v;
      for (int j = 0; j < 9; j++) dA[j] = 0.5 * ln.d[j];
    }
    const double nu = b.nu;
    const double V0 = b.b_param[8 * body], kv = b.b_param[8 * body + 2];
    const double cv = kv * (1.0 - b.b_diag[16 * body] / V0);
    const double an = ab[0] * nv[0] + ab[1] * nv[1] + ab[2] * nv[2];
    double dan[9];
    for (int j = 0; j < 9; j++) dan[j] = ab[0] * dn[0][j] + ab[1] * dn[1][j] + ab[2] * dn[2][j];
    // ds[j]: derivative of this group's part of ab . Ft in vertex coordinate j
    double ds[9];
    for (int j = 0; j < 9; j++) ds[j] = side == 0 ? cv * (dA[j] * an + Av * dan[j]) : 0.0;  // the volume force
    double visc = 0.0;  // d s / d nu
    {
      const double sg = side == 0 ? 1.2 : -1.2, sgn = side == 0 ? 1.0 : -1.0;
      double pp[3];
      for (int k = 0; k < 3; k++) pp[k] = cen[k] + nv[k] * sg;
      // the fits at the probe, with their derivatives in its coordinates
      const Dual<3> q[3] = {dseed<3>(pp[0], 0), dseed<3>(pp[1], 1), dseed<3>(pp[2], 2)};
      Dual<3> r3 = Scal<Dual<3>>::c(0.0), G3[3][3];
      for (int i = 0; i < 3; i++)
        for (int c = 0; c < 3; c++) G3[i][c] = Scal<Dual<3>>::c(0.0);
      mls_each_g<ADJ_GS>(G, a.ncls, q, lane, [&](int, long long node, const Dual<3>(&psi)[4]) {
        double dr, uu[3];
        load_mac<S>(a, node, dr, uu[0], uu[1], uu[2]);
        r3 += psi[0] * dr;
        for (int i = 0; i < 3; i++)
          for (int c = 0; c < 3; c++) G3[i][c] += psi[1 + c] * uu[i];
      });
      r3 = group_sum<ADJ_GS>(r3) + 1.0;  // the weights add up to 1: rho = 1 + the fit of rho - 1
      for (int i = 0; i < 3; i++)
        for (int c = 0; c < 3; c++) G3[i][c] = group_sum<ADJ_GS>(G3[i][c]);
      // s = A sgn r Q with Q = -an/3 + nu sv, sv = sum_ic ab_i (G_ic + G_ci) n_c;
      // the probe moves with the face: dp_m/dx_j = [m == j % 3]/3 + sg dn_m/dx_j
      double sv = 0.0, h[3] = {0.0, 0.0, 0.0}, qc[3] = {0.0, 0.0, 0.0};
      for (int i = 0; i < 3; i++)
        for (int c = 0; c < 3; c++) {
          const double gs = G3[i][c].v + G3[c][i].v;
          sv += ab[i] * gs * nv[c];
          qc[c] += ab[i] * gs;
          for (int m = 0; m < 3; m++) h[m] += ab[i] * (G3[i][c].d[m] + G3[c][i].d[m]) * nv[c];
        }
      const double rv = r3.v, Q = -an / 3.0 + nu * sv;
      for (int j = 0; j < 9; j++) {
        double drj = 0.0, dsvj = 0.0;
        for (int m = 0; m < 3; m++) {
          const double dp = (m == j % 3 ? 1.0 / 3.0 : 0.0) + sg * dn[m][j];
          drj += r3.d[m] * dp;
          dsvj += h[m] * dp + qc[m] * dn[m][j];
        }
        const double dQ = -dan[j] / 3.0 + nu * dsvj;
        ds[j] += sgn * (dA[j] * rv * Q + Av * (drj * Q + rv * dQ));
      }
      visc += Av * sgn * rv * sv;
      // field adjoints at this probe's supports
      const double rbar = Av * sgn * Q;
      double Gbar[3][3];
      for (int i = 0; i < 3; i++)
        for (int c = 0; c < 3; c++) Gbar[i][c] = Av * sgn * nu * rv * (ab[i] * nv[c] + ab[c] * nv[i]);
      if (real)  // (uniform over the group)
        mls_each_g<ADJ_GS>(G, a.ncls, pp, lane, [&](int, long long node, const double(&psi)[4]) {
          atomicAdd(ib.ext + node, rbar * psi[0]);
          for (int i = 0; i < 3; i++)
            atomicAdd(ib.ext + (long long)(1 + i) * G.Np + node,
                      Gbar[i][0] * psi[1] + Gbar[i][1] * psi[2] + Gbar[i][2] * psi[3]);
          set_tile(ib.etf, node);
        });
    }
    const double A_v = Av;
    // the scalar gradients summed over the wave first (one group's lane 0
    // per face side contributes), then one atomic per wave
    const bool lead = real && lane == 0;
    const double gv = group_sum<64>(lead ? visc / 3.0 : 0.0);  // nu = (tau - 1/2) / 3
    const double gk = group_sum<64>(lead && side == 0 && b.b_param[8 * body + 6] != 0.0 ? cv * A_v * an * ikap : 0.0);
    if ((threadIdx.x & 63) == 0) {
      if (gv != 0.0) atomicAdd(ib.gsum, gv);
      if (gk != 0.0) atomicAdd(ib.gsum + 1, gk);
    }
    // sum of A n . dJ/dFt per body: one atomic per wave when its faces
    // belong to one body
    {
      const int bsel = lead && side == 0 ? body : -1;
      const double gb = bsel >= 0 ? A_v * an : 0.0;
      const unsigned long long bm = __ballot(bsel >= 0);
      if (bm) {
        const int first = __shfl(bsel, __ffsll((unsigned long long)bm) - 1, 64);
        if (__ballot(bsel >= 0 && bsel != first) == 0ull) {
          const double t = group_sum<64>(gb);
          if ((threadIdx.x & 63) == 0) atomicAdd(ib.gsum + 2 + first, t);
        } else if (bsel >= 0) {
          atomicAdd(ib.gsum + 2 + bsel, gb);
        }
      }
    }
    if (!lead) return;
    for (int r = 0; r < 3; r++)
      for (int k = 0; k < 3; k++) atomicAdd(ib.LP + 3 * vv[r] + k, ds[3 * r + k]);
    return;
  }
  const long long idx = grp - nfg;
  if (idx >= b.nsoft_v) return;
  // MLS velocity at the vertex: u0 = sum phi_k u_k
  const int v = b.soft_vlist[idx];
  const double ub[3] = {ib.ub0[3 * v], ib.ub0[3 * v + 1], ib.ub0[3 * v + 2]};
  const Dual<3> p[3] = {dseed<3>(X[3 * v], 0), dseed<3>(X[3 * v + 1], 1), dseed<3>(X[3 * v + 2], 2)};
  Dual<3> s = Scal<Dual<3>>::c(0.0);
  mls_each_g<ADJ_GS>(G, a.ncls, p, lane, [&](int, long long node, const Dual<3>(&psi)[4]) {
    double dr, uu[3];
    load_mac<S>(a, node, dr, uu[0], uu[1], uu[2]);
    s += psi[0] * (uu[0] * ub[0] + uu[1] * ub[1] + uu[2] * ub[2]);
    for (int i = 0; i < 3; i++) atomicAdd(ib.ext + (long long)(1 + i) * G.Np + node, psi[0].v * ub[i]);
    set_tile(ib.etf, node);
  });
  s = group_sum<ADJ_GS>(s);
  if (lane == 0)
    for (int k = 0; k < 3; k++) atomicAdd(ib.LP + 3 * v + k, s.d[k]);
}

// Flags the tiles of every forcing marker's support nodes (the force adjoint
// is needed there whatever the step's force was).
__global__ __launch_bounds__(256) void k_adjb_support(Grid G, const uint8_t* ncls, BodyArgs b, uint8_t* etf) {
  const int m = blockIdx.x * 256 + threadIdx.x;
  if (m >= b.nf) return;
  double cen[3], n[3], area;
  face_geom(b.Xcur, b.faces, m, cen, n, area);
  const int bs[3] = {(int)floor(cen[0] + 0.5), (int)floor(cen[1] + 0.5), (int)floor(cen[2] + 0.5)};
  for (int k = 0; k < 27; k++) {
    long long node;
    if (support_node(G, ncls, bs[0] + k % 3 - 1, bs[1] + (k / 3) % 3 - 1, bs[2] + k / 9 - 1, node))
      set_tile(etf, node);
  }
}

// The volume force through V: Ft_f contains k_v (1 - V/V0) A_f n_f, and
// dV/dx_v is a third of the sum of A n over the faces at v.
__global__ __launch_bounds__(256) void k_adjb_volume(BodyArgs b, AdjIB ib) {
  const int f = blockIdx.x * 256 + threadIdx.x;
  if (f >= b.nf) return;
  const int body = b.face_body[f];
  const double V0 = b.b_param[8 * body], kv = b.b_param[8 * body + 2];
  const double c = -kv / V0 * ib.gsum[2 + body] / 3.0;
  double cen[3], n[3], area;
  face_geom(b.Xcur, b.faces, f, cen, n, area);
  for (int r = 0; r < 3; r++)
    for (int k = 0; k < 3; k++) atomicAdd(ib.LP + 3 * b.faces[3 * f + r] + k, c * area * n[k]);
}

// The forcing markers transposed (one thread per face): U = sum phi u*,
// F_l = U_b - U, f_ib += A phi F_l.  dJ/dF_l = A sum phi dJ/dF_k; dJ/dU_b =
// dJ/dF_l (a third to each vertex velocity); dJ/du*_k -= phi_k dJ/dF_l; and
// the positions through the centroid (phi) and the area.
template <class S>
__global__ __launch_bounds__(128) void k_adjb_markers(FluidArgs a, BodyArgs b, AdjIB ib) {
  // a group of ADJ_GS lanes per face, the supports split over it
  const int gt = blockIdx.x * 128 + threadIdx.x;
  const int m = gt / ADJ_GS, lane = gt % ADJ_GS;
  if (m >= b.nf) return;  // whole groups
  const Grid& G = a.g;
  const int vv[3] = {b.faces[3 * m], b.faces[3 * m + 1], b.faces[3 * m + 2]};
  double cen[3], n[3], area, Ub[3];
  face_geom(b.Xcur, b.faces, m, cen, n, area);
  for (int k = 0; k < 3; k++) Ub[k] = (b.Vel[3 * vv[0] + k] + b.Vel[3 * vv[1] + k] + b.Vel[3 * vv[2] + k]) / 3.0;
  double U[3] = {0.0, 0.0, 0.0}, Fs[3] = {0.0, 0.0, 0.0};
  mls_each_g<ADJ_GS>(G, a.ncls, cen, lane, [&](int, long long node, const double(&psi)[4]) {
    const Moments mo = streamed_moments<S>(a, node);
    const double rho = 1.0 + mo.drho;
    for (int k = 0; k < 3; k++) {
      U[k] += psi[0] * (mo.m[k] / rho);
      Fs[k] += psi[0] * ib.fbar[(long long)k * G.Np + node];
    }
  });
  double Fl[3], Fbl[3];
  for (int k = 0; k < 3; k++) {
    U[k] = group_sum<ADJ_GS>(U[k]);
    Fs[k] = group_sum<ADJ_GS>(Fs[k]);
    Fl[k] = Ub[k] - U[k];
    Fbl[k] = area * Fs[k];
  }
  if (lane == 0)
    for (int r = 0; r < 3; r++)
      for (int k = 0; k < 3; k++) atomicAdd(ib.Vn + 3 * vv[r] + k, Fbl[k] / 3.0);
  const Dual<3> q[3] = {dseed<3>(cen[0], 0), dseed<3>(cen[1], 1), dseed<3>(cen[2], 2)};
  Dual<3> s = Scal<Dual<3>>::c(0.0);
  double Abar = 0.0;
  mls_each_g<ADJ_GS>(G, a.ncls, q, lane, [&](int, long long node, const Dual<3>(&psi)[4]) {
    const Moments mo = streamed_moments<S>(a, node);
    const double rho = 1.0 + mo.drho;
    double fF = 0.0, uF = 0.0;
    for (int k = 0; k < 3; k++) {
      fF += Fl[k] * ib.fbar[(long long)k * G.Np + node];
      uF += (mo.m[k] / rho) * Fbl[k];
    }
    s += psi[0] * (area * fF - uF);
    Abar += psi[0].v * fF;
    for (int k = 0; k < 3; k++) atomicAdd(ib.ext + (long long)(4 + k) * G.Np + node, -psi[0].v * Fbl[k]);
    set_tile(ib.etf, node);
  });
  s = group_sum<ADJ_GS>(s);
  Abar = group_sum<ADJ_GS>(Abar);
  if (lane != 0) return;
  // d area / d vertex: (1/2) n x (opposite edge), counter-clockwise
  for (int r = 0; r < 3; r++) {
    const double* xb = b.Xcur + 3 * vv[(r + 1) % 3];
    const double* xc = b.Xcur + 3 * vv[(r + 2) % 3];
    const double e[3] = {xc[0] - xb[0], xc[1] - xb[1], xc[2] - xb[2]};
    const double dA[3] = {0.5 * (n[1] * e[2] - n[2] * e[1]), 0.5 * (n[2] * e[0] - n[0] * e[2]),
                          0.5 * (n[0] * e[1] - n[1] * e[0])};
    for (int k = 0; k < 3; k++) atomicAdd(ib.LP + 3 * vv[r] + k, s.d[k] / 3.0 + Abar * dA[k]);
  }
}

// Eigen-decomposition of a symmetric 3x3 matrix by cyclic Jacobi rotations:
// eigenvalues in d, eigenvectors in the columns of V.
__device__ void jacobi3(double (&M)[3][3], double (&d)[3], double (&V)[3][3]) {
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) V[i][j] = i == j ? 1.0 : 0.0;
  for (int sweep = 0; sweep < 50; sweep++) {
    const double off = M[0][1] * M[0][1] + M[0][2] * M[0][2] + M[1][2] * M[1][2];
    const double dg = M[0][0] * M[0][0] + M[1][1] * M[1][1] + M[2][2] * M[2][2];
    if (off <= 1e-36 * dg) break;
    for (int p = 0; p < 2; p++)
      for (int q = p + 1; q < 3; q++) {
        if (M[p][q] == 0.0) continue;
        const double th = (M[q][q] - M[p][p]) / (2.0 * M[p][q]);
        const double t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
        const double c = 1.0 / sqrt(t * t + 1.0), sn = t * c;
        for (int k = 0; k < 3; k++) {  // M <- M J
          const double mkp = M[k][p], mkq = M[k][q];
          M[k][p] = c * mkp - sn * mkq;
          M[k][q] = sn * mkp + c * mkq;
        }
        for (int k = 0; k < 3; k++) {  // M <- J^T M
          const double mpk = M[p][k], mqk = M[q][k];
          M[p][k] = c * mpk - sn * mqk;
          M[q][k] = sn * mpk + c * mqk;
        }
        for (int k = 0; k < 3; k++) {
          const double vkp = V[k][p], vkq = V[k][q];
          V[k][p] = c * vkp - sn * vkq;
          V[k][q] = sn * vkp + c * vkq;
        }
      }
  }
  for (int i = 0; i < 3; i++) d[i] = M[i][i];
}

// Taylor deformation of a body, D = (sqrt(l1) - sqrt(l3)) / (sqrt(l1) +
// sqrt(l3)) from the largest and smallest eigenvalues of the vertex
// second-moment tensor M = sum (x - xbar)(x - xbar)^T / n; one block.  Adds
// D to *jsum, or theta dD/dx = theta (2/n) G (x - xbar) to aP, with G =
// dD/dl1 v1 v1^T + dD/dl3 v3 v3^T.
__global__ __launch_bounds__(256) void k_taylor(BodyArgs b, const double* X, int body, double theta, double* aP,
                                                double* jsum) {
  __shared__ double sh[8];
  __shared__ double s_G[9], s_m[3];
  const int v0 = b.b_vert0[body], nvb = b.b_nv[body];
  double m[3] = {0.0, 0.0, 0.0};
  for (int v = v0 + threadIdx.x; v < v0 + nvb; v += 256)
    for (int k = 0; k < 3; k++) m[k] += X[3 * v + k];
  for (int k = 0; k < 3; k++) m[k] = block_sum(m[k], sh) / nvb;
  double M6[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  for (int v = v0 + threadIdx.x; v < v0 + nvb; v += 256) {
    const double d[3] = {X[3 * v] - m[0], X[3 * v + 1] - m[1], X[3 * v + 2] - m[2]};
    M6[0] += d[0] * d[0];
    M6[1] += d[0] * d[1];
    M6[2] += d[0] * d[2];
    M6[3] += d[1] * d[1];
    M6[4] += d[1] * d[2];
    M6[5] += d[2] * d[2];
  }
  for (int k = 0; k < 6; k++) M6[k] = block_sum(M6[k], sh) / nvb;
  if (threadIdx.x == 0) {
    double M[3][3] = {{M6[0], M6[1], M6[2]}, {M6[1], M6[3], M6[4]}, {M6[2], M6[4], M6[5]}};
    double d[3], V[3][3];
    jacobi3(M, d, V);
    int i1 = 0, i3 = 0;
    for (int i = 1; i < 3; i++) {
      if (d[i] > d[i1]) i1 = i;
      if (d[i] < d[i3]) i3 = i;
    }
    const double a = sqrt(d[i1]), c = sqrt(d[i3]), s2 = (a + c) * (a + c);
    if (jsum) *jsum += (a - c) / (a + c);
    const double g1 = c / (a * s2), g3 = -a / (c * s2);  // dD/dl1, dD/dl3
    for (int i = 0; i < 3; i++)
      for (int j = 0; j < 3; j++) s_G[3 * i + j] = g1 * V[i][i1] * V[j][i1] + g3 * V[i][i3] * V[j][i3];
    for (int k = 0; k < 3; k++) s_m[k] = m[k];
  }
  __syncthreads();
  if (!aP) return;
  for (int v = v0 + threadIdx.x; v < v0 + nvb; v += 256) {
    const double d[3] = {X[3 * v] - s_m[0], X[3 * v + 1] - s_m[1], X[3 * v + 2] - s_m[2]};
    for (int i = 0; i < 3; i++)
      aP[3 * v + i] += theta * 2.0 / nvb * (s_G[3 * i] * d[0] + s_G[3 * i + 1] * d[1] + s_G[3 * i + 2] * d[2]);
  }
}

// Zero the extra adjoint sources and the fixed-point force in flagged
// tiles (data first, then, in a second launch, the flags).
__global__ __launch_bounds__(256) void k_adjb_clear_data(Grid G, double* ext, const uint8_t* etf, long long* fx,
                                                         const uint8_t* ftf) {
  const long long n = blockIdx.x * 256LL + threadIdx.x;
  if (n >= G.Np) return;
  if (etf[n >> TILE_SHIFT])
    for (int k = 0; k < 7; k++) ext[(long long)k * G.Np + n] = 0.0;
  if (ftf[n >> TILE_SHIFT])
    for (int k = 0; k < 3; k++) fx[(long long)k * G.Np + n] = 0;
}
__global__ __launch_bounds__(256) void k_adjb_clear_flags(long long ntiles, uint8_t* etf, uint8_t* ftf) {
  const long long t = blockIdx.x * 256LL + threadIdx.x;
  if (t >= ntiles) return;
  etf[t] = 0;
  ftf[t] = 0;
}

// <w, g> at the non-solid nodes (those with amask bit 31 when use_mask),
// each block adding its sum to part[block] (grid-stride, fixed order).
template <class S>
__global__ __launch_bounds__(256) void k_adj_wdot(FluidArgs a, const S* g, const double* w, const uint32_t* amask,
                                                  int use_mask, double* part) {
  __shared__ double sh[8];
  const Grid& G = a.g;
  double acc = 0.0;
  const int count = a.nbulk_nodes + a.nrec;
  for (int t = blockIdx.x * 256 + threadIdx.x; t < count; t += gridDim.x * 256) {
    if (use_mask && !(amask[t] >> 31)) continue;
    const long long n = t < a.nbulk_nodes ? (long long)a.bulk_list[t] : (long long)a.rec_node[t - a.nbulk_nodes];
    for (int j = 0; j < 19; j++)
      acc += w[(long long)j * G.plane + n] * (double)to_c(g[(long long)j * G.plane + n]);
  }
  acc = block_sum(acc, sh);
  if (threadIdx.x == 0) part[blockIdx.x] += acc;
}

__global__ void k_adj_sum(const double* part, int n, double* out) {
  if (threadIdx.x != 0) return;
  double t = 0.0;
  for (int k = 0; k < n; k++) t += part[k];
  *out = t;
}

hipError_t launch_adjb_vertex(const BodyArgs& b, const AdjIB& ib, hipStream_t s) {
  const int n = std::max(b.nsoft_v, b.nbody);
  if (n > 0) k_adjb_vertex<<<cdiv(n, 256), 256, 0, s>>>(b, ib);
  return hipGetLastError();
}

// The body state of a coupled step's output slot before the step: x^n
// where x^{n+1} will be written, x^{n-1} = the input's x^n, and the input's
// velocities (three arrays of nv3 doubles each).
__global__ __launch_bounds__(256) void k_body_slots(const double* from, double* to, long long nv3) {
  const long long i = blockIdx.x * 256LL + threadIdx.x;
  if (i >= nv3) return;
  to[i] = from[nv3 + i];
  to[nv3 + i] = from[i];
  to[2 * nv3 + i] = from[2 * nv3 + i];
}

hipError_t launch_body_slots(const double* from, double* to, long long nv3, hipStream_t s) {
  if (nv3 > 0) k_body_slots<<<cdiv(nv3, 256), 256, 0, s>>>(from, to, nv3);
  return hipGetLastError();
}

hipError_t launch_adjb_body(int prec, const FluidArgs& a, const BodyArgs& b, const AdjIB& ib, hipStream_t s) {
  const long long threads = adjb_body_face0(b) + (2LL * b.nf * ADJ_GS + 63) / 64 * 64 + (long long)b.nsoft_v * ADJ_GS;
  if ((long long)b.ne + b.nh + b.nf + b.nsoft_v == 0) return hipSuccess;
  const unsigned grid = cdiv(threads, 128);
  switch (prec) {
    case 0: k_adjb_body<double><<<grid, 128, 0, s>>>(a, b, ib); break;
    case 1: k_adjb_body<float><<<grid, 128, 0, s>>>(a, b, ib); break;
    default: k_adjb_body<_Float16><<<grid, 128, 0, s>>>(a, b, ib); break;
  }
  return hipGetLastError();
}

hipError_t launch_adjb_volume(const BodyArgs& b, const AdjIB& ib, hipStream_t s) {
  if (b.nf > 0) k_adjb_volume<<<cdiv(b.nf, 256), 256, 0, s>>>(b, ib);
  return hipGetLastError();
}

hipError_t launch_adjb_support(const Grid& g, const uint8_t* ncls, const BodyArgs& b, uint8_t* etf, hipStream_t s) {
  if (b.nf > 0) k_adjb_support<<<cdiv(b.nf, 256), 256, 0, s>>>(g, ncls, b, etf);
  return hipGetLastError();
}

hipError_t launch_adjb_markers(int prec, const FluidArgs& a, const BodyArgs& b, const AdjIB& ib, hipStream_t s) {
  if (b.nf == 0) return hipSuccess;
  const unsigned grid = cdiv((long long)b.nf * ADJ_GS, 128);
  switch (prec) {
    case 0: k_adjb_markers<double><<<grid, 128, 0, s>>>(a, b, ib); break;
    case 1: k_adjb_markers<float><<<grid, 128, 0, s>>>(a, b, ib); break;
    default: k_adjb_markers<_Float16><<<grid, 128, 0, s>>>(a, b, ib); break;
  }
  return hipGetLastError();
}

hipError_t launch_taylor(const BodyArgs& b, const double* X, int body, double theta, double* aP, double* jsum,
                         hipStream_t s) {
  k_taylor<<<1, 256, 0, s>>>(b, X, body, theta, aP, jsum);
  return hipGetLastError();
}

hipError_t launch_adjb_clear(const Grid& g, double* ext, uint8_t* etf, long long* fx, uint8_t* ftf, hipStream_t s) {
  const long long ntiles = (g.Np >> TILE_SHIFT) + 1;
  k_adjb_clear_data<<<cdiv(g.Np, 256), 256, 0, s>>>(g, ext, etf, fx, ftf);
  k_adjb_clear_flags<<<cdiv(ntiles, 256), 256, 0, s>>>(ntiles, etf, ftf);
  return hipGetLastError();
}

hipError_t launch_adj_wdot(int prec, const FluidArgs& a, const void* g, const double* w, const uint32_t* amask,
                           int use_mask, double* part, hipStream_t s) {
  const int count = a.nbulk_nodes + a.nrec;
  if (count == 0) return hipSuccess;
  const unsigned grid = std::min<unsigned>(cdiv(count, 256), ADJ_BLOCKS);
  switch (prec) {
    case 0: k_adj_wdot<double><<<grid, 256, 0, s>>>(a, (const double*)g, w, amask, use_mask, part); break;
    case 1: k_adj_wdot<float><<<grid, 256, 0, s>>>(a, (const float*)g, w, amask, use_mask, part); break;
    default: k_adj_wdot<_Float16><<<grid, 256, 0, s>>>(a, (const _Float16*)g, w, amask, use_mask, part); break;
  }
  return hipGetLastError();
}

hipError_t launch_adj_sum(const double* part, int n, double* out, hipStream_t s) {
  k_adj_sum<<<1, 64, 0, s>>>(part, n, out);
  return hipGetLastError();
}

}  // namespace lbm
