// Internal declarations shared by the host side (lbm_abi.cpp) and the
// kernels (lbm_kernels.hip) of the gfx950 library.  Not part of the C ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbm {

// Node classes used by the fused stream-collide kernel.
enum : uint8_t { CLS_SOLID = 0, CLS_BULK = 1, CLS_GENERAL = 2 };

// Status bits raised on the device.
enum : uint32_t { ST_UNSTABLE = 1u, ST_DAMAGED = 2u };

// Fixed-point scale of the spread force: 2^57, so one unit is 2^-57 (the
// rounding of a contribution at most 2^-58 ~ 3.5e-18) and a node holds
// +-64.  A single contribution beyond +-1 stops the run as unstable, which
// keeps node totals in range up to 64 such contributions per node.
constexpr double FX_SCALE = 144115188075855872.0;
constexpr double FX_INV = 1.0 / 144115188075855872.0;

// Force-flag granularity: 64 consecutive nodes (an eighth of a 512-node
// row), so that the tiles touched by a capsule's spread cover little more
// than its support region.
constexpr int TILE_SHIFT = 6;

// Forcing markers per block of the first IB launch (a quad of lanes each),
// and the most support nodes a block's bounding box may hold in LDS (larger
// boxes take the direct path).  64 neighbouring faces of a capsule of
// radius 19 (2562 vertices) need up to ~1430 box nodes; one block in a
// thousand of the 16-capsule workload takes the direct path.
constexpr int MARKERS_PER_BLOCK = 64;
constexpr int BOX_CELLS = 1400;  // 73 KB of LDS: two blocks fit a CU
constexpr int BIN_LDS_KEYS = 8192;  // bodies up to this many faces are binned in LDS (64 KB)
constexpr int BIN_THREADS = 1024;   // threads of the binning block
constexpr int CHUNK_CAP = 3;        // marker chunks per 64 faces of a body

// Work per wave of the probe / vertex-velocity launch: 8 faces (4 lanes per
// MLS point, outer and inner probe) or 16 vertices.
constexpr int MLS_FACES_PER_WAVE = 8, MLS_VERTS_PER_WAVE = 16;

// Vertex incidence table widths (largest vertex valence accepted: 10).
constexpr int VT_E = 10, VT_H = 20, VT_F = 10, VT_SLOTS = VT_E + VT_H + VT_F;

struct DevFlags {
  uint32_t stop;      // sticky stop bits (checked at every kernel entry)
  uint32_t pending;   // bits raised during the current step
  uint32_t overflow;  // a spread contribution exceeded +-1 (also raises ST_UNSTABLE)
  uint32_t pad;
  long long steps_done;
  int mls_singular;
  int pad2;
};

struct Grid {
  int nx, ny, nz;  // logical sizes
  int px;          // padded row pitch (multiple of 8)
  int per[3];
  long long Np;    // px*ny*nz
  long long plane; // distance between population planes (elements)
  long long guard; // elements allocated before plane 0 and after plane 18
  // division of a padded index (< 2^31) by px and by ny as a multiply and a
  // shift: q = (u m) >> s with m = ceil(2^s / d), s = 31 + ceil(log2 d)
  // (exact for every u < 2^31, since m d - 2^s < d <= 2^(s - 31))
  unsigned int mpx, mny;
  int spx, sny;
};

// Everything the fluid and IB kernels need (passed by value).
struct FluidArgs {
  Grid g;
  const void* A;  // populations read this step
  void* B;        // populations written this step
  const uint8_t* ncls;
  const int32_t* rec_of;     // [Np] -> record or -1
  int nrec;
  const int32_t* rec_node;   // padded index
  const uint32_t* rec_mask;  // bit j: pulled direction j comes from a wall link
  const int32_t* rec_link0;
  const uint8_t* rec_face;   // 0xff: none; else face | (kind << 4) (kind 1 = density)
  const double* rec_bc;      // [4][nrec]: ux, uy, uz, rho
  const void* lk_c;          // [3][nlinks] interpolated bounce-back coefficients (compute type)
  const uint32_t* rec_mb;    // [nrec] bit j: the link of direction j has q >= 1/2
  int nlinks;
  const int32_t* tile_list;  // blocks of the bulk part (tile form)
  int nbulk_blocks;
  const int32_t* bulk_list;  // list form (bulk_v 0): the bulk nodes in order, else null
  int nbulk_nodes;
  double omega;              // 1/tau
  double gx, gy, gz;         // uniform body force
  const long long* fx;       // fixed-point IB force [3][Np] of this step (may be null)
  const uint8_t* tflag;      // tile flags of this step (may be null)
  void* mac;                 // [Np][4] rho - 1, u of this step in the compute type (null: not kept)
  DevFlags* flags;
  unsigned int* counter;     // block counter used when this launch closes the step
  int close_step;            // 1: no bodies, this launch is the whole step
  int rec_block;             // threads per block of the record kernel
  int bulk_v;                // nodes per thread of the bulk kernel (0: list form, one)
  int bulk_block;            // threads per block of the bulk kernel
};

// Bodies (all concatenated).
struct BodyArgs {
  int nbody, nv, nf, ne, nh;
  int nsoft_v;                 // number of soft vertices
  const int32_t* soft_vlist;   // [nsoft_v] global vertex ids of soft bodies
  const double* Xcur;          // [nv][3] x^n
  double* Xnext;               // [nv][3] x^{n+1} (holds x^{n-1} on entry)
  double* Vel;                 // [nv][3]
  const int32_t* faces;        // [nf][3] global vertex ids
  const int32_t* face_body;    // [nf]
  const int32_t* vert_body;    // [nv]
  const int32_t* edges;        // [ne][2]
  const double* l0;            // [ne]
  const double* kl;            // [ne]
  const int32_t* hinges;       // [nh][4]
  const double* theta0;        // [nh]
  const double* kb;            // [nh]
  // Forces on vertices by incidence slot, [VT_SLOTS][3][nv]: VT_E edge slots,
  // VT_H hinge slots, VT_F face slots per vertex (unused slots hold 0); the
  // element of slot-major index sl_*[...] writes there.
  double* f_slot;
  const int32_t* sl_edge;      // [ne][2] slot of the edge's force at its two ends
  const int32_t* sl_hinge;     // [nh][4] slot of the hinge's force at its four vertices
  const int32_t* sl_face;      // [nf][3] slot of a third of the face force at its vertices
  // per body tables
  const int32_t* b_face0; const int32_t* b_nf;
  const int32_t* b_vert0; const int32_t* b_nv;
  const int32_t* b_edge0; const int32_t* b_ne;
  const int32_t* b_rigid; const int32_t* b_fixed;
  const double* b_param;       // [nbody][8]: V0, S0, kv, m_v, mass, ks0, unused...
  double* b_rig;               // [nbody][32]: xc3 u3 uprev3 w3 wprev3 R9 Ibody9 (rigid state)
  const double* Xbody;         // [nv][3] body-frame offsets (rigid)
  double* b_diag;              // [nbody][16]: V S bbox(6) max_strain ...
  double* diag_part;           // [n_diag_blocks][12] partial diagnostics
  const int32_t* dblk_body;    // [n_diag_blocks] body of each diagnostics block
  const int32_t* b_dblk0;      // [nbody + 1] first diagnostics block of each body
  int n_marker_blocks, n_elem_blocks, n_diag_blocks;
  // Marker order: the marker blocks take the faces in slot order, slot s
  // holding face perm[s].  perm keeps each body's faces in its own slot
  // range (that of its face indices), sorted by the Hilbert key of their
  // stencil bases (k_bin_faces), so that a block's 64 faces are neighbours
  // whatever order the caller gave.  Results do not depend on it.
  // slot_f[s] = (the three vertex ids, body) of face perm[s], written with
  // perm, so that a marker reaches its vertices in one load instead of two.
  // The marker blocks take chunks of at most 64 consecutive slots: block c
  // the slots chunk_s0[c] .. + chunk_n[c] (0 for an unused chunk); body b
  // owns chunks b_chunk0[b] .. b_chunk0[b + 1] - 1 (CHUNK_CAP chunks per
  // 64 faces), cut by k_bin_faces where the sorted faces jump apart.
  int* perm;                   // [nf]
  int* slot_f;                 // [nf][4]
  int* chunk_s0;               // [n_marker_blocks]
  int* chunk_n;                // [n_marker_blocks]
  const int32_t* b_chunk0;     // [nbody + 1]
  unsigned long long* bin_keys;  // [sum of pow2 >= nf_b] sort buffer of bodies above BIN_LDS_KEYS
  const long long* b_key0;     // [nbody] offset of each body's part of bin_keys
  // per face / vertex work arrays
  double* centroid;            // [nf][3] by slot
  double* fext;                // [nf][3] hydrodynamic + repulsion force
  int* chunk_box;              // [n_marker_blocks][6] box of stencil bases of each chunk
  // Two-pass spread (null: one pass with atomics): each marker block's box
  // sums, [n_marker_blocks][BOX_CELLS][3] fixed point, and the node of each
  // box cell (-1: none), [n_marker_blocks][BOX_CELLS].
  long long* stage;
  int* stage_node;
  double* u0v;                 // [nv][3] interpolated velocity at vertices
  int n_clear_blocks;          // blocks clearing the previous step's force tiles
  double nu, umax;
};

// One instance of a batch: the arguments its own launches take, for one
// step parity (lbm_abi.cpp keeps two tables).
struct BatchItem {
  FluidArgs a;
  BodyArgs b;
  long long* fxc;         // force field written this step
  uint8_t* tfc;           // its tile flags
  long long* fxp;         // previous step's force field (cleared this step)
  uint8_t* tfp;
  unsigned int* counter;  // diagnostics block counter
  int nrb;                // record blocks ahead of the bulk tiles in the fluid phase
  int pad;
};

// Launchers (lbm_kernels.hip)
hipError_t launch_init(int prec, const Grid& g, void* f, const uint8_t* ncls, const double* rho,
                       const double* u, hipStream_t s);
hipError_t launch_fluid_bulk(int prec, const FluidArgs& a, hipStream_t s);
hipError_t launch_fluid_rec(int prec, const FluidArgs& a, hipStream_t s);
hipError_t launch_fluid_all(int prec, const FluidArgs& a, hipStream_t s);
hipError_t launch_close(DevFlags* flags, hipStream_t s);
hipError_t launch_ib_force(int prec, const FluidArgs& a, const BodyArgs& b, long long* fx_cur,
                           uint8_t* tf_cur, long long* fx_prev, uint8_t* tf_prev,
                           unsigned int* counter, hipStream_t s);
hipError_t launch_mls_post(int prec, const FluidArgs& a, const BodyArgs& b, long long* fxp, uint8_t* tfp,
                           hipStream_t s);
// with a counter (zeroed; left zeroed) it closes the step (steps_done, stop
// from pending) in its last block; with null, launch_close must follow
hipError_t launch_body_post(const BodyArgs& b, DevFlags* flags, unsigned int* counter, hipStream_t s);
// blocks of launch_body_post (the host's choice of closing in it)
inline unsigned body_post_blocks(const BodyArgs& b) { return (unsigned)b.nbody + (unsigned)((b.nsoft_v + 63) / 64); }
// Mass and momentum sums of the last completed step into out[5] (non-solid
// node count, sum of deviations, momentum); part holds 5 x 1024 doubles.
hipError_t launch_diag_sums(int prec, const Grid& g, const void* f0, const void* f1, const uint8_t* ncls,
                            const DevFlags* flags, double* part, double* out, hipStream_t s);
// Adjoint of the fluid step (no bodies; FluidArgs with A = the state g^k in
// [19][plane] in the context's storage, prec 0 FP64, 1 FP32 or 2 FP16S,
// bulk_list / nbulk_nodes set); the adjoint quantities are FP64 in all.  Solid entries
// of every buffer of the sweep hold zero and are never written.  merged:
// records and bulk nodes in one launch (small grids), else two.
// Buffers of one reverse step (from state k+1 back to state k).
struct AdjStep {
  const double* hrec;      // records' populations entering the collision of step k
  const double* lam;       // dJ/dg^{k+1} given directly (first step of the sweep), else null
  const double* mu_next;   // mu of step k+1 (when lam is null)
  double* acc_in;          // bounce-back transposes of mu_next, consumed (and cleared) here
  double* acc_out;         // bounce-back transposes of this step's mu, added here
  const double* w;         // per-step observable (may be null)
  double* mu;              // this step's mu
  const uint32_t* pmask;   // per node (bulk list, then records): plainly pulled directions
  const uint32_t* amask;   // per node: directions that can receive a bounce-back transpose
  double* part;            // [blocks][4] gradient partials
  // steps with bodies (null / 0 otherwise)
  const long long* fx;     // fixed-point IB force of the step [3][Np] ...
  const uint8_t* ftf;      // ... and its tile flags
  const double* ext;       // [7][Np] adjoint sources at nodes: dJ/drho, dJ/du of the step's
                           // fields (probes, vertex velocities), dJ/du* (forcing markers)
  const uint8_t* etf;      // tile flags of ext
  double* fbar;            // [3][Np] dJ/dF at the nodes of flagged force tiles (mode 1)
  int mode;                // 0: the step back; 1: only fbar, nothing else written
};
// Adjoint of the immersed-boundary part of a step (soft bodies).  The state
// a step maps is (g, P, Q, V): populations, positions x^n, previous
// positions x^{n-1} and vertex velocities; aP, aQ, aV are dJ/d of the state
// after the step, LP, Qn, Vn of the state before it.
struct AdjIB {
  const double* aP;
  const double* aQ;
  const double* aV;
  double* LP;        // [nv][3] dJ/dx^n (accumulated by several launches)
  double* Qn;        // [nv][3] dJ/dx^{n-1}
  double* Vn;        // [nv][3] dJ/du_v^n (accumulated)
  double* Fb;        // [nv][3] dJ/d(vertex force) of the step
  double* ub0;       // [nv][3] dJ/d(MLS vertex velocity) of the step
  double* ext;       // [7][Np] node sources (see AdjStep)
  uint8_t* etf;      // their tile flags
  const double* fbar;  // [3][Np] dJ/dF at the nodes of flagged force tiles
  double* gsum;      // [0] dJ/dtau through the probes' viscosity, [1] dJ/dkappa,
                     // [2 + b] sum over body b's faces of dJ/dF_face . A n (volume)
  double kappa;      // stiffness scale of the membrane moduli
};
// launch_adjoint_forward: g^{k+1} = step(A) into B; hrec (may be null):
// [19][nrec], the records' populations entering the collision.
// launch_adjoint_mask: pmask / amask (one word per bulk node, then per
// record; amask bit 31: w non-zero at the node), once per sweep, after w
// is in place.
// launch_adjoint_reverse: one step back, mu of step k from dJ/dg^{k+1}
// (st.lam, or P^T st.mu_next with st.acc_in) + st.w; the links' transposes
// of mu into st.acc_out; part[adj_part_blocks][ADJ_PART] += the step's
// derivatives of the inlet-velocity scale, the body force and omega, per
// block in a fixed order.
// launch_adjoint_gather: lam = P^T mu (with acc) after the last step back.
constexpr int ADJ_BLOCKS = 1024;
constexpr int ADJ_PART = 8;  // doubles per block of gradient partials (5 used)
inline int adj_part_blocks(long long nrec, long long nbulk) {
  const long long merged = (nrec + 255) / 256 + (nbulk + 255) / 256;
  return (int)(merged > 2 * ADJ_BLOCKS ? merged : 2 * ADJ_BLOCKS);
}
hipError_t launch_adjoint_forward(int prec, const FluidArgs& a, double* hrec, int merged, hipStream_t s);
hipError_t launch_adjoint_mask(const FluidArgs& a, const double* w, uint32_t* pmask, uint32_t* amask,
                               hipStream_t s);
hipError_t launch_adjoint_reverse(int prec, const FluidArgs& a, const AdjStep& st, int merged, hipStream_t s);
hipError_t launch_adjoint_gather(const FluidArgs& a, const uint32_t* pmask, const uint32_t* amask, const double* mu,
                                 const double* acc, double* lam, hipStream_t s);
hipError_t launch_adjoint_layout(const Grid& g, const uint8_t* ncls, const double* in, double* out, int to_padded,
                                 hipStream_t s);
// grad[0..4] from the partials (dJ/ds, dJ/dF, dJ/dtau), plus ibsum[0] in
// dJ/dtau and grad[5] = ibsum[1] (dJ/dkappa) when nout is 6 (ibsum may be null).
hipError_t launch_adjoint_grad(const double* part, int nblk, double omega, const double* ibsum, int nout,
                               double* grad, hipStream_t s);
// Coupled adjoint (soft bodies): vertex update transposed (Fb, ub0, Qn, LP,
// Vn = 0); elements, probes and vertex velocities transposed (LP, ext, gsum);
// the global volume term (LP); the forcing markers transposed (needs fbar:
// ext's dJ/du*, Vn, LP); the Taylor deformation of body `body` at X (its value
// added to *jsum, or theta times its gradient added to aP when aP is set);
// clearing of the flagged tiles of ext / fx after a step back.
hipError_t launch_adjb_vertex(const BodyArgs& b, const AdjIB& ib, hipStream_t s);
hipError_t launch_adjb_body(int prec, const FluidArgs& a, const BodyArgs& b, const AdjIB& ib, hipStream_t s);
hipError_t launch_adjb_volume(const BodyArgs& b, const AdjIB& ib, hipStream_t s);
hipError_t launch_adjb_support(const Grid& g, const uint8_t* ncls, const BodyArgs& b, uint8_t* etf, hipStream_t s);
hipError_t launch_adjb_markers(int prec, const FluidArgs& a, const BodyArgs& b, const AdjIB& ib, hipStream_t s);
hipError_t launch_taylor(const BodyArgs& b, const double* X, int body, double theta, double* aP, double* jsum,
                         hipStream_t s);
hipError_t launch_adjb_clear(const Grid& g, double* ext, uint8_t* etf, long long* fx, uint8_t* ftf, hipStream_t s);
// <w, g> over the non-solid nodes (where amask bit 31 is set when use_mask),
// added per block into part[ADJ_BLOCKS] (fixed order); the sum in *out.
hipError_t launch_adj_wdot(int prec, const FluidArgs& a, const void* g, const double* w, const uint32_t* amask,
                           int use_mask, double* part, hipStream_t s);
hipError_t launch_adj_sum(const double* part, int n, double* out, hipStream_t s);

hipError_t launch_check(const BodyArgs& b, const double* X0, const double* X1, DevFlags* flags,
                        unsigned int* counter, hipStream_t s);
// Sorts each body's faces into marker slots by the Morton code of their
// stencil bases at b.Xcur (b.perm); one block of 1024 threads per body.
hipError_t launch_bin_faces(const BodyArgs& b, hipStream_t s);
// to[0..nv3) = from[nv3..2 nv3), to[nv3..2 nv3) = from[0..nv3), to[2 nv3..3 nv3)
// = from[2 nv3..3 nv3): a coupled step's body slot set up from its input's.
hipError_t launch_body_slots(const double* from, double* to, long long nv3, hipStream_t s);
// Owner pass of the two-pass spread (b.stage set): adds the staged box sums
// into fxc without atomics and flags the tiles.
hipError_t launch_spread_owner(const Grid& g, const BodyArgs& b, long long* fxc, uint8_t* tfc,
                               const DevFlags* flags, hipStream_t s);
hipError_t launch_set_populations(int prec, const Grid& g, void* f0, void* f1, const uint8_t* ncls,
                                  const DevFlags* flags, const double* pops, hipStream_t s);
hipError_t launch_get_fields(int prec, const Grid& g, const void* f0, const void* f1,
                             const uint8_t* ncls, const long long* fx0, const long long* fx1,
                             const uint8_t* tf0, const uint8_t* tf1, double gx, double gy,
                             double gz, const DevFlags* flags, double* rho, double* u,
                             double* pops, double* fib, hipStream_t s);
hipError_t launch_interp(int prec, const Grid& g, const void* f0, const void* f1,
                         const uint8_t* ncls, const long long* fx0, const long long* fx1,
                         const uint8_t* tf0, const uint8_t* tf1, double gx, double gy, double gz,
                         const DevFlags* flags, long long n, const double* pts,
                         const double* field, double* out, hipStream_t s);
hipError_t launch_spread_api(const Grid& g, const uint8_t* ncls, long long n, const double* pts,
                             const double* F, const double* c, long long* fx, DevFlags* flags,
                             hipStream_t s);
hipError_t launch_flush_fx(const Grid& g, long long* fx, double* fib, hipStream_t s);

// Allocation-free spread: a fixed scratch array in device memory (one copy
// per GPU, held until the process ends) holds the fixed-point sums of up to
// NOALLOC_MAX_NODES padded nodes ([3][NOALLOC_MAX_NODES] 64-bit words, 48 MiB)
// followed by NOALLOC_FLAG_WORDS words for the range flags.
constexpr long long NOALLOC_MAX_NODES = 1LL << 21;
constexpr long long NOALLOC_FLAG_WORDS = 32;
constexpr int NOALLOC_MAX_DEVICES = 64;
static_assert(sizeof(DevFlags) <= NOALLOC_FLAG_WORDS * 8, "flags fit the scratch tail");
// Device address of the scratch on `device` (looked up once per device with
// that device current, then kept).
hipError_t noalloc_scratch(int device, long long** out);
// Clear the scratch for the lattice, spread, add the sums into fib (as
// ib_spread does with its own buffer); overflow is reported in the flags at
// scr + 3 NOALLOC_MAX_NODES.  Requires g.Np <= NOALLOC_MAX_NODES.
hipError_t launch_spread_noalloc(const Grid& g, const uint8_t* ncls, long long n, const double* pts,
                                 const double* F, const double* c, double* fib, long long* scr,
                                 hipStream_t s);

// Launch shape of the batched fluid phase: blocks of `block` threads, V
// nodes per bulk thread (0: list form); mode 0 merged (map_all), 1 split
// (map_rec, then map_bulk); per_xcd > 0 runs the merged units, or the bulk
// tiles, persistently with per_xcd blocks per XCD.
struct BatchFluid {
  int V, block, mode, per_xcd;
  const int2* map_all; int n_all;
  const int2* map_rec; int n_rec;
  const int2* map_bulk; int n_bulk;
};

// Batched phases: n blocks (units) each, map[g] = (instance, unit).
hipError_t launch_batch_ib_force(int prec, const BatchItem* items, const int2* map, int n,
                                 hipStream_t s);
hipError_t launch_batch_fluid(int prec, const BatchFluid& f, const BatchItem* items, hipStream_t s);
hipError_t launch_batch_mls_post(int prec, const BatchItem* items, const int2* map, int n,
                                 hipStream_t s);
hipError_t launch_batch_body_post(const BatchItem* items, const int2* map, int n, hipStream_t s);
hipError_t launch_batch_close(const BatchItem* items, int n, hipStream_t s);

}  // namespace lbm
