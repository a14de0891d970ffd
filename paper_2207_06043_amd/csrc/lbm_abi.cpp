// Host side of the C ABI declared in include/lbm.h: validation, node
// classification, boundary records, body set-up, graph capture and the
// ABI entry points.  All per-step arithmetic runs in lbm_kernels.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <string>
#include <utility>
#include <vector>

#include "lbm.h"
#include "lbm_internal.h"

using namespace lbm;

namespace {

// D3Q19 velocity set (order of the paper's Eq. e_i).
const int HX[19] = {0, 1, -1, 0, 0, 0, 0, 1, 1, 1, 1, -1, -1, -1, -1, 0, 0, 0, 0};
const int HY[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, 0, 0, 1, -1, 0, 0, 1, 1, -1, -1};
const int HZ[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 1, -1, 0, 0, 1, -1, 1, -1, 1, -1};
const int HOPP[19] = {0, 2, 1, 4, 3, 6, 5, 12, 11, 14, 13, 8, 7, 10, 9, 18, 17, 16, 15};

struct HostBody {
  int nv, nf, rigid, fixed;
  std::vector<double> x0, v0;
  std::vector<int> faces;  // local ids
  std::vector<int> edges;  // local ids [ne][2]
  std::vector<double> l0, kl;
  std::vector<int> hinges;  // local [nh][4]
  std::vector<double> theta0, kb;
  double V0, S0, ks0, kv, m_v, mass;
  bool kv_default;  // kv = 10 k_s0 / r_ref (follows the stiffness scale)
  double cm[3], Ibody[9];
  std::vector<double> Xbody;
};

}  // namespace

struct lbm_ctx {
  int device = 0;                  // HIP device the context was created on
  hipStream_t stream = nullptr;
  hipStream_t cap = nullptr;
  hipStream_t side = nullptr;      // boundary-record kernel (forked from the step stream)
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  std::string err;
  bool broken = false;
  Grid g{};
  int prec = 0;
  size_t ssize = 8;
  double tau = 0.8, umax = 0.0, gfx = 0, gfy = 0, gfz = 0;
  int64_t n_fluid = 0, n_bulk = 0, n_general = 0, n_links = 0;
  // fluid device state
  void* f[2] = {nullptr, nullptr};        // first element of plane 0
  void* f_alloc[2] = {nullptr, nullptr};  // allocations (with guard regions)
  uint8_t* ncls = nullptr;
  int32_t* rec_of = nullptr;
  int nrec = 0;
  int32_t* rec_node = nullptr;
  uint32_t* rec_mask = nullptr;
  int32_t* rec_link0 = nullptr;
  uint8_t* rec_face = nullptr;
  double* rec_bc = nullptr;
  void* lk_c = nullptr;        // [3][nlinks] in the compute type
  uint32_t* rec_mb = nullptr;  // [nrec] bit j: link j has q >= 1/2
  int nlinks_rec = 0;
  int32_t* tile_list = nullptr;
  int32_t* bulk_list = nullptr;  // list form: the bulk nodes in order (built on first use)
  int nbulk_blocks = 0;
  long long ntiles = 0;
  long long* fx[2] = {nullptr, nullptr};
  uint8_t* tf[2] = {nullptr, nullptr};
  void* mac = nullptr;  // [Np][4] rho - 1, u of the step in the compute type (bodies only)
  long long* fx_api = nullptr;
  double* gdiag = nullptr;  // global mass/momentum reduction: 5 x 1024 partials + 5 results
  DevFlags* api_flags = nullptr;  // range flags of ib_spread (kept apart from the run's)
  DevFlags* flags = nullptr;  // followed by the block counter
  // bodies
  std::vector<HostBody> bodies;
  int nv = 0, nf = 0, ne = 0, nh = 0, nsoft_v = 0;
  std::vector<void*> bod_alloc;
  BodyArgs bargs[2]{};
  double* X[2] = {nullptr, nullptr};
  double* Vel = nullptr;
  double* b_rig = nullptr;
  double* b_diag = nullptr;
  // graphs
  bool use_graph = true;
  int rec_block = 64;
  int bulk_v = 4;
  int bulk_block = 256;
  bool fluid_merged = false;  // records and bulk tiles in one launch (small grids)
  // spread in two passes (staged block sums, then an owner pass without
  // atomics) instead of atomics; LBM_SPREAD_TWO_PASS=1 at creation
  bool spread_two_pass = false;
  bool graph_valid = false;
  hipGraphExec_t gexec[3] = {nullptr, nullptr, nullptr};
  int64_t enq = 0;
  int64_t bin_enq = 0;  // enq at the last sort of the marker order
  std::vector<uint8_t> ncls_h;  // node classes (host copy: bulk tiles of other launch shapes)
  uint64_t version = 0;         // bumped when bodies or the launch shape change
  // parameter scales (lbm_set_scales): inlet wall velocities and membrane moduli
  double inlet_scale = 1.0, stiff_scale = 1.0;
  std::vector<double> rec_bc_h;  // [4][nrec] as created (scale 1)
};

#define CHK(expr)                                                                    \
  do {                                                                               \
    hipError_t e_ = (expr);                                                          \
    if (e_ != hipSuccess) {                                                          \
      ctx->broken = true;                                                            \
      ctx->err = std::string("HIP error: ") + hipGetErrorString(e_) + " at " + #expr; \
      return LBM_E_HIP;                                                              \
    }                                                                                \
  } while (0)

// Block counters live after the flags word: 0 k_ib_force, 1 k_body_post,
// 2 k_fluid (fluid-only steps), 3 k_check.
static unsigned int* counter(lbm_ctx* ctx, int k) { return (unsigned int*)(ctx->flags + 1) + k; }

static lbm_status fail(lbm_ctx* ctx, lbm_status st, const std::string& msg) {
  if (ctx) ctx->err = msg;
  return st;
}

template <class T>
static hipError_t dalloc(T** p, size_t n) {
  if (n == 0) n = 1;
  return hipMalloc((void**)p, n * sizeof(T));
}

template <class T>
static hipError_t upload(T** p, const std::vector<T>& v) {
  hipError_t e = dalloc(p, v.size());
  if (e != hipSuccess) return e;
  if (!v.empty()) e = hipMemcpy(*p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice);
  return e;
}

static void free_graphs(lbm_ctx* ctx) {
  for (int p = 0; p < 3; p++)
    if (ctx->gexec[p]) {
      (void)hipGraphExecDestroy(ctx->gexec[p]);
      ctx->gexec[p] = nullptr;
    }
  ctx->graph_valid = false;
}

static void free_bodies(lbm_ctx* ctx) {
  for (void* p : ctx->bod_alloc) (void)hipFree(p);
  ctx->bod_alloc.clear();
}

// Bulk tiles: blocks of `block` threads x V nodes holding at least one bulk
// node.
static std::vector<int32_t> bulk_tiles(const Grid& G, const std::vector<uint8_t>& ncls, int block, int V) {
  const long long tnodes = (long long)block * V;
  std::vector<int32_t> tiles;
  for (long long t = 0; t * tnodes < G.Np; t++) {
    bool any = false;
    for (long long k = t * tnodes; k < std::min(G.Np, (t + 1) * tnodes) && !any; k++)
      any = ncls[k] == CLS_BULK;
    if (any) tiles.push_back((int32_t)t);
  }
  return tiles;
}

static bool shape_ok(int prec, int V, int block) {
  const bool vok = V == 0 || (prec == 0 && (V == 1 || V == 2)) ||
                   (prec == 1 && (V == 1 || V == 2 || V == 4)) || (prec == 2 && (V == 2 || V == 4 || V == 8));
  return vok && (block == 64 || block == 128 || block == 256);
}

// List form of the bulk part (launch shape V = 0): the bulk node indices in
// order, one per thread.
static hipError_t ensure_bulk_list(lbm_ctx* ctx) {
  if (ctx->bulk_list) return hipSuccess;
  std::vector<int32_t> lst;
  lst.reserve((size_t)ctx->n_bulk);
  for (long long n = 0; n < (long long)ctx->ncls_h.size(); n++)
    if (ctx->ncls_h[n] == CLS_BULK) lst.push_back((int32_t)n);
  if (lst.empty()) lst.push_back(0);  // never read (no bulk blocks), keeps the allocation non-empty
  return upload(&ctx->bulk_list, lst);
}

static int bulk_blocks(const lbm_ctx* ctx, int V, int block, size_t ntiles) {
  return V == 0 ? (int)((ctx->n_bulk + block - 1) / block) : (int)ntiles;
}

// ------------------------------------------------------------------ create
extern "C" lbm_status lbm_create(const lbm_desc* d, void* hip_stream, lbm_ctx** out) {
  if (!out) return LBM_E_INVAL;
  *out = nullptr;
  if (!d || !d->node_type) return LBM_E_INVAL;
  lbm_ctx* ctx = new lbm_ctx();
  auto bad = [&](const std::string& m) {
    *out = ctx;  // hand back the context so the caller can read the message
    return fail(ctx, LBM_E_INVAL, m);
  };
  if (d->nx < 1 || d->ny < 1 || d->nz < 1) return bad("grid sizes must be >= 1");
  if (!(d->tau > 0.5)) return bad("tau must be > 1/2");
  if (d->precision < 0 || d->precision > 2) return bad("unknown precision");
  if ((long long)d->nx * d->ny * d->nz > (1LL << 31) - (1LL << 20)) return bad("grid too large");
  ctx->stream = (hipStream_t)hip_stream;
  ctx->prec = d->precision;
  {
    // the context lives on the current device; look up that device's
    // scratch of the allocation-free spread once, here, with it current
    if (hipGetDevice(&ctx->device) != hipSuccess) return bad("no HIP device");
    long long* scr = nullptr;
    if (noalloc_scratch(ctx->device, &scr) != hipSuccess) return bad("device scratch not addressable");
  }
  // launch shape (defaults; overridable for tuning): few non-solid nodes
  // (cache-resident, latency-bound; or a sparse box, where big tiles would
  // mostly cover solid nodes): one merged launch, one node per thread (the
  // list form in FP16S); many (HBM-bound): split launches, vector accesses
  long long n_open = 0;
  {
    const long long Nb = (long long)d->nx * d->ny * d->nz;
    for (long long n = 0; n < Nb; n++) n_open += d->node_type[n] != LBM_NODE_SOLID;
  }
  const bool large = n_open >= (4LL << 20);
  // measured on MI355X: FP16S runs 2 nodes per thread in 128-thread blocks
  // on large grids (8 per thread: 1.6x slower) and the list form on small
  // ones (24% faster than 2 per thread on the precision form); FP32 one
  // node per thread (the D = 96 pipe 3% faster than 4, the 256^3 box the same)
  ctx->bulk_v = large ? (d->precision == 0 ? 2 : (d->precision == 1 ? 1 : 2)) : (d->precision == 2 ? 0 : 1);
  // small grids: 128-thread tiles in FP32 (the bifurcation with its capsule:
  // 15.0 us per fluid launch against 15.6 with 64), 64-thread tiles in FP64
  // (the pipe with a sphere: 9.1 against 9.7 us with 128), the list form in
  // 64-thread blocks in FP16S
  ctx->bulk_block = large ? (d->precision == 2 ? 128 : 256) : (d->precision == 1 ? 128 : 64);
  // small grids: one fluid launch (no fork/join between streams) with the
  // record blocks in the same shape as the bulk tiles
  ctx->fluid_merged = !large;
  if (const char* ev = getenv("LBM_RECORD_BLOCK")) ctx->rec_block = atoi(ev);
  if (const char* ev = getenv("LBM_BULK_V")) ctx->bulk_v = atoi(ev);
  if (const char* ev = getenv("LBM_BULK_BLOCK")) ctx->bulk_block = atoi(ev);
  if (const char* ev = getenv("LBM_FLUID_SPLIT")) ctx->fluid_merged = atoi(ev) == 0;
  if (const char* ev = getenv("LBM_SPREAD_TWO_PASS")) ctx->spread_two_pass = atoi(ev) != 0;
  if (ctx->fluid_merged) ctx->rec_block = ctx->bulk_block;
  if (!shape_ok(d->precision, ctx->bulk_v, ctx->bulk_block) ||
      (ctx->rec_block != 64 && ctx->rec_block != 128 && ctx->rec_block != 256))
    return bad("unsupported launch shape");
  ctx->ssize = d->precision == 0 ? 8 : (d->precision == 1 ? 4 : 2);
  ctx->tau = d->tau;
  ctx->umax = d->u_max;
  ctx->gfx = d->body_force[0];
  ctx->gfy = d->body_force[1];
  ctx->gfz = d->body_force[2];
  Grid& G = ctx->g;
  G.nx = d->nx;
  G.ny = d->ny;
  G.nz = d->nz;
  for (int a = 0; a < 3; a++) G.per[a] = d->periodic[a] ? 1 : 0;
  G.px = (d->nx + 7) / 8 * 8;
  G.Np = (long long)G.px * G.ny * G.nz;
  G.plane = (G.Np + 64 + 63) / 64 * 64;
  G.guard = ((long long)G.px * G.ny + G.px + 16 + 63) / 64 * 64;
  {
    auto magic = [](unsigned int d, unsigned int& m, int& s) {
      int l = 0;
      while ((1ull << l) < d) l++;
      s = 31 + l;
      m = (unsigned int)(((1ull << s) + d - 1) / d);
    };
    magic((unsigned int)G.px, G.mpx, G.spx);
    magic((unsigned int)G.ny, G.mny, G.sny);
  }
  // the kernels take padded indices, the guard rows of both sides included,
  // as int
  if ((long long)G.px * G.ny * (G.nz + 2) + 2LL * G.px + 1024 >= (1LL << 31)) return bad("grid too large");
  const long long N = (long long)d->nx * d->ny * d->nz;
  const int nx = d->nx, ny = d->ny, nz = d->nz;
  auto lin = [&](int x, int y, int z) { return x + (long long)nx * (y + (long long)ny * z); };
  auto pad = [&](int x, int y, int z) { return x + (long long)G.px * (y + (long long)G.ny * z); };
  const int dim[3] = {nx, ny, nz};
  // neighbour with periodic wrap; false if it leaves through a closed face
  auto nb = [&](int x, int y, int z, int dx, int dy, int dz, int* c) {
    c[0] = x + dx;
    c[1] = y + dy;
    c[2] = z + dz;
    for (int a = 0; a < 3; a++) {
      if (c[a] < 0 || c[a] >= dim[a]) {
        if (!G.per[a]) return false;
        c[a] = ((c[a] % dim[a]) + dim[a]) % dim[a];
      }
    }
    return true;
  };
  const uint8_t* nt = d->node_type;
  for (long long n = 0; n < N; n++)
    if (nt[n] > 3) return bad("node_type values must be 0..3");
  // wall links, keyed by (node, pulled direction j = opposite of the link direction)
  std::map<std::pair<long long, int>, double> links;
  for (int64_t k = 0; k < d->n_links; k++) {
    const long long n = d->link_node[k];
    const int i = d->link_dir[k];
    const double q = d->link_q[k];
    if (n < 0 || n >= N || i < 1 || i > 18 || !(q >= 0.0 && q <= 1.0))
      return bad("wall link " + std::to_string(k) + " out of range");
    if (nt[n] == LBM_NODE_SOLID) return bad("wall link " + std::to_string(k) + " starts on a solid node");
    const int x = (int)(n % nx), y = (int)((n / nx) % ny), z = (int)(n / ((long long)nx * ny));
    int c[3];
    if (!nb(x, y, z, HX[i], HY[i], HZ[i], c) || nt[lin(c[0], c[1], c[2])] != LBM_NODE_SOLID)
      return bad("wall link " + std::to_string(k) + " does not point at a solid node");
    if (!links.emplace(std::make_pair(n, HOPP[i]), q).second)
      return bad("duplicate wall link " + std::to_string(k));
  }
  ctx->n_links = d->n_links;
  // classify
  std::vector<uint8_t> ncls(G.Np, CLS_SOLID);
  std::vector<int32_t> rec_of(G.Np, -1);
  std::vector<int32_t> r_node;
  std::vector<uint32_t> r_mask;
  std::vector<int32_t> r_link0;
  std::vector<uint8_t> r_face;
  std::vector<double> r_bc;  // 4 per record, transposed later
  std::vector<double> l_c;  // 5 per link, transposed below
  long long n_inlet_seen = 0;
  for (int z = 0; z < nz; z++)
    for (int y = 0; y < ny; y++)
      for (int x = 0; x < nx; x++) {
        const long long n = lin(x, y, z);
        const uint8_t t = nt[n];
        if (t == LBM_NODE_SOLID) continue;
        ctx->n_fluid++;
        const bool open = t == LBM_NODE_INLET || t == LBM_NODE_OUTLET;
        int face = -1, nfaces = 0;
        const int cc[3] = {x, y, z};
        for (int a = 0; a < 3; a++) {
          if (G.per[a]) continue;
          if (cc[a] == 0) { face = 2 * a; nfaces++; }
          if (cc[a] == dim[a] - 1) { face = 2 * a + 1; nfaces++; }
        }
        if (open && nfaces != 1)
          return bad("open node " + std::to_string(n) + " must lie on exactly one non-periodic face");
        bool general = open;
        uint32_t mask = 0;
        for (int j = 1; j < 19; j++) {
          int c[3];
          const bool in = nb(x, y, z, -HX[j], -HY[j], -HZ[j], c);
          if (!in) {
            if (!open) return bad("fluid node " + std::to_string(n) + " on a closed box face");
            continue;
          }
          if (nt[lin(c[0], c[1], c[2])] == LBM_NODE_SOLID) {
            if (!links.count(std::make_pair(n, j)))
              return bad("node " + std::to_string(n) + " has a solid neighbour in direction " +
                         std::to_string(HOPP[j]) + " without a wall link");
            mask |= 1u << j;
            general = true;
          }
        }
        const long long p = pad(x, y, z);
        if (!general) {
          ncls[p] = CLS_BULK;
          ctx->n_bulk++;
          continue;
        }
        ncls[p] = CLS_GENERAL;
        ctx->n_general++;
        rec_of[p] = (int32_t)r_node.size();
        r_node.push_back((int32_t)p);
        r_mask.push_back(mask);
        r_link0.push_back((int32_t)(l_c.size() / 5));
        uint8_t fc = 0xff;
        double bc[4] = {0, 0, 0, 0};
        if (open) {
          fc = (uint8_t)(face | (t == LBM_NODE_OUTLET ? 0x10 : 0));
          if (t == LBM_NODE_INLET) {
            if (d->inlet_u)
              for (int a = 0; a < 3; a++) bc[a] = d->inlet_u[3 * n_inlet_seen + a];
            n_inlet_seen++;
          } else {
            bc[3] = d->outlet_rho;
          }
        }
        r_face.push_back(fc);
        for (int a = 0; a < 4; a++) r_bc.push_back(bc[a]);
        for (int j = 1; j < 19; j++) {
          if (!(mask & (1u << j))) continue;
          const double q = links[std::make_pair(n, j)];
          // availability of x - e_i = x + e_j and x - 2e_i = x + 2e_j (i = opposite of j)
          int c1[3], c2[3];
          const bool a1 = nb(x, y, z, HX[j], HY[j], HZ[j], c1) && nt[lin(c1[0], c1[1], c1[2])] != LBM_NODE_SOLID;
          const bool a2 = nb(x, y, z, 2 * HX[j], 2 * HY[j], 2 * HZ[j], c2) &&
                          nt[lin(c2[0], c2[1], c2[2])] != LBM_NODE_SOLID;
          // Eq. bbouzidi as c0 f*_i(x) + c1 f*_i(x-e_i) + c2 f*_i(x-2e_i) + c3 f*_j(x)
          // + c4 f*_j(x-e_i); linear / plain bounce-back where neighbours are missing
          double c[5] = {0, 0, 0, 0, 0};
          if (q < 0.5) {
            if (a1 && a2) {
              c[0] = q * (1.0 + 2.0 * q);
              c[1] = 1.0 - 4.0 * q * q;
              c[2] = -q * (1.0 - 2.0 * q);
            } else if (a1) {
              c[0] = 2.0 * q;
              c[1] = 1.0 - 2.0 * q;
            } else {
              c[0] = 1.0;
            }
          } else if (a1) {
            c[0] = 1.0 / (q * (2.0 * q + 1.0));
            c[3] = (2.0 * q - 1.0) / q;
            c[4] = (1.0 - 2.0 * q) / (1.0 + 2.0 * q);
          } else {
            c[0] = 1.0 / (2.0 * q);
            c[3] = (2.0 * q - 1.0) / (2.0 * q);
          }
          for (int k = 0; k < 5; k++) l_c.push_back(c[k]);
        }
      }
  for (const auto& kv : links)
    if (!(nt[kv.first.first] != LBM_NODE_SOLID)) return bad("wall link on a solid node");
  ctx->nrec = (int)r_node.size();
  std::vector<double> bcT(4 * (size_t)ctx->nrec);
  for (int r = 0; r < ctx->nrec; r++)
    for (int a = 0; a < 4; a++) bcT[(size_t)a * ctx->nrec + r] = r_bc[4 * (size_t)r + a];
  std::vector<int32_t> tiles =
      ctx->bulk_v > 0 ? bulk_tiles(G, ncls, ctx->bulk_block, ctx->bulk_v) : std::vector<int32_t>(1, 0);
  ctx->nbulk_blocks = bulk_blocks(ctx, ctx->bulk_v, ctx->bulk_block, tiles.size());
  ctx->ntiles = (G.Np >> TILE_SHIFT) + 1;
  // device allocations
  CHK(hipStreamCreateWithFlags(&ctx->cap, hipStreamNonBlocking));
  CHK(hipStreamCreateWithFlags(&ctx->side, hipStreamNonBlocking));
  CHK(hipEventCreateWithFlags(&ctx->ev_fork, hipEventDisableTiming));
  CHK(hipEventCreateWithFlags(&ctx->ev_join, hipEventDisableTiming));
  const size_t fbytes = ((size_t)19 * G.plane + 2 * (size_t)G.guard) * ctx->ssize;
  for (int p = 0; p < 2; p++) {
    CHK(hipMalloc(&ctx->f_alloc[p], fbytes));
    CHK(hipMemset(ctx->f_alloc[p], 0, fbytes));
    ctx->f[p] = (char*)ctx->f_alloc[p] + (size_t)G.guard * ctx->ssize;
  }
  CHK(upload(&ctx->ncls, ncls));
  ctx->ncls_h = ncls;
  if (ctx->bulk_v == 0) CHK(ensure_bulk_list(ctx));
  CHK(upload(&ctx->rec_of, rec_of));
  CHK(upload(&ctx->rec_node, r_node));
  CHK(upload(&ctx->rec_mask, r_mask));
  CHK(upload(&ctx->rec_link0, r_link0));
  CHK(upload(&ctx->rec_face, r_face));
  CHK(upload(&ctx->rec_bc, bcT));
  ctx->rec_bc_h = bcT;
  // Each branch of the rule has three terms: q < 1/2 uses c0 f_i(x),
  // c1 f_i(x-e_i), c2 f_i(x-2e_i); q >= 1/2 uses c0 f_i(x), c3 f_j(x),
  // c4 f_j(x-e_i).  Stored per link as k0, k1, k2 (in that order, [3][nl],
  // compute type) with one bit per record and direction saying which branch.
  const size_t nl = l_c.size() / 5;
  std::vector<double> lcT(std::max<size_t>(3 * nl, 3), 0.0);  // entry 0 always exists
  std::vector<uint32_t> mb((size_t)std::max(ctx->nrec, 1), 0u);
  for (int r = 0; r < ctx->nrec; r++) {
    int lk = r_link0[r];
    for (int j = 1; j < 19; j++) {
      if (!((r_mask[r] >> j) & 1u)) continue;
      const double* c = &l_c[5 * (size_t)lk];
      const bool hq = c[1] == 0.0 && c[2] == 0.0 && (c[3] != 0.0 || c[4] != 0.0);
      if (hq) mb[r] |= 1u << j;
      lcT[lk] = c[0];
      lcT[nl + lk] = hq ? c[3] : c[1];
      lcT[2 * nl + lk] = hq ? c[4] : c[2];
      ++lk;
    }
  }
  ctx->nlinks_rec = (int)nl;
  if (ctx->prec == 0) {
    CHK(upload((double**)&ctx->lk_c, lcT));
  } else {
    std::vector<float> lcf(lcT.begin(), lcT.end());
    CHK(upload((float**)&ctx->lk_c, lcf));
  }
  CHK(upload(&ctx->rec_mb, mb));
  CHK(upload(&ctx->tile_list, tiles));
  CHK(hipMalloc(&ctx->flags, sizeof(DevFlags) + 64));
  CHK(hipMemset(ctx->flags, 0, sizeof(DevFlags) + 64));
  // initial populations: equilibrium of the given fields
  double *drho = nullptr, *du = nullptr;
  if (d->init_rho) {
    CHK(hipMalloc(&drho, N * sizeof(double)));
    CHK(hipMemcpy(drho, d->init_rho, N * sizeof(double), hipMemcpyHostToDevice));
  }
  if (d->init_u) {
    CHK(hipMalloc(&du, 3 * N * sizeof(double)));
    CHK(hipMemcpy(du, d->init_u, 3 * N * sizeof(double), hipMemcpyHostToDevice));
  }
  CHK(launch_init(ctx->prec, G, ctx->f[0], ctx->ncls, drho, du, ctx->cap));
  CHK(hipStreamSynchronize(ctx->cap));
  if (drho) CHK(hipFree(drho));
  if (du) CHK(hipFree(du));
  *out = ctx;
  return LBM_OK;
}

extern "C" lbm_status lbm_destroy(lbm_ctx* ctx) {
  if (!ctx) return LBM_OK;
  (void)hipDeviceSynchronize();
  free_graphs(ctx);
  free_bodies(ctx);
  void* ptrs[] = {ctx->f_alloc[0], ctx->f_alloc[1], ctx->ncls, ctx->rec_of, ctx->rec_node, ctx->rec_mask,
                  ctx->rec_link0, ctx->rec_face, ctx->rec_bc, ctx->lk_c, ctx->rec_mb,
                  ctx->tile_list, ctx->bulk_list, ctx->fx[0], ctx->fx[1], ctx->tf[0], ctx->tf[1], ctx->fx_api,
                  ctx->api_flags, ctx->mac, ctx->flags, ctx->gdiag};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  if (ctx->cap) (void)hipStreamDestroy(ctx->cap);
  if (ctx->side) (void)hipStreamDestroy(ctx->side);
  if (ctx->ev_fork) (void)hipEventDestroy(ctx->ev_fork);
  if (ctx->ev_join) (void)hipEventDestroy(ctx->ev_join);
  delete ctx;
  return LBM_OK;
}

extern "C" const char* lbm_last_error(const lbm_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

static lbm_status read_flags(lbm_ctx* ctx, DevFlags* h) {
  CHK(hipStreamSynchronize(ctx->stream));
  CHK(hipMemcpy(h, ctx->flags, sizeof(DevFlags), hipMemcpyDeviceToHost));
  return LBM_OK;
}

extern "C" lbm_status lbm_info(lbm_ctx* ctx, lbm_info_t* o) {
  if (!ctx || !o) return LBM_E_INVAL;
  if (ctx->broken) return LBM_E_STATE;
  DevFlags h;
  lbm_status st = read_flags(ctx, &h);
  if (st) return st;
  o->n_nodes = (int64_t)ctx->g.nx * ctx->g.ny * ctx->g.nz;
  o->n_fluid = ctx->n_fluid;
  o->n_bulk = ctx->n_bulk;
  o->n_general = ctx->n_general;
  o->n_links = ctx->n_links;
  o->n_bodies = (int64_t)ctx->bodies.size();
  o->n_vertices = ctx->nv;
  o->n_faces = ctx->nf;
  o->steps_done = h.steps_done;
  o->bytes_per_step_alg = 2 * 19 * (int64_t)ctx->ssize * ctx->n_fluid;
  o->precision = ctx->prec;
  o->mls_singular = h.mls_singular;
  o->fluid_launch = ctx->fluid_merged ? 1 : 2;
  o->pad = 0;
  return LBM_OK;
}

// ------------------------------------------------------------------ bodies
static void cross(const double* a, const double* b, double* c) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}

static double dihedral_host(const double* X, const int* h) {
  const double *a = X + 3 * h[0], *b = X + 3 * h[1], *c = X + 3 * h[2], *d = X + 3 * h[3];
  double e[3], ca[3], ab[3], db[3], n1[3], n2[3], t[3];
  for (int k = 0; k < 3; k++) {
    e[k] = b[k] - a[k];
    ca[k] = c[k] - a[k];
    ab[k] = a[k] - b[k];
    db[k] = d[k] - b[k];
  }
  cross(e, ca, n1);
  cross(ab, db, n2);
  double l1 = std::sqrt(n1[0] * n1[0] + n1[1] * n1[1] + n1[2] * n1[2]);
  double l2 = std::sqrt(n2[0] * n2[0] + n2[1] * n2[1] + n2[2] * n2[2]);
  double le = std::sqrt(e[0] * e[0] + e[1] * e[1] + e[2] * e[2]);
  for (int k = 0; k < 3; k++) {
    n1[k] /= l1;
    n2[k] /= l2;
  }
  cross(n1, n2, t);
  return std::atan2((t[0] * e[0] + t[1] * e[1] + t[2] * e[2]) / le,
                    n1[0] * n2[0] + n1[1] * n2[1] + n1[2] * n2[2]);
}

static double tri_area(const double* X, int a, int b, int c) {
  double u[3], v[3], n[3];
  for (int k = 0; k < 3; k++) {
    u[k] = X[3 * b + k] - X[3 * a + k];
    v[k] = X[3 * c + k] - X[3 * a + k];
  }
  cross(u, v, n);
  return 0.5 * std::sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
}

// Upload all bodies (host rest data + current dynamic state) into fresh
// device arrays; dyn_* hold the dynamic state of the bodies already present.
static lbm_status build_body_arrays(lbm_ctx* ctx, int cur, const std::vector<double>& Xc,
                                    const std::vector<double>& Xp, const std::vector<double>& Vl,
                                    const std::vector<double>& rig) {
  free_bodies(ctx);
  const int nb = (int)ctx->bodies.size();
  std::vector<int32_t> faces, face_body, vert_body, edges, hinges, soft;
  std::vector<double> l0, kl, th0, kb, Xbody, param(8 * (size_t)nb + 9 * (size_t)nb);
  std::vector<int32_t> bf0, bnf, bv0, bnv, be0, bne, brig, bfix;
  int v0 = 0, f0 = 0, e0 = 0;
  for (int b = 0; b < nb; b++) {
    const HostBody& B = ctx->bodies[b];
    bf0.push_back(f0);
    bnf.push_back(B.nf);
    bv0.push_back(v0);
    bnv.push_back(B.nv);
    be0.push_back(e0);
    bne.push_back((int)B.l0.size());
    brig.push_back(B.rigid || B.fixed);
    bfix.push_back(B.fixed);
    for (int k = 0; k < 3 * B.nf; k++) faces.push_back(B.faces[k] + v0);
    for (int f = 0; f < B.nf; f++) face_body.push_back(b);
    for (int v = 0; v < B.nv; v++) {
      vert_body.push_back(b);
      if (!(B.rigid || B.fixed)) soft.push_back(v0 + v);
    }
    for (size_t k = 0; k < B.edges.size(); k++) edges.push_back(B.edges[k] + v0);
    for (size_t k = 0; k < B.hinges.size(); k++) hinges.push_back(B.hinges[k] + v0);
    l0.insert(l0.end(), B.l0.begin(), B.l0.end());
    for (double k : B.kl) kl.push_back(k * ctx->stiff_scale);
    th0.insert(th0.end(), B.theta0.begin(), B.theta0.end());
    for (double k : B.kb) kb.push_back(k * ctx->stiff_scale);
    Xbody.insert(Xbody.end(), B.Xbody.begin(), B.Xbody.end());
    double* pp = param.data() + 8 * b;
    pp[0] = B.V0;
    pp[1] = B.S0;
    pp[2] = B.kv * (B.kv_default ? ctx->stiff_scale : 1.0);
    pp[3] = B.m_v;
    pp[4] = B.mass;
    pp[5] = B.ks0 * ctx->stiff_scale;
    pp[6] = B.kv_default ? 1.0 : 0.0;
    for (int k = 0; k < 9; k++) param[8 * (size_t)nb + 9 * b + k] = B.Ibody[k];
    v0 += B.nv;
    f0 += B.nf;
    e0 += (int)B.l0.size();
  }
  ctx->nv = v0;
  ctx->nf = f0;
  ctx->ne = e0;
  ctx->nh = e0;
  ctx->nsoft_v = (int)soft.size();
  // vertex incidence tables, slot-major [VT_SLOTS][nv]
  std::vector<int32_t> vtab((size_t)VT_SLOTS * v0, 0);
  // and the slot each (element, vertex role) writes its force into
  std::vector<int> ne_cnt(v0, 0), nh_cnt(v0, 0), nf_cnt(v0, 0);
  std::vector<int32_t> sl_edge(2 * (size_t)e0), sl_hinge(4 * (size_t)e0), sl_face(3 * (size_t)f0);
  auto put = [&](int v, int slot0, int width, std::vector<int>& cnt, int32_t val, int32_t& slot) {
    if (cnt[v] >= width) return false;
    slot = slot0 + cnt[v]++;
    vtab[(size_t)slot * v0 + v] = val;
    return true;
  };
  for (int e = 0; e < e0; e++) {
    if (!put(edges[2 * e], 0, VT_E, ne_cnt, e + 1, sl_edge[2 * e]) ||
        !put(edges[2 * e + 1], 0, VT_E, ne_cnt, -(e + 1), sl_edge[2 * e + 1]))
      return fail(ctx, LBM_E_INVAL, "vertex valence above 10");
  }
  for (int h = 0; h < e0; h++)
    for (int r = 0; r < 4; r++)
      if (!put(hinges[4 * h + r], VT_E, VT_H, nh_cnt, 4 * h + r + 1, sl_hinge[4 * h + r]))
        return fail(ctx, LBM_E_INVAL, "vertex in more than 20 hinges");
  for (int f = 0; f < f0; f++)
    for (int r = 0; r < 3; r++)
      if (!put(faces[3 * f + r], VT_E + VT_H, VT_F, nf_cnt, f + 1, sl_face[3 * f + r]))
        return fail(ctx, LBM_E_INVAL, "vertex valence above 10");
  auto up = [&](auto** p, const auto& v) -> hipError_t {
    hipError_t e = upload(p, v);
    ctx->bod_alloc.push_back((void*)*p);
    return e;
  };
  BodyArgs B{};
  B.nbody = nb;
  B.nv = v0;
  B.nf = f0;
  B.ne = e0;
  B.nh = e0;
  B.nsoft_v = ctx->nsoft_v;
  int32_t *d_soft, *d_faces, *d_fb, *d_vb, *d_edges, *d_hinges, *d_bf0, *d_bnf, *d_bv0,
      *d_bnv, *d_be0, *d_bne, *d_brig, *d_bfix;
  double *d_l0, *d_kl, *d_th0, *d_kb, *d_param, *d_Xbody;
  CHK(up(&d_soft, soft));
  CHK(up(&d_faces, faces));
  CHK(up(&d_fb, face_body));
  CHK(up(&d_vb, vert_body));
  CHK(up(&d_edges, edges));
  CHK(up(&d_hinges, hinges));
  CHK(up(&d_bf0, bf0));
  CHK(up(&d_bnf, bnf));
  CHK(up(&d_bv0, bv0));
  CHK(up(&d_bnv, bnv));
  CHK(up(&d_be0, be0));
  CHK(up(&d_bne, bne));
  CHK(up(&d_brig, brig));
  CHK(up(&d_bfix, bfix));
  CHK(up(&d_l0, l0));
  CHK(up(&d_kl, kl));
  CHK(up(&d_th0, th0));
  CHK(up(&d_kb, kb));
  CHK(up(&d_param, param));
  CHK(up(&d_Xbody, Xbody));
  // dynamic state
  std::vector<double> X0(Xc), X1(Xp);
  CHK(up(&ctx->X[cur], X0));
  CHK(up(&ctx->X[cur ^ 1], X1));
  CHK(up(&ctx->Vel, Vl));
  CHK(up(&ctx->b_rig, rig));
  // diagnostics blocks: one thread per face, vertex and edge of a body
  std::vector<int32_t> dblk0(1, 0), dblk_body;
  for (int b = 0; b < nb; b++) {
    const HostBody& HB = ctx->bodies[b];
    const int items = std::max(HB.nf, std::max(HB.nv, (int)HB.l0.size()));
    const int nblk = (items + 255) / 256;
    for (int k = 0; k < nblk; k++) dblk_body.push_back(b);
    dblk0.push_back(dblk0.back() + nblk);
  }
  std::vector<double> diag(16 * (size_t)nb, 0.0), dpart(12 * dblk_body.size(), 0.0);
  // first reference centre of each body's bounding sphere: its vertex mean
  for (int b = 0; b < nb; b++)
    for (int k = 0; k < 3; k++) {
      double m = 0.0;
      for (int v = bv0[b]; v < bv0[b] + bnv[b]; v++) m += Xc[3 * (size_t)v + k];
      diag[16 * (size_t)b + 13 + k] = m / std::max(bnv[b], 1);
    }
  CHK(up(&ctx->b_diag, diag));
  double* d_dpart;
  int32_t *d_dblk0, *d_dblkb;
  CHK(up(&d_dpart, dpart));
  CHK(up(&d_dblk0, dblk0));
  CHK(up(&d_dblkb, dblk_body));
  B.diag_part = d_dpart;
  B.b_dblk0 = d_dblk0;
  B.dblk_body = d_dblkb;
  B.n_diag_blocks = (int)dblk_body.size();
  // marker chunks: CHUNK_CAP per 64 faces of each body, plain runs of 64 in
  // face order until k_bin_faces cuts them
  std::vector<int32_t> bch0(1, 0), ch_s0, ch_n;
  for (int b = 0; b < nb; b++) {
    const int nrun = (bnf[b] + MARKERS_PER_BLOCK - 1) / MARKERS_PER_BLOCK;
    for (int c = 0; c < CHUNK_CAP * nrun; c++) {
      ch_s0.push_back(bf0[b] + std::min(c, nrun) * MARKERS_PER_BLOCK);
      ch_n.push_back(c < nrun ? std::min(MARKERS_PER_BLOCK, bnf[b] - c * MARKERS_PER_BLOCK) : 0);
    }
    bch0.push_back(bch0.back() + CHUNK_CAP * nrun);
  }
  B.n_marker_blocks = bch0.back();
  B.n_elem_blocks = (2 * e0 + 255) / 256;
  // one flag per thread: blocks of 256 threads cover 256 tiles each
  B.n_clear_blocks = (int)std::min<long long>(64, ((ctx->g.Np >> TILE_SHIFT) + 1 + 255) / 256);
  std::vector<double> zf(3 * (size_t)f0, 0.0), zv(3 * (size_t)v0, 0.0);
  double *d_cen, *d_fext, *d_u0v, *d_fslot;
  int32_t *d_sle, *d_slh, *d_slf, *d_cbox;
  CHK(up(&d_cen, zf));
  CHK(up(&d_cbox, std::vector<int32_t>(6 * (size_t)B.n_marker_blocks, 0)));
  CHK(up(&d_fext, zf));
  CHK(up(&d_u0v, zv));
  // slots nobody writes stay zero
  CHK(up(&d_fslot, std::vector<double>((size_t)VT_SLOTS * 3 * v0, 0.0)));
  CHK(up(&d_sle, sl_edge));
  CHK(up(&d_slh, sl_hinge));
  CHK(up(&d_slf, sl_face));
  B.f_slot = d_fslot;
  B.sl_edge = d_sle;
  B.sl_hinge = d_slh;
  B.sl_face = d_slf;
  B.soft_vlist = d_soft;
  B.Vel = ctx->Vel;
  B.faces = d_faces;
  B.face_body = d_fb;
  B.vert_body = d_vb;
  B.edges = d_edges;
  B.l0 = d_l0;
  B.kl = d_kl;
  B.hinges = d_hinges;
  B.theta0 = d_th0;
  B.kb = d_kb;
  B.b_face0 = d_bf0;
  B.b_nf = d_bnf;
  B.b_vert0 = d_bv0;
  B.b_nv = d_bnv;
  B.b_edge0 = d_be0;
  B.b_ne = d_bne;
  B.b_rigid = d_brig;
  B.b_fixed = d_bfix;
  B.b_param = d_param;
  B.b_rig = ctx->b_rig;
  B.Xbody = d_Xbody;
  B.b_diag = ctx->b_diag;
  // marker order: identity until k_bin_faces runs (below, and every
  // BIN_EVERY steps); sort space in global memory for bodies above the LDS
  // capacity of the binning kernel
  std::vector<int32_t> ident(f0), slot_f(4 * (size_t)f0);
  for (int f = 0; f < f0; f++) {
    ident[f] = f;
    for (int k = 0; k < 3; k++) slot_f[4 * (size_t)f + k] = faces[3 * (size_t)f + k];
    slot_f[4 * (size_t)f + 3] = face_body[f];
  }
  std::vector<long long> key0(nb, 0);
  long long nkeys = 0;
  for (int b = 0; b < nb; b++) {
    long long n2 = 1;
    while (n2 < bnf[b]) n2 <<= 1;
    key0[b] = nkeys;
    if (n2 > BIN_LDS_KEYS) nkeys += n2;
  }
  int32_t* d_perm;
  long long* d_key0;
  unsigned long long* d_bkeys;
  CHK(up(&d_perm, ident));
  int32_t* d_slotf;
  CHK(up(&d_slotf, slot_f));
  CHK(up(&d_key0, key0));
  CHK(up(&d_bkeys, std::vector<unsigned long long>(std::max<long long>(nkeys, 1), 0ull)));
  int32_t *d_chs0, *d_chn, *d_bch0;
  CHK(up(&d_chs0, ch_s0));
  CHK(up(&d_chn, ch_n));
  CHK(up(&d_bch0, bch0));
  B.chunk_s0 = d_chs0;
  B.chunk_n = d_chn;
  B.b_chunk0 = d_bch0;
  if (ctx->spread_two_pass) {
    long long* d_stage;
    int32_t* d_snode;
    CHK(up(&d_stage, std::vector<long long>((size_t)B.n_marker_blocks * BOX_CELLS * 3, 0)));
    CHK(up(&d_snode, std::vector<int32_t>((size_t)B.n_marker_blocks * BOX_CELLS, -1)));
    B.stage = d_stage;
    B.stage_node = d_snode;
  }
  B.perm = d_perm;
  B.slot_f = d_slotf;
  B.b_key0 = d_key0;
  B.bin_keys = d_bkeys;
  B.centroid = d_cen;
  B.fext = d_fext;
  B.chunk_box = d_cbox;
  B.u0v = d_u0v;
  B.nu = (ctx->tau - 0.5) / 3.0;
  B.umax = ctx->umax;
  for (int p = 0; p < 2; p++) {
    ctx->bargs[p] = B;
    ctx->bargs[p].Xcur = ctx->X[p];
    ctx->bargs[p].Xnext = ctx->X[p ^ 1];
  }
  // force buffers (once)
  if (!ctx->fx[0]) {
    const size_t fxb = 3 * (size_t)ctx->g.Np * sizeof(long long);
    for (int p = 0; p < 2; p++) {
      CHK(hipMalloc(&ctx->fx[p], fxb));
      CHK(hipMemset(ctx->fx[p], 0, fxb));
      CHK(hipMalloc(&ctx->tf[p], ctx->ntiles));
      CHK(hipMemset(ctx->tf[p], 0, ctx->ntiles));
    }
    const size_t macb = 4 * (size_t)ctx->g.Np * (ctx->prec == 0 ? sizeof(double) : sizeof(float));
    CHK(hipMalloc(&ctx->mac, macb));
    CHK(hipMemset(ctx->mac, 0, macb));
  }
  // marker order of the current positions, and their diagnostics
  CHK(launch_bin_faces(ctx->bargs[cur], ctx->stream));
  ctx->bin_enq = ctx->enq;
  CHK(launch_check(ctx->bargs[cur], ctx->X[0], ctx->X[1], ctx->flags, counter(ctx, 3), ctx->stream));
  CHK(hipStreamSynchronize(ctx->stream));
  return LBM_OK;
}

extern "C" lbm_status lbm_add_body(lbm_ctx* ctx, const lbm_body_desc* bd, int32_t* body_id) {
  if (!ctx || !bd) return LBM_E_INVAL;
  if (ctx->broken) return LBM_E_STATE;
  if (bd->nv < 4 || bd->nf < 4 || !bd->x || !bd->faces) return fail(ctx, LBM_E_INVAL, "mesh too small");
  HostBody B;
  B.nv = bd->nv;
  B.nf = bd->nf;
  B.rigid = bd->rigid || bd->fixed;
  B.fixed = bd->fixed ? 1 : 0;
  B.x0.assign(bd->x, bd->x + 3 * (size_t)bd->nv);
  B.faces.assign(bd->faces, bd->faces + 3 * (size_t)bd->nf);
  for (int k = 0; k < 3 * bd->nf; k++)
    if (B.faces[k] < 0 || B.faces[k] >= bd->nv) return fail(ctx, LBM_E_INVAL, "face index out of range");
  // canonical face order: each face turned to start at its smallest vertex
  // (orientation kept), the faces sorted by their vertex triples, so that no
  // sum or table below depends on the order or rotation the caller chose
  {
    std::vector<std::array<int, 3>> fl((size_t)bd->nf);
    for (int f = 0; f < bd->nf; f++) {
      int a = B.faces[3 * f], b = B.faces[3 * f + 1], c = B.faces[3 * f + 2];
      if (b < a && b < c) fl[f] = {b, c, a};
      else if (c < a && c < b) fl[f] = {c, a, b};
      else fl[f] = {a, b, c};
    }
    std::sort(fl.begin(), fl.end());
    for (int f = 0; f < bd->nf; f++)
      for (int k = 0; k < 3; k++) B.faces[3 * f + k] = fl[f][k];
  }
  // closed, consistently oriented: each directed edge once, with its reverse
  std::map<std::pair<int, int>, int> dir_edge;  // (a, b) -> face
  for (int f = 0; f < bd->nf; f++)
    for (int k = 0; k < 3; k++) {
      const int a = B.faces[3 * f + k], b = B.faces[3 * f + (k + 1) % 3];
      if (a == b) return fail(ctx, LBM_E_INVAL, "degenerate face");
      if (!dir_edge.emplace(std::make_pair(a, b), f).second)
        return fail(ctx, LBM_E_INVAL, "mesh is not consistently oriented");
    }
  std::vector<double> Af(bd->nf);
  for (int f = 0; f < bd->nf; f++) Af[f] = tri_area(bd->x, B.faces[3 * f], B.faces[3 * f + 1], B.faces[3 * f + 2]);
  double V0 = 0.0, S0 = 0.0;
  for (int f = 0; f < bd->nf; f++) {
    const double *a = bd->x + 3 * B.faces[3 * f], *b = bd->x + 3 * B.faces[3 * f + 1], *c = bd->x + 3 * B.faces[3 * f + 2];
    double bc[3];
    cross(b, c, bc);
    V0 += (a[0] * bc[0] + a[1] * bc[1] + a[2] * bc[2]) / 6.0;
    S0 += Af[f];
  }
  if (!(V0 > 0.0)) return fail(ctx, LBM_E_INVAL, "mesh encloses no volume (inward faces?)");
  const double nu = (ctx->tau - 0.5) / 3.0;
  B.ks0 = bd->ca > 0.0 ? nu * bd->u_ref / bd->ca : 0.0;
  B.kv = bd->kv > 0.0 ? bd->kv : 10.0 * B.ks0 / bd->r_ref;
  B.kv_default = !(bd->kv > 0.0);
  B.V0 = V0;
  B.S0 = S0;
  B.mass = bd->rho_ratio * V0;
  B.m_v = B.mass / bd->nv;
  for (const auto& kv : dir_edge) {
    const int a = kv.first.first, b = kv.first.second;
    auto it = dir_edge.find(std::make_pair(b, a));
    if (it == dir_edge.end()) return fail(ctx, LBM_E_INVAL, "mesh is not closed");
    if (a > b) continue;  // each undirected edge once, oriented as in its first face
    const int f1 = kv.second, f2 = it->second;
    int c = -1, d = -1;
    for (int k = 0; k < 3; k++) {
      if (B.faces[3 * f1 + k] != a && B.faces[3 * f1 + k] != b) c = B.faces[3 * f1 + k];
      if (B.faces[3 * f2 + k] != a && B.faces[3 * f2 + k] != b) d = B.faces[3 * f2 + k];
    }
    B.edges.push_back(a);
    B.edges.push_back(b);
    const double* xa = bd->x + 3 * a;
    const double* xb = bd->x + 3 * b;
    const double l = std::sqrt((xa[0] - xb[0]) * (xa[0] - xb[0]) + (xa[1] - xb[1]) * (xa[1] - xb[1]) +
                               (xa[2] - xb[2]) * (xa[2] - xb[2]));
    B.l0.push_back(l);
    // k_s,l = k_s0 T (A1 + A2) / l0^2 with T = 1
    const double k = B.ks0 * (Af[f1] + Af[f2]) / (l * l);
    B.kl.push_back(k);
    const int h[4] = {a, b, c, d};
    for (int r = 0; r < 4; r++) B.hinges.push_back(h[r]);
    B.theta0.push_back(dihedral_host(bd->x, h));
    B.kb.push_back(bd->eb * k * bd->r_ref * bd->r_ref);
  }
  // centre of mass and inertia of the enclosed uniform solid (rigid bodies)
  {
    double vol = 0.0, cm[3] = {0, 0, 0}, C[9] = {0};
    for (int f = 0; f < bd->nf; f++) {
      const double* P[3] = {bd->x + 3 * B.faces[3 * f], bd->x + 3 * B.faces[3 * f + 1],
                            bd->x + 3 * B.faces[3 * f + 2]};
      double bc[3];
      cross(P[1], P[2], bc);
      const double vt = (P[0][0] * bc[0] + P[0][1] * bc[1] + P[0][2] * bc[2]) / 6.0;
      vol += vt;
      for (int a = 0; a < 3; a++) cm[a] += vt * (P[0][a] + P[1][a] + P[2][a]) / 4.0;
      for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
          double sp = 0, si = 0, sj = 0;
          for (int k = 0; k < 3; k++) {
            sp += P[k][i] * P[k][j];
            si += P[k][i];
            sj += P[k][j];
          }
          C[3 * i + j] += vt / 20.0 * (sp + si * sj);
        }
    }
    for (int a = 0; a < 3; a++) cm[a] /= vol;
    for (int i = 0; i < 3; i++)
      for (int j = 0; j < 3; j++) C[3 * i + j] -= vol * cm[i] * cm[j];
    const double tr = C[0] + C[4] + C[8];
    for (int i = 0; i < 3; i++)
      for (int j = 0; j < 3; j++) B.Ibody[3 * i + j] = bd->rho_ratio * ((i == j ? tr : 0.0) - C[3 * i + j]);
    for (int a = 0; a < 3; a++) B.cm[a] = cm[a];
    B.Xbody.resize(3 * (size_t)bd->nv);
    for (int v = 0; v < bd->nv; v++)
      for (int a = 0; a < 3; a++) B.Xbody[3 * v + a] = bd->x[3 * v + a] - cm[a];
  }
  // current dynamic state of the existing bodies
  DevFlags h;
  lbm_status st = read_flags(ctx, &h);
  if (st) return st;
  const int cur = (int)(h.steps_done & 1);
  const int nb_old = (int)ctx->bodies.size();
  std::vector<double> Xc(3 * (size_t)ctx->nv), Xp(3 * (size_t)ctx->nv), Vl(3 * (size_t)ctx->nv),
      rig(32 * (size_t)nb_old);
  if (nb_old > 0) {
    CHK(hipMemcpy(Xc.data(), ctx->X[cur], Xc.size() * 8, hipMemcpyDeviceToHost));
    CHK(hipMemcpy(Xp.data(), ctx->X[cur ^ 1], Xp.size() * 8, hipMemcpyDeviceToHost));
    CHK(hipMemcpy(Vl.data(), ctx->Vel, Vl.size() * 8, hipMemcpyDeviceToHost));
    CHK(hipMemcpy(rig.data(), ctx->b_rig, rig.size() * 8, hipMemcpyDeviceToHost));
  }
  // append the new body: x^n = x, x^{n-1} = x - v0 (soft), velocities v0
  std::vector<double> v0(3 * (size_t)bd->nv, 0.0);
  if (bd->v0 && !bd->fixed) v0.assign(bd->v0, bd->v0 + 3 * (size_t)bd->nv);
  double rs[32] = {0};
  for (int a = 0; a < 3; a++) rs[a] = B.cm[a];
  rs[15] = rs[19] = rs[23] = 1.0;
  if (B.rigid && !B.fixed && bd->v0) {
    for (int a = 0; a < 3; a++) {
      double m = 0.0;
      for (int v = 0; v < bd->nv; v++) m += v0[3 * v + a];
      rs[3 + a] = rs[6 + a] = m / bd->nv;
    }
    for (int v = 0; v < bd->nv; v++)
      for (int a = 0; a < 3; a++) v0[3 * v + a] = rs[3 + a];
  }
  for (int v = 0; v < bd->nv; v++)
    for (int a = 0; a < 3; a++) {
      Xc.push_back(bd->x[3 * v + a]);
      Xp.push_back(bd->x[3 * v + a] - (B.rigid ? 0.0 : v0[3 * v + a]));
      Vl.push_back(v0[3 * v + a]);
    }
  rig.insert(rig.end(), rs, rs + 32);
  ctx->bodies.push_back(std::move(B));
  free_graphs(ctx);
  ctx->version++;
  st = build_body_arrays(ctx, cur, Xc, Xp, Vl, rig);
  if (st) return st;
  if (body_id) *body_id = (int32_t)ctx->bodies.size() - 1;
  return LBM_OK;
}

// -------------------------------------------------------------------- step
static FluidArgs fluid_args(lbm_ctx* ctx, int p) {
  FluidArgs a{};
  a.g = ctx->g;
  a.A = ctx->f[p];
  a.B = ctx->f[p ^ 1];
  a.ncls = ctx->ncls;
  a.rec_of = ctx->rec_of;
  a.nrec = ctx->nrec;
  a.rec_node = ctx->rec_node;
  a.rec_mask = ctx->rec_mask;
  a.rec_link0 = ctx->rec_link0;
  a.rec_face = ctx->rec_face;
  a.rec_bc = ctx->rec_bc;
  a.lk_c = ctx->lk_c;
  a.rec_mb = ctx->rec_mb;
  a.nlinks = ctx->nlinks_rec;
  a.tile_list = ctx->tile_list;
  a.nbulk_blocks = ctx->nbulk_blocks;
  a.bulk_list = ctx->bulk_v == 0 ? ctx->bulk_list : nullptr;
  a.nbulk_nodes = (int)ctx->n_bulk;
  a.omega = 1.0 / ctx->tau;
  a.gx = ctx->gfx;
  a.gy = ctx->gfy;
  a.gz = ctx->gfz;
  const bool ib = ctx->nf > 0;
  a.fx = ib ? ctx->fx[p] : nullptr;
  a.tflag = ib ? ctx->tf[p] : nullptr;
  a.mac = ib ? ctx->mac : nullptr;
  a.flags = ctx->flags;
  a.rec_block = ctx->rec_block;
  a.bulk_v = ctx->bulk_v;
  a.bulk_block = ctx->bulk_block;
  return a;
}

static BodyArgs empty_body_args() {
  BodyArgs b{};
  return b;
}

// The launches of one step of parity p; if ev is given, HIP events bracket
// the fused stream-collide kernel.
// The launches of one step of parity p on stream s.  The boundary-record
// kernel runs on a second stream (fork/join with events) concurrently with
// the bulk stream-collide kernel.  If ev0/ev1 are given they bracket the
// stream-collide pair.
static hipError_t enqueue_step(lbm_ctx* ctx, int p, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1,
                               int fluid_reps = 1) {
  hipError_t e;
  FluidArgs a = fluid_args(ctx, p);
  const bool ib = ctx->nf > 0;
  if (ib) {
    const BodyArgs& b = ctx->bargs[p];
    if ((e = launch_ib_force(ctx->prec, a, b, ctx->fx[p], ctx->tf[p], ctx->fx[p ^ 1], ctx->tf[p ^ 1],
                             counter(ctx, 0), s)) != hipSuccess)
      return e;
    if (b.stage && (e = launch_spread_owner(ctx->g, b, ctx->fx[p], ctx->tf[p], ctx->flags, s)) != hipSuccess)
      return e;
  }
  if (ev0 && (e = hipEventRecord(ev0, s)) != hipSuccess) return e;
  // (fluid_reps > 1 only for timing: the phase rewrites B and the macro field
  // from the same inputs, so repeating it leaves the step unchanged)
  for (int r = 0; r < fluid_reps; r++) {
    if (ctx->fluid_merged) {
      if ((e = launch_fluid_all(ctx->prec, a, s)) != hipSuccess) return e;
    } else {
      // large grids: records on the side stream, bulk tiles on this one
      if (ctx->nrec > 0) {
        if ((e = hipEventRecord(ctx->ev_fork, s)) != hipSuccess) return e;
        if ((e = hipStreamWaitEvent(ctx->side, ctx->ev_fork, 0)) != hipSuccess) return e;
        if ((e = launch_fluid_rec(ctx->prec, a, ctx->side)) != hipSuccess) return e;
        if ((e = hipEventRecord(ctx->ev_join, ctx->side)) != hipSuccess) return e;
      }
      if ((e = launch_fluid_bulk(ctx->prec, a, s)) != hipSuccess) return e;
      if (ctx->nrec > 0 && (e = hipStreamWaitEvent(s, ctx->ev_join, 0)) != hipSuccess) return e;
    }
  }
  if (ev1 && (e = hipEventRecord(ev1, s)) != hipSuccess) return e;
  if (ib) {
    const BodyArgs& b = ctx->bargs[p];
    if ((e = launch_mls_post(ctx->prec, a, b, ctx->fx[p ^ 1], ctx->tf[p ^ 1], s)) != hipSuccess) return e;
    // a few tens of blocks close the step in their last one; more: k_close
    const bool fold = body_post_blocks(b) <= 128;
    if ((e = launch_body_post(b, ctx->flags, fold ? counter(ctx, 1) : nullptr, s)) != hipSuccess) return e;
    if (!fold && (e = launch_close(ctx->flags, s)) != hipSuccess) return e;
  } else {
    if ((e = launch_close(ctx->flags, s)) != hipSuccess) return e;
  }
  return hipSuccess;
}

// Graphs: one step of each parity, and a chunk of GRAPH_CHUNK steps (even,
// starting at parity 0) so that the launch gap between graphs is paid once
// per chunk.
static const int GRAPH_CHUNK = 16;
// Steps between re-sorts of the marker order (between graph launches; the
// faces of a membrane patch stay neighbours as it deforms, so the order
// only needs refreshing now and then)
static const long long BIN_EVERY = 512;

static lbm_status build_graphs(lbm_ctx* ctx) {
  free_graphs(ctx);
  for (int k = 0; k < 3; k++) {
    hipGraph_t g;
    CHK(hipStreamBeginCapture(ctx->cap, hipStreamCaptureModeThreadLocal));
    hipError_t e = hipSuccess;
    if (k < 2) e = enqueue_step(ctx, k, ctx->cap, nullptr, nullptr);
    else
      for (int q = 0; q < GRAPH_CHUNK && e == hipSuccess; q++) e = enqueue_step(ctx, q & 1, ctx->cap, nullptr, nullptr);
    hipError_t e2 = hipStreamEndCapture(ctx->cap, &g);
    CHK(e);
    CHK(e2);
    CHK(hipGraphInstantiate(&ctx->gexec[k], g, nullptr, nullptr, 0));
    CHK(hipGraphDestroy(g));
  }
  ctx->graph_valid = true;
  return LBM_OK;
}

extern "C" lbm_status lbm_step(lbm_ctx* ctx, int32_t n) {
  if (!ctx || n < 0) return LBM_E_INVAL;
  if (ctx->broken) return LBM_E_STATE;
  if (ctx->use_graph && !ctx->graph_valid) {
    lbm_status st = build_graphs(ctx);
    if (st) return st;
  }
  int32_t k = 0;
  while (k < n) {
    const int p = (int)(ctx->enq & 1);
    if (!ctx->bodies.empty() && ctx->enq - ctx->bin_enq >= BIN_EVERY) {
      CHK(launch_bin_faces(ctx->bargs[p], ctx->stream));
      ctx->bin_enq = ctx->enq;
    }
    if (ctx->use_graph && p == 0 && n - k >= GRAPH_CHUNK) {
      CHK(hipGraphLaunch(ctx->gexec[2], ctx->stream));
      ctx->enq += GRAPH_CHUNK;
      k += GRAPH_CHUNK;
      continue;
    }
    if (ctx->use_graph) CHK(hipGraphLaunch(ctx->gexec[p], ctx->stream));
    else CHK(enqueue_step(ctx, p, ctx->stream, nullptr, nullptr));
    ctx->enq++;
    k++;
  }
  return LBM_OK;
}

extern "C" lbm_status lbm_set_graph(lbm_ctx* ctx, int32_t enable) {
  if (!ctx) return LBM_E_INVAL;
  ctx->use_graph = enable != 0;
  return LBM_OK;
}

extern "C" lbm_status lbm_sync(lbm_ctx* ctx) {
  if (!ctx) return LBM_E_INVAL;
  if (ctx->broken) return LBM_E_STATE;
  // damage or non-finite positions of the last completed step
  if (ctx->nf > 0)
    CHK(launch_check(ctx->bargs[0], ctx->X[0], ctx->X[1], ctx->flags, counter(ctx, 3), ctx->stream));
  DevFlags h;
  lbm_status st = read_flags(ctx, &h);
  if (st) return st;
  // the host's step counter follows the device once it has stopped
  if (h.stop & ST_DAMAGED) return fail(ctx, LBM_E_DAMAGED, "a membrane link reached twice its rest length");
  if (h.stop & ST_UNSTABLE)
    return fail(ctx, LBM_E_UNSTABLE, h.overflow ? "a spread force contribution exceeded +-1 (IB unstable)"
                                                : "|u| > 0.3 or NaN");
  return LBM_OK;
}

// Launches of the fluid phase per timed step: back to back on one stream, so
// that the span between the events is kernel time, not launch latency.
static const int TIMING_REPS = 8;

extern "C" lbm_status lbm_time_fluid_kernel(lbm_ctx* ctx, int32_t n, double* avg_ms) {
  if (!ctx || n <= 0 || !avg_ms) return LBM_E_INVAL;
  if (ctx->broken) return LBM_E_STATE;
  std::vector<hipEvent_t> e0(n), e1(n);
  for (int k = 0; k < n; k++) {
    CHK(hipEventCreate(&e0[k]));
    CHK(hipEventCreate(&e1[k]));
  }
  for (int k = 0; k < n; k++) {
    const int p = (int)(ctx->enq & 1);
    CHK(enqueue_step(ctx, p, ctx->stream, e0[k], e1[k], TIMING_REPS));
    ctx->enq++;
  }
  CHK(hipStreamSynchronize(ctx->stream));
  double tot = 0.0;
  for (int k = 0; k < n; k++) {
    float ms = 0.f;
    CHK(hipEventElapsedTime(&ms, e0[k], e1[k]));
    tot += ms;
    CHK(hipEventDestroy(e0[k]));
    CHK(hipEventDestroy(e1[k]));
  }
  *avg_ms = tot / n / TIMING_REPS;
  return LBM_OK;
}

extern "C" lbm_status lbm_set_launch_shape(lbm_ctx* ctx, int32_t bulk_v, int32_t block) {
  if (!ctx) return LBM_E_INVAL;
  if (ctx->broken) return LBM_E_STATE;
  if (!shape_ok(ctx->prec, bulk_v, block)) return fail(ctx, LBM_E_INVAL, "unsupported launch shape");
  if (bulk_v == ctx->bulk_v && block == ctx->bulk_block) return LBM_OK;
  // the old tile list may still be read by enqueued work
  CHK(hipStreamSynchronize(ctx->stream));
  free_graphs(ctx);
  if (bulk_v == 0) {
    CHK(ensure_bulk_list(ctx));
    ctx->nbulk_blocks = bulk_blocks(ctx, 0, block, 0);
  } else {
    std::vector<int32_t> tiles = bulk_tiles(ctx->g, ctx->ncls_h, block, bulk_v);
    int32_t* old = ctx->tile_list;
    ctx->tile_list = nullptr;
    CHK(upload(&ctx->tile_list, tiles));
    if (old) CHK(hipFree(old));
    ctx->nbulk_blocks = (int)tiles.size();
  }
  ctx->bulk_v = bulk_v;
  ctx->bulk_block = block;
  if (ctx->fluid_merged) ctx->rec_block = block;
  ctx->version++;
  return LBM_OK;
}

// ------------------------------------------------------------------ batches
struct lbm_batch {
  std::vector<lbm_ctx*> ctx;
  hipStream_t stream = nullptr;
  hipStream_t cap = nullptr;
  int prec = 0;
  std::string err;
  bool broken = false;
  // launch shape of the fluid phase
  int V = 1, block = 64, mode = 0, per_xcd = 0;
  // device tables for the two step parities, and the phase maps
  BatchItem* items = nullptr;  // [2][n]
  int2* maps = nullptr;
  int n_ib = 0, n_all = 0, n_rec = 0, n_bulk = 0, n_mls = 0, n_body = 0;
  int2 *m_ib = nullptr, *m_all = nullptr, *m_rec = nullptr, *m_bulk = nullptr, *m_mls = nullptr,
       *m_body = nullptr;
  std::vector<uint64_t> ver;  // context versions the tables were built for
  std::vector<int> par;       // context parity relative to the batch's at that time
  bool tables_valid = false;
  bool use_graph = true;
  bool graph_valid = false;
  hipGraphExec_t gexec[3] = {nullptr, nullptr, nullptr};
  int64_t enq = 0;
};

#define CHKB(expr)                                                                   \
  do {                                                                               \
    hipError_t e_ = (expr);                                                          \
    if (e_ != hipSuccess) {                                                          \
      b->broken = true;                                                              \
      b->err = std::string("HIP error: ") + hipGetErrorString(e_) + " at " + #expr;  \
      return LBM_E_HIP;                                                              \
    }                                                                                \
  } while (0)

static lbm_status bfail(lbm_batch* b, lbm_status st, const std::string& msg) {
  b->err = msg;
  return st;
}

static void batch_free_graphs(lbm_batch* b) {
  for (int k = 0; k < 3; k++)
    if (b->gexec[k]) {
      (void)hipGraphExecDestroy(b->gexec[k]);
      b->gexec[k] = nullptr;
    }
  b->graph_valid = false;
}

// Physical block g of a one-unit-per-block launch takes logical unit
// xcd_order(g, n): consecutive units land on the same XCD (blocks are
// dispatched round-robin over the 8 XCDs).
static int xcd_order(int g, int n) {
  const int full = n & ~7;
  if (g >= full) return g;
  return (g & 7) * (full >> 3) + (g >> 3);
}

static lbm_status batch_build_tables(lbm_batch* b) {
  const int n = (int)b->ctx.size();
  std::vector<BatchItem> items(2 * (size_t)n);
  std::vector<int2> ib, all, rec, bulk, mls, body;
  b->ver.assign(n, 0);
  b->par.assign(n, 0);
  for (int i = 0; i < n; i++) {
    lbm_ctx* c = b->ctx[i];
    b->ver[i] = c->version;
    b->par[i] = (int)((c->enq - b->enq) & 1);
    const int nrb = c->nrec > 0 ? (c->nrec + b->block - 1) / b->block : 0;
    for (int q = 0; q < 2; q++) {
      const int p = (q + b->par[i]) & 1;
      BatchItem& it = items[(size_t)q * n + i];
      it.a = fluid_args(c, p);
      if (c->nf > 0) {
        it.b = c->bargs[p];
        it.b.stage = nullptr;  // the batched forcing spreads in one pass
        it.b.stage_node = nullptr;
        it.fxc = c->fx[p];
        it.tfc = c->tf[p];
        it.fxp = c->fx[p ^ 1];
        it.tfp = c->tf[p ^ 1];
      }
      it.counter = counter(c, 0);
      it.nrb = nrb;
    }
    for (int j = 0; j < nrb; j++) {
      all.push_back(make_int2(i, j));
      rec.push_back(make_int2(i, j));
    }
    for (int j = 0; j < c->nbulk_blocks; j++) {
      all.push_back(make_int2(i, nrb + j));
      bulk.push_back(make_int2(i, j));
    }
    if (c->nf > 0) {
      const BodyArgs& B = c->bargs[0];
      const int nib = B.n_marker_blocks + B.n_elem_blocks + B.n_diag_blocks;
      for (int j = 0; j < nib; j++) ib.push_back(make_int2(i, j));
      // probe / vertex-velocity blocks, then the previous step's tile clears
      const long long waves = (long long)(B.nf + MLS_FACES_PER_WAVE - 1) / MLS_FACES_PER_WAVE +
                              (B.nsoft_v + MLS_VERTS_PER_WAVE - 1) / MLS_VERTS_PER_WAVE;
      const int nm = (int)((waves * 64 + 255) / 256) + B.n_clear_blocks;
      for (int j = 0; j < nm; j++) mls.push_back(make_int2(i, j));
      const int nbp = B.nbody + (B.nsoft_v + 63) / 64;
      for (int j = 0; j < nbp; j++) body.push_back(make_int2(i, j));
    }
  }
  auto order = [](std::vector<int2>& v) {
    std::vector<int2> o(v.size());
    for (size_t g = 0; g < v.size(); g++) o[g] = v[xcd_order((int)g, (int)v.size())];
    v.swap(o);
  };
  order(rec);
  if (b->per_xcd == 0) {  // the persistent forms walk the units in logical order
    order(all);
    order(bulk);
  }
  // upload (previous tables may still be read by enqueued work)
  CHKB(hipStreamSynchronize(b->stream));
  batch_free_graphs(b);
  if (b->items) CHKB(hipFree(b->items));
  if (b->maps) CHKB(hipFree(b->maps));
  b->items = nullptr;
  b->maps = nullptr;
  CHKB(hipMalloc(&b->items, sizeof(BatchItem) * items.size()));
  CHKB(hipMemcpy(b->items, items.data(), sizeof(BatchItem) * items.size(), hipMemcpyHostToDevice));
  std::vector<int2> m;
  const std::vector<int2>* parts[6] = {&ib, &all, &rec, &bulk, &mls, &body};
  for (auto* v : parts) m.insert(m.end(), v->begin(), v->end());
  CHKB(hipMalloc(&b->maps, sizeof(int2) * std::max<size_t>(m.size(), 1)));
  if (!m.empty()) CHKB(hipMemcpy(b->maps, m.data(), sizeof(int2) * m.size(), hipMemcpyHostToDevice));
  int2* base = b->maps;
  b->m_ib = base;   base += ib.size();
  b->m_all = base;  base += all.size();
  b->m_rec = base;  base += rec.size();
  b->m_bulk = base; base += bulk.size();
  b->m_mls = base;  base += mls.size();
  b->m_body = base;
  b->n_ib = (int)ib.size();
  b->n_all = (int)all.size();
  b->n_rec = (int)rec.size();
  b->n_bulk = (int)bulk.size();
  b->n_mls = (int)mls.size();
  b->n_body = (int)body.size();
  b->tables_valid = true;
  return LBM_OK;
}

static BatchFluid batch_fluid(const lbm_batch* b) {
  BatchFluid f{};
  f.V = b->V;
  f.block = b->block;
  f.mode = b->mode;
  f.per_xcd = b->per_xcd;
  f.map_all = b->m_all;
  f.n_all = b->n_all;
  f.map_rec = b->m_rec;
  f.n_rec = b->n_rec;
  f.map_bulk = b->m_bulk;
  f.n_bulk = b->n_bulk;
  return f;
}

// One coupled step of every instance at batch parity q on stream s.
static hipError_t batch_enqueue(lbm_batch* b, int q, hipStream_t s) {
  hipError_t e;
  const BatchItem* it = b->items + (size_t)q * b->ctx.size();
  if ((e = launch_batch_ib_force(b->prec, it, b->m_ib, b->n_ib, s)) != hipSuccess) return e;
  if ((e = launch_batch_fluid(b->prec, batch_fluid(b), it, s)) != hipSuccess) return e;
  if ((e = launch_batch_mls_post(b->prec, it, b->m_mls, b->n_mls, s)) != hipSuccess) return e;
  if ((e = launch_batch_body_post(it, b->m_body, b->n_body, s)) != hipSuccess) return e;
  return launch_batch_close(it, (int)b->ctx.size(), s);
}

static lbm_status batch_ready(lbm_batch* b) {
  if (b->broken) return LBM_E_STATE;
  bool stale = !b->tables_valid;
  for (size_t i = 0; i < b->ctx.size(); i++) {
    lbm_ctx* c = b->ctx[i];
    if (c->broken) return bfail(b, LBM_E_STATE, "a context of the batch has failed");
    // a context given another launch shape on its own gets the batch's back:
    // its bulk tiles must match the batched kernels' block and V
    if (c->bulk_v != b->V || c->bulk_block != b->block) {
      lbm_status st = lbm_set_launch_shape(c, b->V, b->block);
      if (st) return bfail(b, st, std::string("launch shape: ") + c->err);
    }
    if (!stale && (c->version != b->ver[i] || (int)((c->enq - b->enq) & 1) != b->par[i])) stale = true;
  }
  if (stale) return batch_build_tables(b);
  return LBM_OK;
}

static lbm_status batch_build_graphs(lbm_batch* b) {
  batch_free_graphs(b);
  for (int k = 0; k < 3; k++) {
    hipGraph_t g;
    CHKB(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
    hipError_t e = hipSuccess;
    if (k < 2) e = batch_enqueue(b, k, b->cap);
    else
      for (int q = 0; q < GRAPH_CHUNK && e == hipSuccess; q++) e = batch_enqueue(b, q & 1, b->cap);
    hipError_t e2 = hipStreamEndCapture(b->cap, &g);
    CHKB(e);
    CHKB(e2);
    CHKB(hipGraphInstantiate(&b->gexec[k], g, nullptr, nullptr, 0));
    CHKB(hipGraphDestroy(g));
  }
  b->graph_valid = true;
  return LBM_OK;
}

extern "C" lbm_status lbm_batch_create(lbm_ctx* const* ctxs, int32_t n, lbm_batch** out) {
  if (!out) return LBM_E_INVAL;
  *out = nullptr;
  if (!ctxs || n < 1) return LBM_E_INVAL;
  lbm_batch* b = new lbm_batch();
  *out = b;  // handed back so that the caller can read the message
  b->ctx.assign(ctxs, ctxs + n);
  for (int i = 0; i < n; i++)
    if (!ctxs[i]) return bfail(b, LBM_E_INVAL, "null context");
  for (int i = 0; i < n; i++)
    for (int j = 0; j < i; j++)
      if (ctxs[i] == ctxs[j]) return bfail(b, LBM_E_INVAL, "a context appears twice");
  lbm_ctx* c0 = ctxs[0];
  b->stream = c0->stream;
  b->prec = c0->prec;
  for (int i = 0; i < n; i++) {
    lbm_ctx* c = ctxs[i];
    if (c->broken) return bfail(b, LBM_E_STATE, "a context has failed");
    if (c->prec != b->prec) return bfail(b, LBM_E_INVAL, "contexts of one batch share their precision");
    if (c->stream != b->stream) return bfail(b, LBM_E_INVAL, "contexts of one batch share their stream");
    if (c->g.per[0]) return bfail(b, LBM_E_UNSUPPORTED, "periodic-x contexts are not batched");
  }
  // start from the first context's launch shape (the autotuner may change it)
  b->V = c0->bulk_v;
  b->block = c0->bulk_block;
  for (int i = 0; i < n; i++) {
    lbm_status st = lbm_set_launch_shape(ctxs[i], b->V, b->block);
    if (st) return bfail(b, st, std::string("launch shape: ") + ctxs[i]->err);
  }
  CHKB(hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking));
  return batch_build_tables(b);
}

extern "C" lbm_status lbm_batch_destroy(lbm_batch* b) {
  if (!b) return LBM_OK;
  if (b->stream || b->cap) (void)hipDeviceSynchronize();
  batch_free_graphs(b);
  if (b->items) (void)hipFree(b->items);
  if (b->maps) (void)hipFree(b->maps);
  if (b->cap) (void)hipStreamDestroy(b->cap);
  delete b;
  return LBM_OK;
}

extern "C" const char* lbm_batch_last_error(const lbm_batch* b) {
  return b ? b->err.c_str() : "null batch";
}

extern "C" lbm_status lbm_batch_set_shape(lbm_batch* b, const lbm_batch_shape* sh) {
  if (!b || !sh) return LBM_E_INVAL;
  if (b->broken) return LBM_E_STATE;
  if (!shape_ok(b->prec, sh->bulk_v, sh->block) || sh->mode < 0 || sh->mode > 1 || sh->per_xcd < 0 ||
      sh->per_xcd > 1024)
    return bfail(b, LBM_E_INVAL, "unsupported batch launch shape");
  for (lbm_ctx* c : b->ctx) {
    lbm_status st = lbm_set_launch_shape(c, sh->bulk_v, sh->block);
    if (st) return bfail(b, st, std::string("launch shape: ") + c->err);
  }
  b->V = sh->bulk_v;
  b->block = sh->block;
  b->mode = sh->mode;
  b->per_xcd = sh->per_xcd;
  b->tables_valid = false;
  return batch_ready(b);
}

extern "C" lbm_status lbm_batch_get_shape(lbm_batch* b, lbm_batch_shape* sh) {
  if (!b || !sh) return LBM_E_INVAL;
  sh->bulk_v = b->V;
  sh->block = b->block;
  sh->mode = b->mode;
  sh->per_xcd = b->per_xcd;
  sh->fluid_ms = 0.0;
  return LBM_OK;
}

// Average duration of the batched fluid phase at the current step parity
// over reps launches (after two untimed ones).  The phase only rewrites the
// next populations and the macroscopic field, which the next step rewrites
// again from the same inputs, so timing it leaves the run unchanged; status
// bits it may raise are cleared afterwards.
static lbm_status batch_time_fluid(lbm_batch* b, int reps, double* ms) {
  lbm_status st = batch_ready(b);
  if (st) return st;
  const int q = (int)(b->enq & 1);
  const BatchItem* it = b->items + (size_t)q * b->ctx.size();
  const BatchFluid f = batch_fluid(b);
  hipEvent_t e0, e1;
  CHKB(hipEventCreate(&e0));
  CHKB(hipEventCreate(&e1));
  for (int k = 0; k < 2; k++) CHKB(launch_batch_fluid(b->prec, f, it, b->stream));
  CHKB(hipEventRecord(e0, b->stream));
  for (int k = 0; k < reps; k++) CHKB(launch_batch_fluid(b->prec, f, it, b->stream));
  CHKB(hipEventRecord(e1, b->stream));
  CHKB(hipEventSynchronize(e1));
  float t = 0.f;
  CHKB(hipEventElapsedTime(&t, e0, e1));
  CHKB(hipEventDestroy(e0));
  CHKB(hipEventDestroy(e1));
  for (lbm_ctx* c : b->ctx)
    CHKB(hipMemsetAsync((char*)c->flags + offsetof(DevFlags, pending), 0, sizeof(uint32_t), b->stream));
  CHKB(hipStreamSynchronize(b->stream));
  *ms = (double)t / reps;
  return LBM_OK;
}

// The autotuner: times the batched fluid phase for every launch shape this
// precision supports (V nodes per bulk thread or the list form, block size,
// merged or split records, one block per tile or persistent bulk blocks)
// and keeps the fastest.  Results go to out[0..min(max, count)) in the order tried.
extern "C" lbm_status lbm_batch_tune(lbm_batch* b, int32_t reps, lbm_batch_shape* out,
                                     int32_t max_out, int32_t* n_out) {
  if (!b || reps < 1) return LBM_E_INVAL;
  if (b->broken) return LBM_E_STATE;
  std::vector<int> Vs = b->prec == 0 ? std::vector<int>{0, 1, 2}
                                     : (b->prec == 1 ? std::vector<int>{0, 1, 2, 4} : std::vector<int>{0, 2, 4, 8});
  std::vector<lbm_batch_shape> cand;
  for (int V : Vs)
    for (int block : {64, 128, 256}) {
      for (int mode : {0, 1}) {
        cand.push_back({V, block, mode, 0, 0.0});
        for (int px : {64, 128}) cand.push_back({V, block, mode, px, 0.0});
      }
    }
  int best = -1;
  for (size_t k = 0; k < cand.size(); k++) {
    lbm_status st = lbm_batch_set_shape(b, &cand[k]);
    if (st) return st;
    st = batch_time_fluid(b, reps, &cand[k].fluid_ms);
    if (st) return st;
    if (best < 0 || cand[k].fluid_ms < cand[best].fluid_ms) best = (int)k;
  }
  lbm_status st = lbm_batch_set_shape(b, &cand[best]);
  if (st) return st;
  if (out)
    for (int k = 0; k < std::min<int>(max_out, (int)cand.size()); k++) out[k] = cand[k];
  if (n_out) *n_out = (int32_t)cand.size();
  return LBM_OK;
}

extern "C" lbm_status lbm_batch_step(lbm_batch* b, int32_t n) {
  if (!b || n < 0) return LBM_E_INVAL;
  lbm_status st = batch_ready(b);
  if (st) return st;
  if (b->use_graph && !b->graph_valid) {
    st = batch_build_graphs(b);
    if (st) return st;
  }
  int32_t k = 0;
  while (k < n) {
    const int q = (int)(b->enq & 1);
    int steps = 1;
    if (b->use_graph && q == 0 && n - k >= GRAPH_CHUNK) {
      CHKB(hipGraphLaunch(b->gexec[2], b->stream));
      steps = GRAPH_CHUNK;
    } else if (b->use_graph) {
      CHKB(hipGraphLaunch(b->gexec[q], b->stream));
    } else {
      CHKB(batch_enqueue(b, q, b->stream));
    }
    b->enq += steps;
    for (lbm_ctx* c : b->ctx) c->enq += steps;
    k += steps;
  }
  return LBM_OK;
}

extern "C" lbm_status lbm_batch_set_graph(lbm_batch* b, int32_t enable) {
  if (!b) return LBM_E_INVAL;
  b->use_graph = enable != 0;
  return LBM_OK;
}

extern "C" lbm_status lbm_batch_time_fluid(lbm_batch* b, int32_t reps, double* avg_ms) {
  if (!b || reps < 1 || !avg_ms) return LBM_E_INVAL;
  return batch_time_fluid(b, reps, avg_ms);
}

extern "C" lbm_status lbm_diagnostics(lbm_ctx* ctx, double* out) {
  if (!ctx || !out) return LBM_E_INVAL;
  if (ctx->broken) return LBM_E_STATE;
  if (!ctx->gdiag) CHK(hipMalloc(&ctx->gdiag, sizeof(double) * (5 * 1024 + 8)));
  // the bodies' volume, area and stretch of the current positions
  if (ctx->nf > 0)
    CHK(launch_check(ctx->bargs[0], ctx->X[0], ctx->X[1], ctx->flags, counter(ctx, 3), ctx->stream));
  CHK(launch_diag_sums(ctx->prec, ctx->g, ctx->f[0], ctx->f[1], ctx->ncls, ctx->flags, ctx->gdiag,
                       ctx->gdiag + 5 * 1024, ctx->stream));
  double sums[5];
  const size_t nb = ctx->bodies.size();
  std::vector<double> bd(16 * nb);
  CHK(hipMemcpyAsync(sums, ctx->gdiag + 5 * 1024, sizeof sums, hipMemcpyDeviceToHost, ctx->stream));
  if (nb) CHK(hipMemcpyAsync(bd.data(), ctx->b_diag, sizeof(double) * bd.size(), hipMemcpyDeviceToHost, ctx->stream));
  CHK(hipStreamSynchronize(ctx->stream));
  out[0] = sums[0] + sums[1];  // each non-solid node holds 1 + the sum of its deviations
  out[1] = sums[2];
  out[2] = sums[3];
  out[3] = sums[4];
  for (size_t b = 0; b < nb; b++) {
    out[4 + 3 * b] = bd[16 * b];          // enclosed volume
    out[4 + 3 * b + 1] = bd[16 * b + 1];  // surface
    out[4 + 3 * b + 2] = bd[16 * b + 8];  // largest stretch l / l0
  }
  return LBM_OK;
}

// ----------------------------------------------------------------- outputs
static lbm_status fields_common(lbm_ctx* ctx, double* rho, double* u, double* pops, double* fib) {
  if (!ctx) return LBM_E_INVAL;
  if (ctx->broken) return LBM_E_STATE;
  CHK(launch_get_fields(ctx->prec, ctx->g, ctx->f[0], ctx->f[1], ctx->ncls, ctx->fx[0], ctx->fx[1],
                        ctx->tf[0], ctx->tf[1], ctx->gfx, ctx->gfy, ctx->gfz, ctx->flags, rho, u, pops,
                        fib, ctx->stream));
  return LBM_OK;
}

extern "C" lbm_status lbm_get_fields(lbm_ctx* ctx, double* d_rho, double* d_u) {
  return fields_common(ctx, d_rho, d_u, nullptr, nullptr);
}
extern "C" lbm_status lbm_get_populations(lbm_ctx* ctx, double* d_f) {
  if (!d_f) return LBM_E_INVAL;
  return fields_common(ctx, nullptr, nullptr, d_f, nullptr);
}
extern "C" lbm_status lbm_set_populations(lbm_ctx* ctx, const double* d_f) {
  if (!ctx) return LBM_E_INVAL;
  if (ctx->broken) return LBM_E_STATE;
  if (!d_f) return fail(ctx, LBM_E_INVAL, "set_populations: null input");
  CHK(launch_set_populations(ctx->prec, ctx->g, ctx->f[0], ctx->f[1], ctx->ncls, ctx->flags, d_f, ctx->stream));
  return LBM_OK;
}
extern "C" lbm_status lbm_get_force(lbm_ctx* ctx, double* d_fib) {
  if (!d_fib) return LBM_E_INVAL;
  return fields_common(ctx, nullptr, nullptr, nullptr, d_fib);
}

extern "C" lbm_status lbm_get_body(lbm_ctx* ctx, int32_t id, double* d_x, double* d_v) {
  if (!ctx) return LBM_E_INVAL;
  if (ctx->broken) return LBM_E_STATE;
  if (id < 0 || id >= (int)ctx->bodies.size()) return fail(ctx, LBM_E_INVAL, "no such body");
  DevFlags h;
  lbm_status st = read_flags(ctx, &h);
  if (st) return st;
  const int cur = (int)(h.steps_done & 1);
  int v0 = 0;
  for (int b = 0; b < id; b++) v0 += ctx->bodies[b].nv;
  const size_t bytes = 3 * sizeof(double) * ctx->bodies[id].nv;
  if (d_x) CHK(hipMemcpyAsync(d_x, ctx->X[cur] + 3 * (size_t)v0, bytes, hipMemcpyDeviceToDevice, ctx->stream));
  if (d_v) CHK(hipMemcpyAsync(d_v, ctx->Vel + 3 * (size_t)v0, bytes, hipMemcpyDeviceToDevice, ctx->stream));
  return LBM_OK;
}

extern "C" lbm_status ib_interpolate(lbm_ctx* ctx, int64_t n, const double* d_pts,
                                     const double* d_field, double* d_u) {
  if (!ctx || n < 0 || (n > 0 && (!d_pts || !d_u))) return LBM_E_INVAL;
  if (ctx->broken) return LBM_E_STATE;
  CHK(launch_interp(ctx->prec, ctx->g, ctx->f[0], ctx->f[1], ctx->ncls, ctx->fx[0], ctx->fx[1],
                    ctx->tf[0], ctx->tf[1], ctx->gfx, ctx->gfy, ctx->gfz, ctx->flags, n, d_pts,
                    d_field, d_u, ctx->stream));
  return LBM_OK;
}

extern "C" lbm_status ib_spread(lbm_ctx* ctx, int64_t n, const double* d_pts, const double* d_F,
                                const double* d_c, double* d_fib) {
  if (!ctx || n < 0 || !d_fib || (n > 0 && (!d_pts || !d_F || !d_c))) return LBM_E_INVAL;
  if (ctx->broken) return LBM_E_STATE;
  if (!ctx->fx_api) {
    const size_t b = 3 * (size_t)ctx->g.Np * sizeof(long long);
    CHK(hipMalloc(&ctx->fx_api, b));
    CHK(hipMemset(ctx->fx_api, 0, b));
    CHK(hipMalloc(&ctx->api_flags, sizeof(DevFlags)));
    CHK(hipMemset(ctx->api_flags, 0, sizeof(DevFlags)));
  }
  CHK(launch_spread_api(ctx->g, ctx->ncls, n, d_pts, d_F, d_c, ctx->fx_api, ctx->api_flags, ctx->stream));
  CHK(launch_flush_fx(ctx->g, ctx->fx_api, d_fib, ctx->stream));
  // contributions beyond the fixed-point range were dropped: report them
  DevFlags h;
  CHK(hipStreamSynchronize(ctx->stream));
  CHK(hipMemcpy(&h, ctx->api_flags, sizeof(DevFlags), hipMemcpyDeviceToHost));
  if (h.overflow) {
    CHK(hipMemset(ctx->api_flags, 0, sizeof(DevFlags)));
    return fail(ctx, LBM_E_INVAL, "ib_spread: a contribution c*phi*F exceeded +-1 (dropped)");
  }
  return LBM_OK;
}

extern "C" lbm_status ib_spread_noalloc(lbm_ctx* ctx, int64_t n, const double* d_pts, const double* d_F,
                                        const double* d_c, double* d_fib) {
  if (!ctx || n < 0 || !d_fib || (n > 0 && (!d_pts || !d_F || !d_c))) return LBM_E_INVAL;
  if (ctx->broken) return LBM_E_STATE;
  if (ctx->g.Np > NOALLOC_MAX_NODES)
    return fail(ctx, LBM_E_INVAL,
                "ib_spread_noalloc: the lattice has " + std::to_string(ctx->g.Np) +
                    " padded nodes; the scratch holds at most " + std::to_string(NOALLOC_MAX_NODES));
  long long* scr = nullptr;
  CHK(noalloc_scratch(ctx->device, &scr));
  CHK(launch_spread_noalloc(ctx->g, ctx->ncls, n, d_pts, d_F, d_c, d_fib, scr, ctx->stream));
  DevFlags h;
  CHK(hipStreamSynchronize(ctx->stream));
  CHK(hipMemcpy(&h, scr + 3 * NOALLOC_MAX_NODES, sizeof(DevFlags), hipMemcpyDeviceToHost));
  if (h.overflow) return fail(ctx, LBM_E_INVAL, "ib_spread_noalloc: a contribution c*phi*F exceeded +-1 (dropped)");
  return LBM_OK;
}

// ----------------------------------------------------------------- adjoint
// Reverse sweep over n steps from the current state with checkpoints every
// K steps: a forward pass keeps g at the start of every segment; then, from
// the last segment back, the segment's states are recomputed into a tape
// and the adjoint steps run over them in reverse.  The context's own state
// and counters are left as they are.
namespace {
struct DevArena {  // one allocation, carved in 256-byte aligned pieces
  char* base = nullptr;
  ~DevArena() {
    if (base) hipFree(base);
  }
};
}  // namespace

extern "C" lbm_status lbm_set_scales(lbm_ctx* ctx, double inlet_scale, double stiffness_scale) {
  if (!ctx) return LBM_E_INVAL;
  if (ctx->broken) return LBM_E_STATE;
  if (!std::isfinite(inlet_scale) || !(stiffness_scale > 0.0) || !std::isfinite(stiffness_scale))
    return fail(ctx, LBM_E_INVAL, "scales: a finite inlet scale and a positive stiffness scale");
  CHK(hipStreamSynchronize(ctx->stream));
  ctx->inlet_scale = inlet_scale;
  ctx->stiff_scale = stiffness_scale;
  // velocity-face records: their wall velocity times the scale
  std::vector<double> bc = ctx->rec_bc_h;
  std::vector<uint8_t> face(ctx->nrec);
  if (ctx->nrec > 0) CHK(hipMemcpy(face.data(), ctx->rec_face, ctx->nrec, hipMemcpyDeviceToHost));
  for (int r = 0; r < ctx->nrec; r++)
    if (face[r] != 0xff && !((face[r] >> 4) & 1))
      for (int c = 0; c < 3; c++) bc[(size_t)c * ctx->nrec + r] *= inlet_scale;
  if (!bc.empty()) CHK(hipMemcpy(ctx->rec_bc, bc.data(), sizeof(double) * bc.size(), hipMemcpyHostToDevice));
  // membrane moduli of every body
  if (!ctx->bodies.empty()) {
    std::vector<double> kl, kb;
    for (const HostBody& B : ctx->bodies) {
      for (double k : B.kl) kl.push_back(k * stiffness_scale);
      for (double k : B.kb) kb.push_back(k * stiffness_scale);
    }
    CHK(hipMemcpy((void*)ctx->bargs[0].kl, kl.data(), sizeof(double) * kl.size(), hipMemcpyHostToDevice));
    CHK(hipMemcpy((void*)ctx->bargs[0].kb, kb.data(), sizeof(double) * kb.size(), hipMemcpyHostToDevice));
    for (size_t b = 0; b < ctx->bodies.size(); b++) {
      const HostBody& B = ctx->bodies[b];
      const double kv = B.kv * (B.kv_default ? stiffness_scale : 1.0), ks0 = B.ks0 * stiffness_scale;
      CHK(hipMemcpy((void*)(ctx->bargs[0].b_param + 8 * b + 2), &kv, sizeof(double), hipMemcpyHostToDevice));
      CHK(hipMemcpy((void*)(ctx->bargs[0].b_param + 8 * b + 5), &ks0, sizeof(double), hipMemcpyHostToDevice));
    }
  }
  return LBM_OK;
}

// The sweep of lbm_adjoint_step and lbm_adjoint_run.  With bodies, each
// step of the recompute is the coupled step (forcing, stream-collide with the
// per-node force, probes and vertex velocities, vertex update) on buffers of
// the sweep, keeping the body state (P, Q, V) of every step of the segment;
// each step back first re-runs the step's forcing and stream-collide (for
// the force field and the step's rho, u), then transposes the vertex update,
// the elements, probes and vertex velocities, the volume term, the force
// adjoint at the forced nodes (mode 1), the forcing markers, and finally the
// fluid step with all node sources (mode 0).
static lbm_status adjoint_sweep(lbm_ctx* ctx, int32_t n_steps, int32_t every, const double* d_w, double theta,
                                int32_t tbody, double* d_lambda, double* d_grad, int nout, double* d_body,
                                double* h_J) {
  if (!ctx) return LBM_E_INVAL;
  if (ctx->broken) return LBM_E_STATE;
  if (n_steps < 0 || every < 1 || !d_lambda || !d_grad)
    return fail(ctx, LBM_E_INVAL, "adjoint: n_steps >= 0, checkpoint interval >= 1, lambda and grad required");
  const int nb = (int)ctx->bodies.size();
  for (const HostBody& B : ctx->bodies)
    if (B.rigid || B.fixed)
      return fail(ctx, LBM_E_UNSUPPORTED, "adjoint: soft bodies only (the rigid-body transpose is not built)");
  if (nb > 1)
    return fail(ctx, LBM_E_UNSUPPORTED, "adjoint: at most one body (the repulsion transpose is not built)");
  if (theta != 0.0 && (tbody < 0 || tbody >= nb)) return fail(ctx, LBM_E_INVAL, "adjoint: no such body");
  if (d_body && nb == 0) return fail(ctx, LBM_E_INVAL, "adjoint: no bodies for the body gradient");
  DevFlags h;
  lbm_status st = read_flags(ctx, &h);
  if (st) return st;
  CHK(ensure_bulk_list(ctx));
  const bool ib = nb > 0;
  const Grid& G = ctx->g;
  auto up256 = [](size_t b) { return (b + 255) & ~(size_t)255; };
  const size_t dbytes = up256(19 * (size_t)G.plane * sizeof(double));  // an adjoint field (FP64)
  const size_t xraw = 19 * (size_t)G.plane * ctx->ssize;                // a state (context's storage)
  const size_t xbytes = up256(xraw);
  const int nseg = n_steps == 0 ? 0 : (n_steps + every - 1) / every;
  const int tlen = n_steps == 0 ? 0 : std::min(every, n_steps);
  const int ntape = std::max(tlen, 2);
  // one arena: lam, the two mu, w, the two bounce-back accumulators (FP64),
  // the checkpoints and the tape (storage type), then the small pieces
  const size_t big_bytes = 6 * dbytes + (size_t)(nseg + ntape) * xbytes;
  const size_t hbytes = 19 * (size_t)ctx->nrec * sizeof(double);  // one step's record populations
  const int npart = adj_part_blocks(ctx->nrec, ctx->n_bulk);
  const size_t pbytes = ADJ_PART * (size_t)npart * sizeof(double);
  // with bodies: two force fields and their tile flags, the node sources and
  // flags, dJ/dF at nodes, a scratch state, body checkpoints and tape (P, Q,
  // V per step), eight body adjoint arrays
  const long long ntiles = (G.Np >> TILE_SHIFT) + 1;
  const size_t bstate = 9 * sizeof(double) * (size_t)ctx->nv;  // P, Q, V
  const size_t ib_bytes = ib ? 2 * up256(3 * (size_t)G.Np * 8) + 2 * up256(ntiles) + up256(7 * (size_t)G.Np * 8) +
                                   up256(ntiles) + up256(3 * (size_t)G.Np * 8) + xbytes +
                                   (size_t)(nseg + tlen + 1) * up256(bstate) + 8 * up256(bstate / 3) +
                                   up256(sizeof(double) * (2 + nb)) + up256(sizeof(DevFlags) + 64)
                             : 0;
  const size_t jbytes = up256(sizeof(double) * (ADJ_BLOCKS + 8));
  const size_t small = pbytes + 2 * ((size_t)ctx->n_bulk + ctx->nrec) * sizeof(uint32_t) + tlen * (hbytes + 256) +
                       4 * 256 + jbytes;
  // one launch for records and bulk nodes below 4M non-solid nodes (the
  // records' blocks are latency-bound; LBM_ADJ_SPLIT=1 forces two)
  const char* sp_env = getenv("LBM_ADJ_SPLIT");
  const int merged = (ctx->n_bulk + ctx->nrec < (4LL << 20)) && !(sp_env && atoi(sp_env) != 0);
  DevArena ar;
  if (hipMalloc(&ar.base, big_bytes + small + ib_bytes + 16 * 256) != hipSuccess) {
    (void)hipGetLastError();
    ar.base = nullptr;
    return fail(ctx, LBM_E_NOMEM, "adjoint: not enough device memory for the checkpoints and the tape");
  }
  auto big = [&](size_t i) { return (double*)(ar.base + i * dbytes); };
  auto state = [&](size_t i) { return (void*)(ar.base + 6 * dbytes + i * xbytes); };
  struct {
    double *lam, *mu[2], *acc[2], *w, *part, *jpart;
    uint32_t *pmask, *amask;
    std::vector<void*> ck, tape;
    std::vector<double*> hrec;
  } m;
  m.lam = big(0);
  m.mu[0] = big(1);
  m.mu[1] = big(2);
  m.w = d_w ? big(3) : nullptr;
  m.acc[0] = big(4);
  m.acc[1] = big(5);
  for (int c = 0; c < nseg; c++) m.ck.push_back(state(c));
  for (int k = 0; k < ntape; k++) m.tape.push_back(state(nseg + k));
  char* sp = ar.base + big_bytes;
  auto carve = [&](size_t bytes) {
    char* p = (char*)(((uintptr_t)sp + 255) & ~(uintptr_t)255);
    sp = p + bytes;
    return (void*)p;
  };
  m.part = (double*)carve(pbytes);
  m.jpart = (double*)carve(sizeof(double) * (ADJ_BLOCKS + 8));
  m.pmask = (uint32_t*)carve(((size_t)ctx->n_bulk + ctx->nrec) * sizeof(uint32_t));
  m.amask = (uint32_t*)carve(((size_t)ctx->n_bulk + ctx->nrec) * sizeof(uint32_t));
  for (int k = 0; k < tlen; k++) m.hrec.push_back((double*)carve(hbytes));
  hipStream_t s = ctx->stream;
  // solid entries stay zero in every buffer (never written by the sweep)
  CHK(hipMemsetAsync(ar.base, 0, big_bytes + pbytes + sizeof(double) * (ADJ_BLOCKS + 8) + 512, s));
  // the body part of the arena
  struct {
    long long* fx[2];
    uint8_t* tf[2];
    double *ext, *fbar, *gsum;
    uint8_t* etf;
    void* gB;
    std::vector<double*> bck, bt;
    double *arr[8];
    DevFlags* flags;
    unsigned int* cnt;
  } q{};
  double* bdiag_save = nullptr;
  std::vector<double> bdiag_h;
  if (ib) {
    char* ib0 = (char*)carve(ib_bytes);
    sp = ib0;
    for (int k = 0; k < 2; k++) q.fx[k] = (long long*)carve(3 * (size_t)G.Np * 8);
    for (int k = 0; k < 2; k++) q.tf[k] = (uint8_t*)carve(ntiles);
    q.ext = (double*)carve(7 * (size_t)G.Np * 8);
    q.etf = (uint8_t*)carve(ntiles);
    q.fbar = (double*)carve(3 * (size_t)G.Np * 8);
    q.gB = carve(xraw);
    for (int c = 0; c < nseg; c++) q.bck.push_back((double*)carve(bstate));
    for (int k = 0; k <= tlen; k++) q.bt.push_back((double*)carve(bstate));
    for (int k = 0; k < 8; k++) q.arr[k] = (double*)carve(bstate / 3);
    q.gsum = (double*)carve(sizeof(double) * (2 + nb));
    q.flags = (DevFlags*)carve(sizeof(DevFlags) + 64);
    q.cnt = (unsigned int*)(q.flags + 1);
    CHK(hipMemsetAsync(ib0, 0, (size_t)(sp - ib0), s));
    bdiag_h.resize(16 * (size_t)nb);
    CHK(hipMemcpyAsync(bdiag_h.data(), ctx->b_diag, sizeof(double) * bdiag_h.size(), hipMemcpyDeviceToHost, s));
    CHK(hipStreamSynchronize(s));
    bdiag_save = ctx->b_diag;
  }
  CHK(launch_adjoint_layout(G, ctx->ncls, d_lambda, m.lam, 1, s));
  if (d_w) CHK(launch_adjoint_layout(G, ctx->ncls, d_w, m.w, 1, s));
  FluidArgs a = fluid_args(ctx, 0);
  a.fx = nullptr;
  a.tflag = nullptr;
  a.mac = nullptr;
  a.bulk_list = ctx->bulk_list;
  a.nbulk_nodes = (int)ctx->n_bulk;
  CHK(launch_adjoint_mask(a, m.w, m.pmask, m.amask, s));
  const int nv3 = 3 * ctx->nv;
  const size_t vb = sizeof(double) * nv3;
  BodyArgs bb = ib ? ctx->bargs[0] : BodyArgs{};
  bb.stage = nullptr;  // the recomputed steps spread in one pass
  bb.stage_node = nullptr;
  // one coupled step from (gin, body slot `from`) into (gout, slot `to`)
  auto coupled = [&](const void* gin, void* gout, double* from, double* to, double* hrec) -> hipError_t {
    hipError_t e;
    // slot to: P' (written), Q' = P, V' (written): the step reads x^{n-1}
    // from Xnext and V from Vel before overwriting them
    if ((e = launch_body_slots(from, to, (long long)nv3, s)) != hipSuccess) return e;
    FluidArgs fa = a;
    fa.A = gin;
    fa.B = gout;
    fa.fx = q.fx[0];
    fa.tflag = q.tf[0];
    fa.mac = ctx->mac;
    fa.flags = q.flags;
    BodyArgs b2 = bb;
    b2.Xcur = from;
    b2.Xnext = to;
    b2.Vel = to + 2 * nv3;
    if ((e = launch_ib_force(ctx->prec, fa, b2, q.fx[0], q.tf[0], q.fx[1], q.tf[1], q.cnt, s)) != hipSuccess) return e;
    if ((e = launch_adjoint_forward(ctx->prec, fa, hrec, merged, s)) != hipSuccess) return e;
    if ((e = launch_mls_post(ctx->prec, fa, b2, q.fx[1], q.tf[1], s)) != hipSuccess) return e;
    if ((e = launch_body_post(b2, q.flags, nullptr, s)) != hipSuccess) return e;
    if ((e = launch_close(q.flags, s)) != hipSuccess) return e;
    // this step's force field is not needed again: clear it (the forcing of
    // the next step spreads into the same buffer)
    return launch_adjb_clear(G, q.ext, q.etf, q.fx[0], q.tf[0], s);
  };
  // forward pass: the state at the start of every segment
  const int cur0 = (int)(h.steps_done & 1);
  if (nseg > 0) {
    CHK(hipMemcpyAsync(m.ck[0], ctx->f[cur0], xraw, hipMemcpyDeviceToDevice, s));
    if (ib) {
      double* b0 = q.bck[0];
      CHK(hipMemcpyAsync(b0, ctx->X[cur0], vb, hipMemcpyDeviceToDevice, s));
      CHK(hipMemcpyAsync(b0 + nv3, ctx->X[cur0 ^ 1], vb, hipMemcpyDeviceToDevice, s));
      CHK(hipMemcpyAsync(b0 + 2 * nv3, ctx->Vel, vb, hipMemcpyDeviceToDevice, s));
    }
    for (int c = 1; c < nseg; c++) {
      const void* src = m.ck[c - 1];
      double* bsrc = ib ? q.bck[c - 1] : nullptr;
      for (int k = 0; k < every; k++) {
        void* dst = k == every - 1 ? m.ck[c] : m.tape[k & 1];
        if (ib) {
          double* bdst = k == every - 1 ? q.bck[c] : q.bt[k & 1];
          CHK(coupled(src, dst, bsrc, bdst, nullptr));
          bsrc = bdst;
        } else {
          a.A = src;
          a.B = dst;
          CHK(launch_adjoint_forward(ctx->prec, a, nullptr, merged, s));
        }
        src = dst;
      }
    }
  }
  // the recompute's extras: J's terms along the trajectory
  double* jsum = m.jpart + ADJ_BLOCKS;  // [0] sum of D_T
  auto observe = [&](const void* g, const double* P) -> hipError_t {
    hipError_t e = hipSuccess;
    if (!h_J) return e;
    if (m.w && (e = launch_adj_wdot(ctx->prec, a, g, m.w, m.amask, 1, m.jpart, s)) != hipSuccess) return e;
    if (ib && (e = launch_taylor(bb, P, std::max(tbody, 0), 0.0, nullptr, jsum, s)) != hipSuccess) return e;
    return e;
  };
  // reverse pass, segment by segment: recompute its states (and the records'
  // populations entering each collision; the last step's output goes to the
  // mu buffer that the next step back rewrites at every non-solid node), then
  // step back.  mu and the bounce-back accumulator alternate between two
  // buffers: each step reads those of the step after it.
  int cur = 0;
  bool first = true;
  double* A3[3] = {nullptr, nullptr, nullptr};  // aP, aQ, aV
  double* B3[3] = {nullptr, nullptr, nullptr};  // LP, Qn, Vn
  if (ib) {
    for (int k = 0; k < 3; k++) {
      A3[k] = q.arr[k];
      B3[k] = q.arr[3 + k];
    }
  }
  for (int c = nseg - 1; c >= 0; c--) {
    const int len = std::min(every, n_steps - c * every);
    CHK(hipMemcpyAsync(m.tape[0], m.ck[c], xraw, hipMemcpyDeviceToDevice, s));
    if (ib) CHK(hipMemcpyAsync(q.bt[0], q.bck[c], bstate, hipMemcpyDeviceToDevice, s));
    for (int k = 0; k < len; k++) {
      void* out = k + 1 < len ? m.tape[k + 1] : (void*)m.mu[cur];  // mu[cur]: large enough for any storage
      if (ib) {
        CHK(coupled(m.tape[k], out, q.bt[k], q.bt[k + 1], m.hrec[k]));
      } else {
        a.A = m.tape[k];
        a.B = out;
        CHK(launch_adjoint_forward(ctx->prec, a, m.hrec[k], merged, s));
      }
      CHK(observe(out, ib ? q.bt[k + 1] : nullptr));
      if (h_J && first && c == nseg - 1 && k == len - 1)  // <lambda, g^n>
        CHK(launch_adj_wdot(ctx->prec, a, out, m.lam, m.amask, 0, m.jpart, s));
    }
    for (int k = len - 1; k >= 0; k--) {
      a.A = m.tape[k];
      AdjStep st{};
      st.hrec = m.hrec[k];
      st.lam = first ? m.lam : nullptr;
      st.mu_next = m.mu[cur ^ 1];
      st.acc_in = m.acc[cur ^ 1];
      st.acc_out = m.acc[cur];
      st.w = m.w;
      st.mu = m.mu[cur];
      st.pmask = m.pmask;
      st.amask = m.amask;
      st.part = m.part;
      if (ib) {
        double* Pk = q.bt[k];  // the state the step started from
        if (theta != 0.0) CHK(launch_taylor(bb, q.bt[k + 1], tbody, theta, A3[0], nullptr, s));
        // the step's force field and fields again (into scratch)
        FluidArgs fa = a;
        fa.B = q.gB;
        fa.fx = q.fx[0];
        fa.tflag = q.tf[0];
        fa.mac = ctx->mac;
        fa.flags = q.flags;
        BodyArgs b2 = bb;
        b2.Xcur = Pk;
        b2.Xnext = q.bt[k + 1];  // not written by the forcing launch
        b2.Vel = Pk + 2 * nv3;
        CHK(launch_ib_force(ctx->prec, fa, b2, q.fx[0], q.tf[0], q.fx[1], q.tf[1], q.cnt, s));
        CHK(launch_adjoint_forward(ctx->prec, fa, nullptr, merged, s));
        AdjIB ibp{};
        ibp.aP = A3[0];
        ibp.aQ = A3[1];
        ibp.aV = A3[2];
        ibp.LP = B3[0];
        ibp.Qn = B3[1];
        ibp.Vn = B3[2];
        ibp.Fb = q.arr[6];
        ibp.ub0 = q.arr[7];
        ibp.ext = q.ext;
        ibp.etf = q.etf;
        ibp.fbar = q.fbar;
        ibp.gsum = q.gsum;
        ibp.kappa = ctx->stiff_scale;
        CHK(launch_adjb_vertex(b2, ibp, s));
        CHK(launch_adjb_body(ctx->prec, fa, b2, ibp, s));
        CHK(launch_adjb_volume(b2, ibp, s));
        CHK(launch_adjb_support(G, ctx->ncls, b2, q.etf, s));
        st.fx = q.fx[0];
        st.ftf = q.tf[0];
        st.ext = q.ext;
        st.etf = q.etf;
        st.fbar = q.fbar;
        st.mode = 1;
        CHK(launch_adjoint_reverse(ctx->prec, a, st, merged, s));
        CHK(launch_adjb_markers(ctx->prec, fa, b2, ibp, s));
        st.mode = 0;
      }
      CHK(launch_adjoint_reverse(ctx->prec, a, st, merged, s));
      if (ib) {
        CHK(launch_adjb_clear(G, q.ext, q.etf, q.fx[0], q.tf[0], s));
        for (int t = 0; t < 3; t++) std::swap(A3[t], B3[t]);
      }
      first = false;
      cur ^= 1;
    }
  }
  // dJ/dg^0 = P^T mu of the last step back (plain pulls and bounce-back)
  if (n_steps > 0) CHK(launch_adjoint_gather(a, m.pmask, m.amask, m.mu[cur ^ 1], m.acc[cur ^ 1], m.lam, s));
  CHK(launch_adjoint_layout(G, ctx->ncls, m.lam, d_lambda, 0, s));
  CHK(launch_adjoint_grad(m.part, npart, 1.0 / ctx->tau, ib ? q.gsum : nullptr, nout, d_grad, s));
  if (d_body) {
    for (int t = 0; t < 3; t++)
      CHK(hipMemcpyAsync(d_body + (size_t)t * nv3, A3[t], vb, hipMemcpyDeviceToDevice, s));
  }
  double jv[2] = {0.0, 0.0};
  if (h_J) {
    CHK(launch_adj_sum(m.jpart, ADJ_BLOCKS, m.jpart + ADJ_BLOCKS + 1, s));
    double hj[2];
    CHK(hipMemcpyAsync(hj, m.jpart + ADJ_BLOCKS, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
    CHK(hipStreamSynchronize(s));
    jv[0] = hj[1];
    jv[1] = hj[0];
  }
  DevFlags hf{};
  if (ib) {
    CHK(hipMemcpyAsync(&hf, q.flags, sizeof hf, hipMemcpyDeviceToHost, s));
    CHK(hipMemcpyAsync(bdiag_save, bdiag_h.data(), sizeof(double) * bdiag_h.size(), hipMemcpyHostToDevice, s));
  }
  CHK(hipStreamSynchronize(s));
  if (h_J) {
    h_J[0] = jv[0];
    h_J[1] = jv[1];
  }
  if (hf.stop & ST_DAMAGED) return fail(ctx, LBM_E_DAMAGED, "adjoint: a capsule was damaged along the trajectory");
  if (hf.stop & ST_UNSTABLE) return fail(ctx, LBM_E_UNSTABLE, "adjoint: the trajectory became unstable");
  return LBM_OK;
}

extern "C" lbm_status lbm_adjoint_step(lbm_ctx* ctx, int32_t n_steps, int32_t every, const double* d_w,
                                       double* d_lambda, double* d_grad) {
  return adjoint_sweep(ctx, n_steps, every, d_w, 0.0, -1, d_lambda, d_grad, 5, nullptr, nullptr);
}

extern "C" lbm_status lbm_adjoint_run(lbm_ctx* ctx, int32_t n_steps, int32_t every, const double* d_w,
                                      double taylor_weight, int32_t taylor_body, double* d_lambda,
                                      double* d_grad, double* d_body_grad, double* J) {
  return adjoint_sweep(ctx, n_steps, every, d_w, taylor_weight, taylor_body, d_lambda, d_grad, 6, d_body_grad, J);
}

// ------------------------------------------------------- checkpoint / restart
namespace {
struct CkptHeader {
  char magic[8];
  int32_t nx, ny, nz, prec, nbody, nv, nf, pad;
  int64_t steps_done;
};
}  // namespace

// The sections of a checkpoint after the header and flags, in file order:
// both population buffers; with bodies, per parity the force field, its tile
// flags and the vertex positions, then the velocities and the rigid-body and
// diagnostics tables.
static std::vector<std::pair<void*, size_t>> ckpt_sections(lbm_ctx* ctx) {
  std::vector<std::pair<void*, size_t>> v;
  const size_t fbytes = (size_t)19 * ctx->g.plane * ctx->ssize;
  for (int p = 0; p < 2; p++) v.emplace_back(ctx->f[p], fbytes);
  if (ctx->nf > 0) {
    const size_t fxb = 3 * (size_t)ctx->g.Np * sizeof(long long);
    for (int p = 0; p < 2; p++) {
      v.emplace_back(ctx->fx[p], fxb);
      v.emplace_back(ctx->tf[p], (size_t)ctx->ntiles);
      v.emplace_back(ctx->X[p], 3 * sizeof(double) * ctx->nv);
    }
    v.emplace_back(ctx->Vel, 3 * sizeof(double) * ctx->nv);
    v.emplace_back(ctx->b_rig, 32 * sizeof(double) * ctx->bodies.size());
    v.emplace_back(ctx->b_diag, 16 * sizeof(double) * ctx->bodies.size());
  }
  return v;
}

static CkptHeader ckpt_header(lbm_ctx* ctx, int64_t steps_done) {
  CkptHeader hd{};
  memcpy(hd.magic, "LBMIB01", 8);
  hd.nx = ctx->g.nx;
  hd.ny = ctx->g.ny;
  hd.nz = ctx->g.nz;
  hd.prec = ctx->prec;
  hd.nbody = (int)ctx->bodies.size();
  hd.nv = ctx->nv;
  hd.nf = ctx->nf;
  hd.steps_done = steps_done;
  return hd;
}

extern "C" lbm_status lbm_save(lbm_ctx* ctx, const char* path) {
  if (!ctx || !path) return LBM_E_INVAL;
  if (ctx->broken) return LBM_E_STATE;
  DevFlags h;
  lbm_status st = read_flags(ctx, &h);
  if (st) return st;
  const CkptHeader hd = ckpt_header(ctx, h.steps_done);
  // everything is copied to the host first, so a device error leaves no file behind
  const auto secs = ckpt_sections(ctx);
  std::vector<std::vector<char>> bufs(secs.size());
  for (size_t k = 0; k < secs.size(); k++) {
    bufs[k].resize(secs[k].second);
    CHK(hipMemcpy(bufs[k].data(), secs[k].first, secs[k].second, hipMemcpyDeviceToHost));
  }
  FILE* fp = fopen(path, "wb");
  if (!fp) return fail(ctx, LBM_E_INVAL, std::string("cannot open ") + path);
  bool ok = fwrite(&hd, sizeof hd, 1, fp) == 1 && fwrite(&h, sizeof h, 1, fp) == 1;
  for (size_t k = 0; ok && k < bufs.size(); k++)
    ok = fwrite(bufs[k].data(), 1, bufs[k].size(), fp) == bufs[k].size();
  ok = (fflush(fp) == 0) && ok;
  ok = (fclose(fp) == 0) && ok;
  if (!ok) return fail(ctx, LBM_E_INVAL, std::string("short write to ") + path);
  return LBM_OK;
}

extern "C" lbm_status lbm_load(lbm_ctx* ctx, const char* path) {
  if (!ctx || !path) return LBM_E_INVAL;
  if (ctx->broken) return LBM_E_STATE;
  FILE* fp = fopen(path, "rb");
  if (!fp) return fail(ctx, LBM_E_INVAL, std::string("cannot open ") + path);
  CkptHeader hd{};
  DevFlags h{};
  bool ok = fread(&hd, sizeof hd, 1, fp) == 1 && fread(&h, sizeof h, 1, fp) == 1;
  ok = ok && memcmp(hd.magic, "LBMIB01", 8) == 0 && hd.nx == ctx->g.nx && hd.ny == ctx->g.ny &&
       hd.nz == ctx->g.nz && hd.prec == ctx->prec && hd.nbody == (int)ctx->bodies.size() &&
       hd.nv == ctx->nv && hd.nf == ctx->nf && hd.steps_done == h.steps_done;
  if (!ok) {
    fclose(fp);
    return fail(ctx, LBM_E_INVAL, "checkpoint does not match this context");
  }
  // read and size-check the whole file before the first device copy: a
  // truncated or oversized file leaves the context as it was
  const auto secs = ckpt_sections(ctx);
  std::vector<std::vector<char>> bufs(secs.size());
  for (size_t k = 0; ok && k < secs.size(); k++) {
    bufs[k].resize(secs[k].second);
    ok = fread(bufs[k].data(), 1, secs[k].second, fp) == secs[k].second;
  }
  const bool at_end = ok && fgetc(fp) == EOF;
  fclose(fp);
  if (!ok) return fail(ctx, LBM_E_INVAL, "truncated checkpoint (context unchanged)");
  if (!at_end) return fail(ctx, LBM_E_INVAL, "checkpoint longer than this context's state (context unchanged)");
  CHK(hipStreamSynchronize(ctx->stream));
  for (size_t k = 0; k < secs.size(); k++)
    CHK(hipMemcpy(secs[k].first, bufs[k].data(), secs[k].second, hipMemcpyHostToDevice));
  CHK(hipMemcpy(ctx->flags, &h, sizeof h, hipMemcpyHostToDevice));
  ctx->enq = h.steps_done;
  if (!ctx->bodies.empty()) {
    // the marker order of the restored positions
    CHK(launch_bin_faces(ctx->bargs[ctx->enq & 1], ctx->stream));
    CHK(hipStreamSynchronize(ctx->stream));
  }
  ctx->bin_enq = ctx->enq;
  return LBM_OK;
}
