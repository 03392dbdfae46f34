// C ABI of libplbm (declared in include/plbm.h): lattice handles bound to
// caller-owned device memory, kernel launches on the caller's stream, and the
// continuous-batching slot table.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "plbm_aux.hpp"
#include "plbm_host.hpp"
#include "plbm_launch.hpp"

using namespace plbm;

namespace plbm {

static thread_local std::string g_err;

int set_error(int code, const char* fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

}  // namespace plbm

#define HIPCHK(x)                                                                              \
  do {                                                                                         \
    hipError_t e_ = (x);                                                                       \
    if (e_ != hipSuccess) return set_error(PLBM_E_DEVICE, "%s: %s", #x, hipGetErrorString(e_)); \
  } while (0)

namespace {

constexpr uint64_t kAlign = 256;
uint64_t align_up(uint64_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

int storage_bytes(int storage) { return storage == PLBM_F64 ? 8 : storage == PLBM_F32 ? 4 : 2; }

void d3_tile_shape(int storage, int aa, int* tx, int* ty) {
  switch (storage) {
    case PLBM_F64: return tile_shape_f64(aa, tx, ty);
    case PLBM_F32: return tile_shape_f32(aa, tx, ty);
    case PLBM_F16S: return tile_shape_f16s(aa, tx, ty);
    case PLBM_BF16S: return tile_shape_bf16s(aa, tx, ty);
    case PLBM_F16R: return tile_shape_f16r(aa, tx, ty);
    default: return tile_shape_bf16r(aa, tx, ty);
  }
}

struct Layout {
  int Q, D;
  int nxk, nyk, nzk;  // kernel axes
  int tx, ty, cz, tiles_x, tiles_y, tiles_z, ntiles;
  int cz2, ncl, ntl;  // two-class z partition (see choose_partition)
  int nxb;         // 128-byte x blocks per row of stored populations
  uint64_t zdata;  // bytes of node data of one z plane of stored populations
  uint64_t zblock; // zdata plus a trash area for the ragged-tile lanes of one workgroup
  int64_t N;
  uint64_t popA, popB, refA, refB, psi, aux, uprev, red, kp, wbmu, total;
};

bool local_shift(int storage) { return storage == PLBM_F16R || storage == PLBM_BF16R; }

// Planes per z chunk.  A workgroup spends about cz + 2 plane times on a
// chunk (the two extra planes of psi are recomputed), and the grid runs in
// workgroups / resident rounds, where `resident` is how many step workgroups
// the device holds at once (CUs times the occupancy of the kernel).  A
// partly filled last round costs about half a round more than its share
// (measured on the 256^3 cube and the 384x384x128 channel), so a uniform
// chunk costs (workgroups / resident + ceil(workgroups / resident)) / 2 (cz + 2)
// plane times; the chunk minimises that, on ties the longer chunk.  Without
// a device (resident <= 0), aim at 512 workgroups.
struct ZPart {
  int cz;   // planes per chunk of the first ncl columns (whole columns when ncl > 0)
  int cz2;  // planes per chunk of the other columns
  int ncl;  // columns split with cz; 0 for a uniform partition with cz2
};

static double uniform_cost(int nzk, int64_t cols, int cz, int64_t resident) {
  const int64_t wg = cols * ((nzk + cz - 1) / cz);
  return 0.5 * ((double)wg / resident + (double)((wg + resident - 1) / resident)) * (cz + 2);
}

static int best_uniform(int nzk, int64_t cols, int64_t resident, double* cost) {
  int best = nzk;
  double bc = -1.0;
  for (int cz = nzk; cz >= 1 && cz >= (nzk < 4 ? 1 : 4); --cz) {
    const double c = uniform_cost(nzk, cols, cz, resident);
    if (bc < 0.0 || c < bc) {
      bc = c;
      best = cz;
    }
  }
  *cost = bc;
  return best;
}

// Two classes of work items when a lattice has more columns (tiles_xy) than
// the device holds workgroups: the first m * resident columns as whole
// columns (m rounds in which every workgroup ends together, no partial
// round), then the remaining columns in shorter chunks that fill the last
// round (launched in that order, so the long items start first).  On the
// 384x384x128 channel (288 columns of 64 x 8 nodes, 256 resident) that is
// 256 whole columns plus 32 columns in chunks of 16 planes, 148 plane times
// against 161.5 for the best uniform chunk (32 planes, 4.5 rounds).
ZPart choose_partition(int nzk, int tiles_xy, int64_t resident) {
  ZPart z{0, 0, 0};
  if (const char* e = std::getenv("PLBM_CZ")) {
    int v = std::atoi(e);
    if (v > 0) {
      z.cz = z.cz2 = v < nzk ? v : nzk;
      return z;
    }
  }
  if (resident <= 0) {
    int64_t cz = ((int64_t)nzk * tiles_xy + 511) / 512;
    if (cz < 4) cz = 4;
    if (cz > 128) cz = 128;
    z.cz = z.cz2 = (int)(cz > nzk ? nzk : cz);
    return z;
  }
  double best;
  z.cz = z.cz2 = best_uniform(nzk, tiles_xy, resident, &best);
  const char* u = std::getenv("PLBM_UNIFORM_CHUNKS");
  if (u && std::atoi(u) != 0) return z;
  for (int64_t m = 1; m * resident <= tiles_xy; ++m) {
    const int64_t rest = tiles_xy - m * resident;
    double c2 = 0.0;
    int cz2 = nzk;
    if (rest > 0) cz2 = best_uniform(nzk, rest, resident, &c2);
    const double c = (double)m * (nzk + 2) + c2;
    if (c < best) {
      best = c;
      z.cz = nzk;
      z.cz2 = cz2;
      z.ncl = (int)(m * resident);
    }
  }
  return z;
}

int make_layout(const plbm_lattice_desc* d, Layout* L, int64_t resident = 0) {
  if (!d) return set_error(PLBM_E_INVALID, "null descriptor");
  if (d->lattice != PLBM_D2Q9 && d->lattice != PLBM_D3Q19) return set_error(PLBM_E_INVALID, "unknown lattice kind");
  if (d->collision != PLBM_BGK && d->collision != PLBM_MRT) return set_error(PLBM_E_INVALID, "unknown collision");
  if (d->storage < PLBM_F64 || d->storage > PLBM_BF16R) return set_error(PLBM_E_INVALID, "unknown storage");
  if (d->nx < 1 || d->ny < 1 || d->nz < 1) return set_error(PLBM_E_INVALID, "lattice sizes must be >= 1");
  if (d->pattern != PLBM_PATTERN_AB && d->pattern != PLBM_PATTERN_AA)
    return set_error(PLBM_E_INVALID, "unknown storage pattern");
  const bool aa = d->pattern == PLBM_PATTERN_AA;
  if (d->scheme != PLBM_SCHEME_PSEUDOPOTENTIAL && d->scheme != PLBM_SCHEME_WELL_BALANCED)
    return set_error(PLBM_E_INVALID, "unknown scheme");
  const bool wb = d->scheme == PLBM_SCHEME_WELL_BALANCED;
  if (wb) {
    if (!(d->wb_k > 0.0) || !std::isfinite(d->wb_k)) return set_error(PLBM_E_INVALID, "well-balanced scheme: wb_k > 0");
    if (!(d->wb_rho0 >= 0.0) || !std::isfinite(d->wb_rho0))
      return set_error(PLBM_E_INVALID, "well-balanced scheme: wb_rho0 >= 0");
    if (aa) return set_error(PLBM_E_UNSUPPORTED, "well-balanced scheme: A-B pattern only");
    if (d->storage != PLBM_F64 && d->storage != PLBM_F32)
      return set_error(PLBM_E_UNSUPPORTED, "well-balanced scheme: F64 or F32 storage only");
    if (d->rho_wall[0] > 0.0 || d->rho_wall[1] > 0.0)
      return set_error(PLBM_E_UNSUPPORTED, "well-balanced scheme: mirror walls only");
  }
  for (int k = 0; k < 2; ++k) {
    if (!std::isfinite(d->rho_wall[k]) || d->rho_wall[k] < 0.0)
      return set_error(PLBM_E_INVALID, "wall densities must be finite and >= 0");
    if (d->rho_wall[k] > 0.0 && d->bc[d->lattice == PLBM_D2Q9 ? 1 : 2] != PLBM_HALFWAY_BB)
      return set_error(PLBM_E_INVALID, "a wall density needs walls on the last axis");
  }
  const bool is2d = d->lattice == PLBM_D2Q9;
  if (is2d && d->nz != 1) return set_error(PLBM_E_INVALID, "D2Q9 requires nz = 1");
  for (int a = 0; a < 3; ++a)
    if (d->bc[a] != PLBM_PERIODIC && d->bc[a] != PLBM_HALFWAY_BB) return set_error(PLBM_E_INVALID, "unknown boundary kind");
  const int last = is2d ? 1 : 2;
  for (int a = 0; a < 3; ++a)
    if (a != last && d->bc[a] != PLBM_PERIODIC)
      return set_error(PLBM_E_UNSUPPORTED, "walls are supported on the last axis only (axis %d given)", a);
  L->Q = is2d ? 9 : 19;
  L->D = is2d ? 2 : 3;
  L->nxk = d->nx;
  L->nyk = is2d ? 1 : d->ny;
  L->nzk = is2d ? d->ny : d->nz;
  L->N = (int64_t)d->nx * d->ny * d->nz;
  if (L->N > 0x7fffffffLL) return set_error(PLBM_E_INVALID, "lattice larger than 2^31 - 1 nodes");
  if (is2d) {
    L->tx = TileShape<D2Q9L>::TX;
    L->ty = TileShape<D2Q9L>::TY;
  } else {
    d3_tile_shape(d->storage, aa, &L->tx, &L->ty);
  }
  L->tiles_x = (L->nxk + L->tx - 1) / L->tx;
  L->tiles_y = (L->nyk + L->ty - 1) / L->ty;
  {
    const ZPart zp = choose_partition(L->nzk, L->tiles_x * L->tiles_y, resident);
    L->cz = zp.cz;
    L->cz2 = zp.cz2;
    L->ncl = zp.ncl;
  }
  L->tiles_z = (L->nzk + L->cz2 - 1) / L->cz2;  // chunks per column of the second class
  L->ntl = L->ncl * ((L->nzk + L->cz - 1) / L->cz);
  int64_t nt = (int64_t)L->ntl + (int64_t)(L->tiles_x * L->tiles_y - L->ncl) * L->tiles_z;
  if ((int64_t)L->tiles_x * L->tiles_y * L->nzk > 0x3fffffff) return set_error(PLBM_E_INVALID, "too many tiles");
  L->ntiles = (int)nt;
  // reduction records are sized for the shortest chunk, so that the byte
  // count does not depend on the device the lattice is created on
  const int64_t max_tiles = (int64_t)L->tiles_x * L->tiles_y * L->nzk;
  const uint64_t S = storage_bytes(d->storage);
  // block width of the population layout (Lines<T> in the kernels)
  const int XB = (int)(128 / S) < PLBM_XB ? (int)(128 / S) : PLBM_XB;
  const uint64_t QB = (uint64_t)XB * S;
  const uint64_t blk = (L->Q * QB + 127) / 128 * 128;  // bytes of one block of XB nodes (Lines<T>::slots)
  L->nxb = (L->nxk + XB - 1) / XB;
  L->zdata = (uint64_t)L->nyk * L->nxb * blk;
  const int nthr = L->tx * L->ty;  // threads per workgroup (one node each)
  // a trash area after each plane takes the stores of ragged-tile lanes
  L->zblock = L->zdata + (uint64_t)((nthr + XB - 1) / XB) * blk;
  if (L->zblock >= (1ull << 31)) return set_error(PLBM_E_UNSUPPORTED, "one z plane of populations exceeds 2 GiB");
  uint64_t off = 0;
  L->popA = off;
  off = align_up(off + L->zblock * L->nzk);
  L->popB = aa ? L->popA : off;  // the in-place pattern has one array
  if (!aa) off = align_up(off + L->zblock * L->nzk);
  // in-place pattern: psi of every node in the arithmetic type (float64 for
  // float64 storage, float32 otherwise)
  L->psi = off;
  if (aa) off = align_up(off + (uint64_t)L->N * (d->storage == PLBM_F64 ? 8 : 4));
  // reference densities of locally shifted storage: N nodes + a trash slot per thread
  const uint64_t nref = local_shift(d->storage) ? (uint64_t)(L->N + 256) * 2 : 0;
  L->refA = off;
  off = align_up(off + nref);
  L->refB = off;
  off = align_up(off + nref);
  L->aux = off;
  off = align_up(off + 4ull * L->N * 8);
  L->uprev = off;
  off = align_up(off + (uint64_t)L->D * L->N * 4);
  L->red = off;
  off = align_up(off + (uint64_t)(max_tiles + 1) * sizeof(RedRec));
  L->kp = off;
  off = align_up(off + sizeof(KParams));
  // well-balanced scheme: chemical potential of every node (arithmetic type)
  const uint64_t cb = d->storage == PLBM_F64 ? 8 : 4;
  L->wbmu = off;
  if (wb) off = align_up(off + (uint64_t)L->N * cb);
  L->total = off;
  return PLBM_OK;
}

}  // namespace

struct plbm_lattice {
  plbm_lattice_desc desc;
  plbm_lattice_params prm;
  Layout lay;
  KParams kp;
  KParams* kp_dev;
  hipStream_t stream;
  char* mem;
  int64_t t;
  int64_t t_red;
  bool has_red;
  hipGraphExec_t graph2;  // two steps (phase 0, phase 1)
  hipGraphExec_t graphL;  // long_steps() steps from phase 0
  bool has_graph;
  plbm_batch* batch;  // the batch the lattice is attached to, or null
  int32_t slot;
};

static void batch_forget(plbm_batch* b, int32_t slot);

namespace {

// Calls that change a lattice's state are refused while a batch owns it.
int check_free(plbm_lattice* L) {
  if (!L) return set_error(PLBM_E_INVALID, "null lattice");
  if (L->batch) return set_error(PLBM_E_INVALID, "lattice is attached to a batch (slot %d); detach it first", L->slot);
  return PLBM_OK;
}

hipError_t launch_step(const plbm_lattice_desc& d, StepLaunch& a) {
  switch (d.storage) {
    case PLBM_F64: return launch_step_f64(a);
    case PLBM_F32: return launch_step_f32(a);
    case PLBM_F16S: return launch_step_f16s(a);
    case PLBM_BF16S: return launch_step_bf16s(a);
    case PLBM_F16R: return launch_step_f16r(a);
    default: return launch_step_bf16r(a);
  }
}

// Update workgroups the current device holds at once for this descriptor
// (CUs x occupancy), or 0 if it cannot be queried.
int64_t resident_workgroups(const plbm_lattice_desc& d) {
  const int lat = d.lattice == PLBM_D3Q19 ? 1 : 0;
  const int last = lat ? 2 : 1;
  const int walls = d.bc[last] == PLBM_HALFWAY_BB;
  const int aa = d.pattern == PLBM_PATTERN_AA;
  int blocks = 0, dev = 0, cus = 0;
  hipError_t e;
  switch (d.storage) {
    case PLBM_F64: e = occupancy_step_f64(lat, d.collision, walls, aa, &blocks); break;
    case PLBM_F32: e = occupancy_step_f32(lat, d.collision, walls, aa, &blocks); break;
    case PLBM_F16S: e = occupancy_step_f16s(lat, d.collision, walls, aa, &blocks); break;
    case PLBM_BF16S: e = occupancy_step_bf16s(lat, d.collision, walls, aa, &blocks); break;
    case PLBM_F16R: e = occupancy_step_f16r(lat, d.collision, walls, aa, &blocks); break;
    default: e = occupancy_step_bf16r(lat, d.collision, walls, aa, &blocks); break;
  }
  if (e != hipSuccess || blocks <= 0) return 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) return 0;
  return (int64_t)blocks * cus;
}

hipError_t launch_aux(const plbm_lattice_desc& d, AuxLaunch& a) {
  switch (d.storage) {
    case PLBM_F64: return launch_aux_f64(a);
    case PLBM_F32: return launch_aux_f32(a);
    case PLBM_F16S: return launch_aux_f16s(a);
    case PLBM_BF16S: return launch_aux_bf16s(a);
    case PLBM_F16R: return launch_aux_f16r(a);
    default: return launch_aux_bf16r(a);
  }
}

int aux_blocks(int64_t N) {
  int64_t b = (N + 255) / 256;
  return (int)(b < 4096 ? (b < 1 ? 1 : b) : 4096);
}

// Records the reduce pass of a lattice writes (one per tile).
int reduce_records(const plbm_lattice* L) { return L->lay.ntiles; }

// Workgroups per tile chunk of the in-place pattern's psi pass (measured on
// 256^3: float32 and float64 fastest with one, 16-bit storage with eight;
// PLBM_PSI_SPLIT overrides, for tuning; read once).
int psi_split(int storage) {
  static const int forced = [] {
    const char* e = std::getenv("PLBM_PSI_SPLIT");
    return e ? std::atoi(e) : 0;
  }();
  if (forced > 0) return forced;
  return storage_bytes(storage) == 2 ? 8 : 1;
}

// Multi-step calls replay captured graphs unless PLBM_NO_GRAPH is set (read
// once).
bool graphs_enabled() {
  static const bool on = std::getenv("PLBM_NO_GRAPH") == nullptr;
  return on;
}

// Steps of the long replay graph (one graph launch carries many kernels, so
// the gap the runtime leaves between consecutive graph launches, about 8 us on
// MI355X, is paid once per that many steps); PLBM_LONG_GRAPH overrides (an
// even count from 4 to 1024; anything else: two-step graphs only), read once.
int long_steps() {
  static const int n = [] {
    const char* e = std::getenv("PLBM_LONG_GRAPH");
    if (!e) return 16;
    const int v = std::atoi(e);
    return (v >= 4 && v <= 1024 && v % 2 == 0) ? v : 0;  // even: each replay starts at phase 0
  }();
  return n;
}

int run_step_kernel(plbm_lattice* L, int mode, int phase, double* orho, double* ou, void* red = nullptr) {
  StepLaunch a{};
  a.lattice = L->desc.lattice;
  a.coll = L->desc.collision;
  a.mode = mode;
  a.walls = L->kp.bb_z;
  a.aa = L->kp.aa;
  a.psplit = psi_split(L->desc.storage);
  a.nblocks = L->lay.ntiles;
  a.stream = L->stream;
  a.P = L->kp_dev;
  a.work = nullptr;
  a.nwork = 0;
  a.phase = phase;
  a.out_rho = orho;
  a.out_u = ou;
  a.red = red;
  a.wb = L->kp.wb;
  HIPCHK(launch_step(L->desc, a));
  return PLBM_OK;
}

int run_aux(plbm_lattice* L, int what, int dir, const double* in0, const double* in1, double* out,
            const ShapeK* shape) {
  AuxLaunch a{};
  a.lattice = L->desc.lattice;
  a.what = what;
  a.nblocks = aux_blocks(L->lay.N);
  a.stream = L->stream;
  a.P = L->kp_dev;
  a.par = (int)(L->t & 1);
  a.dir = dir;
  a.in0 = in0;
  a.in1 = in1;
  a.out = out;
  a.shape = shape;
  HIPCHK(launch_aux(L->desc, a));
  return PLBM_OK;
}

double* aux_ptr(plbm_lattice* L) { return reinterpret_cast<double*>(L->mem + L->lay.aux); }

void fill_kparams(plbm_lattice* L) {
  const Layout& y = L->lay;
  const plbm_lattice_params& p = L->prm;
  KParams& k = L->kp;
  std::memset(&k, 0, sizeof(k));
  k.pop[0] = L->mem + y.popA;
  k.pop[1] = L->mem + y.popB;
  k.ref[0] = local_shift(L->desc.storage) ? L->mem + y.refA : nullptr;
  k.ref[1] = local_shift(L->desc.storage) ? L->mem + y.refB : nullptr;
  k.aa = L->desc.pattern == PLBM_PATTERN_AA;
  k.rho_wall[0] = L->desc.rho_wall[0];
  k.rho_wall[1] = L->desc.rho_wall[1];
  k.psi = k.aa ? L->mem + y.psi : nullptr;
  k.aux = reinterpret_cast<double*>(L->mem + y.aux);
  k.uprev = reinterpret_cast<float*>(L->mem + y.uprev);
  k.red = reinterpret_cast<double*>(L->mem + y.red);
  k.N = y.N;
  k.nx = y.nxk;
  k.ny = y.nyk;
  k.nz = y.nzk;
  k.bb_z = L->desc.bc[L->desc.lattice == PLBM_D2Q9 ? 1 : 2] == PLBM_HALFWAY_BB;
  k.tiles_x = y.tiles_x;
  k.tiles_y = y.tiles_y;
  k.tiles_z = y.tiles_z;
  k.cz = y.cz;
  k.cz2 = y.cz2;
  k.ncl = y.ncl;
  k.ntl = y.ntl;
  k.ntiles = y.ntiles;
  k.eos = p.eos;
  k.K = p.K;
  k.e_rv = p.eos_rho_v;
  k.e_rl = p.eos_rho_l;
  k.e_sqrt_rv = std::sqrt(p.eos_rho_v);
  k.pr_RT = p.pr_R * p.pr_T;
  k.pr_b = p.pr_b;
  k.pr_aalpha = p.pr_a * p.pr_alpha;
  k.eps = p.epsilon;
  k.kappa = p.kappa;
  k.G = p.G;
  k.tau_v = p.tau_v;
  k.tau_slope = (p.tau_l - p.tau_v) / (p.rho_l - p.rho_v);
  k.rho_v = p.rho_v;
  for (int a = 0; a < 3; ++a) k.Fg[a] = p.body_force[a];
  const double defaults[4] = {0.8, 0.8, 1.1, 1.1};
  for (int a = 0; a < 4; ++a) k.rates[a] = L->desc.mrt_rates[a] > 0 ? L->desc.mrt_rates[a] : defaults[a];
  k.rho0_shift = (L->desc.storage == PLBM_F16S || L->desc.storage == PLBM_BF16S)
                     ? (L->desc.rho0_shift > 0 ? L->desc.rho0_shift : p.rho_l)
                     : 0.0;
  k.parity = 0;
  k.nxb = y.nxb;
  k.zblock = (int64_t)y.zblock;
  k.zdata = (int64_t)y.zdata;
  k.wb = L->desc.scheme == PLBM_SCHEME_WELL_BALANCED;
  k.wb_k = L->desc.wb_k;
  k.wb_rho0 = L->desc.wb_rho0 > 0.0 ? L->desc.wb_rho0 : p.rho_v;
  k.wb_mu = k.wb ? L->mem + y.wbmu : nullptr;
}

int check_lat(plbm_lattice* L) { return L ? PLBM_OK : set_error(PLBM_E_INVALID, "null lattice"); }

// Capture `len` steps, phases 0, 1, 0, ..., issued by `launch(phase)` on
// `stream`, into an executable graph.
template <class F>
int capture_steps(hipStream_t stream, int len, F&& launch, hipGraphExec_t* out) {
  hipGraph_t g;
  HIPCHK(hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal));
  int st = PLBM_OK;
  for (int k = 0; k < len && st == PLBM_OK; ++k) st = launch(k & 1);
  hipError_t e = hipStreamEndCapture(stream, &g);
  if (st != PLBM_OK) {
    if (e == hipSuccess) (void)hipGraphDestroy(g);
    return st;
  }
  if (e != hipSuccess) return set_error(PLBM_E_DEVICE, "hipStreamEndCapture: %s", hipGetErrorString(e));
  e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) return set_error(PLBM_E_DEVICE, "hipGraphInstantiate: %s", hipGetErrorString(e));
  return PLBM_OK;
}

int capture_graphs(plbm_lattice* L) {
  if (L->has_graph) return PLBM_OK;
  auto launch = [L](int phase) { return run_step_kernel(L, MODE_STEP, phase, nullptr, nullptr); };
  int st = capture_steps(L->stream, 2, launch, &L->graph2);
  if (st) return st;
  if (long_steps() > 0) {
    st = capture_steps(L->stream, long_steps(), launch, &L->graphL);
    if (st) {
      (void)hipGraphExecDestroy(L->graph2);
      return st;
    }
  }
  L->has_graph = true;
  return PLBM_OK;
}

}  // namespace

extern "C" {

int plbm_abi_version(void) { return PLBM_ABI_VERSION; }

const char* plbm_last_error(void) { return g_err.c_str(); }

int plbm_resolve_params(const plbm_phys_params* phys, const plbm_lattice_map* map, plbm_lattice_params* out) {
  return params_resolve(phys, map, out);
}

int plbm_params_pr_lattice(double T_over_Tc, double omega, double epsilon, double kappa, double tau_v, double tau_l,
                           const double* body_force, plbm_lattice_params* out) {
  if (!out) return set_error(PLBM_E_INVALID, "null output");
  return params_pr_lattice(T_over_Tc, omega, epsilon, kappa, tau_v, tau_l, body_force, out);
}

int plbm_params_paper_lattice(double rho_v, double rho_l, double xi, double epsilon, double kappa, double tau_v,
                              double tau_l, const double* body_force, plbm_lattice_params* out) {
  if (!out) return set_error(PLBM_E_INVALID, "null output");
  return params_paper_lattice(rho_v, rho_l, xi, epsilon, kappa, tau_v, tau_l, body_force, out);
}

int plbm_lattice_bytes(const plbm_lattice_desc* desc, uint64_t* bytes) {
  if (!bytes) return set_error(PLBM_E_INVALID, "null output");
  Layout L;
  int st = make_layout(desc, &L);
  if (st) return st;
  *bytes = L.total;
  return PLBM_OK;
}

int plbm_create(const plbm_lattice_desc* desc, const plbm_lattice_params* params, void* dev_mem, uint64_t dev_bytes,
                void* hip_stream, plbm_lattice** out) {
  if (!out || !params) return set_error(PLBM_E_INVALID, "null argument");
  *out = nullptr;
  Layout lay;
  if (!desc) return set_error(PLBM_E_INVALID, "null descriptor");
  int st = make_layout(desc, &lay, resident_workgroups(*desc));
  if (st) return st;
  if (!dev_mem) return set_error(PLBM_E_INVALID, "null device memory");
  if (((uintptr_t)dev_mem) % kAlign) return set_error(PLBM_E_INVALID, "device memory must be 256-byte aligned");
  if (dev_bytes < lay.total)
    return set_error(PLBM_E_NOMEM, "device buffer holds %llu bytes, lattice needs %llu", (unsigned long long)dev_bytes,
                     (unsigned long long)lay.total);
  if (!(params->rho_l > params->rho_v) || !(params->tau_v > 0.5) || !(params->tau_l > 0.5))
    return set_error(PLBM_E_INVALID, "parameters: need rho_v < rho_l and tau > 1/2");
  if (params->eos != PLBM_EOS_PAPER && params->eos != PLBM_EOS_PENG_ROBINSON)
    return set_error(PLBM_E_INVALID, "parameters: unknown EOS");
  plbm_lattice* L = new plbm_lattice();
  L->desc = *desc;
  L->prm = *params;
  L->lay = lay;
  L->mem = static_cast<char*>(dev_mem);
  L->stream = static_cast<hipStream_t>(hip_stream);
  L->t = 0;
  L->t_red = 0;
  L->has_red = false;
  L->has_graph = false;
  L->batch = nullptr;
  L->slot = -1;
  L->kp_dev = reinterpret_cast<KParams*>(L->mem + lay.kp);
  fill_kparams(L);
  hipError_t e = hipMemcpyAsync(L->kp_dev, &L->kp, sizeof(KParams), hipMemcpyHostToDevice, L->stream);
  if (e == hipSuccess) e = hipMemsetAsync(L->mem + lay.uprev, 0, (size_t)lay.D * lay.N * 4, L->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(L->stream);
  if (e != hipSuccess) {
    delete L;
    return set_error(PLBM_E_DEVICE, "plbm_create: %s", hipGetErrorString(e));
  }
  *out = L;
  return PLBM_OK;
}

int plbm_init_fields(plbm_lattice* L, const double* rho, const double* u) {
  if (check_free(L)) return PLBM_E_INVALID;
  if (!rho) return set_error(PLBM_E_INVALID, "null rho");
  const int64_t N = L->lay.N;
  double* aux = aux_ptr(L);
  HIPCHK(hipMemcpyAsync(aux, rho, N * 8, hipMemcpyHostToDevice, L->stream));
  if (u) HIPCHK(hipMemcpyAsync(aux + N, u, (size_t)L->lay.D * N * 8, hipMemcpyHostToDevice, L->stream));
  L->t = 0;
  L->has_red = false;
  int st = run_aux(L, AUX_INIT_FIELDS, 0, aux, u ? aux + N : nullptr, nullptr, nullptr);
  if (st) return st;
  HIPCHK(hipStreamSynchronize(L->stream));
  return PLBM_OK;
}

int plbm_init_shape(plbm_lattice* L, const plbm_shape* s) {
  if (check_free(L)) return PLBM_E_INVALID;
  if (!s || s->kind < 0 || s->kind > 2 || !(s->W > 0)) return set_error(PLBM_E_INVALID, "bad shape");
  if (s->axis < 0 || s->axis >= L->lay.D) return set_error(PLBM_E_INVALID, "shape axis out of range");
  ShapeK k;
  k.kind = s->kind;
  k.axis = s->axis;
  k.rho_in = s->rho_in;
  k.rho_out = s->rho_out;
  k.W = s->W;
  k.R = s->R;
  for (int a = 0; a < 3; ++a) {
    k.centre[a] = s->centre[a];
    k.u0[a] = a < L->lay.D ? s->u0[a] : 0.0;
  }
  k.level = s->level;
  L->t = 0;
  L->has_red = false;
  int st = run_aux(L, AUX_INIT_SHAPE, 0, nullptr, nullptr, nullptr, &k);
  if (st) return st;
  HIPCHK(hipStreamSynchronize(L->stream));
  return PLBM_OK;
}

int plbm_step(plbm_lattice* L, int64_t n) {
  if (check_free(L)) return PLBM_E_INVALID;
  if (n < 0) return set_error(PLBM_E_INVALID, "negative step count");
  // Steps replay captured graphs of long_steps() and two steps.  They are
  // captured on the first call (n = 0 included), so no later call pays for
  // capture and instantiation.  The legacy null stream cannot be captured, and a stream
  // the caller is capturing takes the launches directly into its own graph.
  bool replay = false;
  if (L->stream != nullptr && graphs_enabled()) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    HIPCHK(hipStreamIsCapturing(L->stream, &cs));
    if (cs == hipStreamCaptureStatusNone) {
      int st = capture_graphs(L);
      if (st) return st;
      replay = true;
    }
  }
  if (replay && n >= 2) {
    int st;
    if (L->t & 1) {
      st = run_step_kernel(L, MODE_STEP, 1, nullptr, nullptr);
      if (st) return st;
      ++L->t;
      --n;
    }
    for (const int m = long_steps(); m > 0 && n >= m; n -= m) {
      HIPCHK(hipGraphLaunch(L->graphL, L->stream));
      L->t += m;
    }
    for (; n >= 2; n -= 2) {
      HIPCHK(hipGraphLaunch(L->graph2, L->stream));
      L->t += 2;
    }
  }
  for (; n > 0; --n) {
    int st = run_step_kernel(L, MODE_STEP, (int)(L->t & 1), nullptr, nullptr);
    if (st) return st;
    ++L->t;
  }
  return PLBM_OK;
}

int plbm_moments_device(plbm_lattice* L, void* rho_dev, void* u_dev) {
  if (check_lat(L)) return PLBM_E_INVALID;
  if (!rho_dev || !u_dev) return set_error(PLBM_E_INVALID, "null output");
  return run_step_kernel(L, MODE_MOMENTS, (int)(L->t & 1), static_cast<double*>(rho_dev), static_cast<double*>(u_dev));
}

int plbm_read_moments(plbm_lattice* L, double* rho, double* u) {
  if (check_lat(L)) return PLBM_E_INVALID;
  if (!rho || !u) return set_error(PLBM_E_INVALID, "null output");
  const int64_t N = L->lay.N;
  double* aux = aux_ptr(L);
  int st = run_step_kernel(L, MODE_MOMENTS, (int)(L->t & 1), aux, aux + N);
  if (st) return st;
  HIPCHK(hipMemcpyAsync(rho, aux, N * 8, hipMemcpyDeviceToHost, L->stream));
  HIPCHK(hipMemcpyAsync(u, aux + N, (size_t)L->lay.D * N * 8, hipMemcpyDeviceToHost, L->stream));
  HIPCHK(hipStreamSynchronize(L->stream));
  return PLBM_OK;
}

int plbm_read_populations(plbm_lattice* L, double* f) {
  if (check_lat(L)) return PLBM_E_INVALID;
  if (!f) return set_error(PLBM_E_INVALID, "null output");
  const int64_t N = L->lay.N;
  double* aux = aux_ptr(L);
  for (int q = 0; q < L->lay.Q; ++q) {
    int st = run_aux(L, AUX_READ_POP, q, nullptr, nullptr, aux, nullptr);
    if (st) return st;
    HIPCHK(hipMemcpyAsync(f + (size_t)q * N, aux, N * 8, hipMemcpyDeviceToHost, L->stream));
    HIPCHK(hipStreamSynchronize(L->stream));
  }
  return PLBM_OK;
}

int plbm_write_populations(plbm_lattice* L, const double* f) {
  if (check_free(L)) return PLBM_E_INVALID;
  if (!f) return set_error(PLBM_E_INVALID, "null input");
  const int64_t N = L->lay.N;
  double* aux = aux_ptr(L);
  if (local_shift(L->desc.storage)) {
    // reference densities first: rho = sum_q f_q, then half precision
    for (int q = 0; q < L->lay.Q; ++q) {
      HIPCHK(hipMemcpyAsync(aux, f + (size_t)q * N, N * 8, hipMemcpyHostToDevice, L->stream));
      HIPCHK(launch_accum(L->stream, aux_blocks(N), N, q == 0, aux, aux + N));
      HIPCHK(hipStreamSynchronize(L->stream));
    }
    HIPCHK(launch_set_ref(L->stream, aux_blocks(N), L->kp_dev, (int)(L->t & 1), aux + N));
  }
  for (int q = 0; q < L->lay.Q; ++q) {
    HIPCHK(hipMemcpyAsync(aux, f + (size_t)q * N, N * 8, hipMemcpyHostToDevice, L->stream));
    int st = run_aux(L, AUX_WRITE_POP, q, aux, nullptr, nullptr, nullptr);
    if (st) return st;
    HIPCHK(hipStreamSynchronize(L->stream));
  }
  return PLBM_OK;
}

int plbm_get_time(plbm_lattice* L, int64_t* t) {
  if (check_lat(L)) return PLBM_E_INVALID;
  if (!t) return set_error(PLBM_E_INVALID, "null output");
  *t = L->t;
  return PLBM_OK;
}

}  // extern "C"

namespace {

void fill_diag(plbm_lattice* L, const RedRec& r, plbm_diag* out) {
  std::memset(out, 0, sizeof(*out));
  out->mass = r.mass_s + r.mass_c;
  out->mass_comp_err = std::fabs(r.mass_c);
  for (int a = 0; a < 3; ++a) out->momentum[a] = r.mom[a];
  out->max_u = r.max_u;
  out->max_du_per_step = (L->has_red && L->t > L->t_red) ? r.max_du / (double)(L->t - L->t_red) : 0.0;
  out->time = L->t;
  out->flags = (int)r.flags;
  L->t_red = L->t;
  L->has_red = true;
}

}  // namespace

extern "C" {

int plbm_reduce(plbm_lattice* L, plbm_diag* out) {
  if (check_lat(L)) return PLBM_E_INVALID;
  if (!out) return set_error(PLBM_E_INVALID, "null output");
  int st = run_step_kernel(L, MODE_REDUCE, (int)(L->t & 1), nullptr, nullptr);
  if (st) return st;
  RedRec* fin = reinterpret_cast<RedRec*>(L->mem + L->lay.red) + L->lay.ntiles;
  HIPCHK(launch_reduce_final(L->stream, L->kp_dev, reduce_records(L), fin, nullptr));
  RedRec r;
  HIPCHK(hipMemcpyAsync(&r, fin, sizeof(r), hipMemcpyDeviceToHost, L->stream));
  HIPCHK(hipStreamSynchronize(L->stream));
  fill_diag(L, r, out);
  if (out->flags & (PLBM_FLAG_NAN | PLBM_FLAG_RHO_NONPOS))
    return set_error(PLBM_E_UNSTABLE, "lattice unstable (flags 0x%x at t = %lld)", out->flags, (long long)L->t);
  return PLBM_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Reductions without a workspace in the lattice's buffer: the tile records
// and the final record live in a file-scope device array, one per GPU (each
// device holds its own copy at its own address, kept until the process
// ends).  Every tile record is written before it is read, so nothing in it
// needs clearing between calls; calls that overlap on one GPU (two streams)
// race on it.

namespace {

constexpr int kScratchRecs = 1 << 15;  // 32 768 records of 64 bytes: 2 MiB per GPU
static __device__ __align__(256) RedRec scratch[kScratchRecs];

std::mutex g_scratch_mu;
std::vector<void*> g_scratch_ptr;  // device address of scratch, by device ordinal

// Device address of this device's scratch array (looked up once per device,
// with that device current).
int scratch_address(void** out) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if ((int)g_scratch_ptr.size() <= dev) g_scratch_ptr.resize(dev + 1, nullptr);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return set_error(PLBM_E_DEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return PLBM_OK;
}

}  // namespace

extern "C" {

int plbm_reduce_static(plbm_lattice* L, plbm_diag* out) {
  if (check_lat(L)) return PLBM_E_INVALID;
  if (!out) return set_error(PLBM_E_INVALID, "null output");
  const int ntiles = reduce_records(L);
  if (ntiles + 1 > kScratchRecs)
    return set_error(PLBM_E_NOMEM,
                     "plbm_reduce_static: the lattice has %d tiles, the static workspace holds %d (use plbm_reduce)",
                     ntiles, kScratchRecs - 1);
  void* sp = nullptr;
  int st = scratch_address(&sp);
  if (st) return st;
  st = run_step_kernel(L, MODE_REDUCE, (int)(L->t & 1), nullptr, nullptr, sp);
  if (st) return st;
  RedRec* fin = reinterpret_cast<RedRec*>(sp) + ntiles;
  HIPCHK(launch_reduce_final(L->stream, L->kp_dev, ntiles, fin, sp));
  RedRec r;
  HIPCHK(hipMemcpyAsync(&r, fin, sizeof(r), hipMemcpyDeviceToHost, L->stream));
  HIPCHK(hipStreamSynchronize(L->stream));
  fill_diag(L, r, out);
  if (out->flags & (PLBM_FLAG_NAN | PLBM_FLAG_RHO_NONPOS))
    return set_error(PLBM_E_UNSTABLE, "lattice unstable (flags 0x%x at t = %lld)", out->flags, (long long)L->t);
  return PLBM_OK;
}

void plbm_destroy(plbm_lattice* L) {
  if (!L) return;
  if (L->batch) batch_forget(L->batch, L->slot);  // leaves the batch it was attached to
  if (L->has_graph) {
    (void)hipGraphExecDestroy(L->graph2);
    if (long_steps() > 0) (void)hipGraphExecDestroy(L->graphL);
  }
  delete L;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// continuous batching

struct plbm_batch {
  int max_slots;
  int64_t max_tiles;
  char* mem;
  hipStream_t stream;
  KParams* slots_dev;
  WorkItem* work_dev;
  char* red_dev;  // max_slots final reduction records
  std::vector<plbm_lattice*> lat;
  struct Group {
    int lattice, coll, storage, walls, aa, wb;
    int offset, count;  // segment of the work table
  };
  std::vector<Group> groups;
  std::vector<KParams> slots_host;
  std::vector<WorkItem> work_host;
  int64_t g;  // steps since the last rebuild
  bool dirty;
  hipGraphExec_t graph2;  // two steps (phase 0, phase 1)
  hipGraphExec_t graphL;  // long_steps() steps from phase 0
  bool has_graph;
};

namespace {

// Batch device buffer: the slots' kernel parameters, the work table, and one
// final reduction record per slot.
uint64_t batch_layout(int max_slots, int64_t max_tiles, uint64_t* off_work, uint64_t* off_red) {
  uint64_t off = align_up((uint64_t)max_slots * sizeof(KParams));
  *off_work = off;
  off = align_up(off + (uint64_t)max_tiles * sizeof(WorkItem));
  *off_red = off;
  off = align_up(off + (uint64_t)max_slots * sizeof(RedRec));
  return off;
}

}  // namespace

static void batch_forget(plbm_batch* b, int32_t slot) {
  b->lat[slot] = nullptr;
  b->dirty = true;
}

namespace {

int batch_rebuild(plbm_batch* b) {
  if (!b->dirty) return PLBM_OK;
  if (b->has_graph) {
    (void)hipGraphExecDestroy(b->graph2);
    if (long_steps() > 0) (void)hipGraphExecDestroy(b->graphL);
    b->has_graph = false;
  }
  b->groups.clear();
  b->work_host.clear();
  std::map<std::tuple<int, int, int, int, int, int>, std::vector<int>> by_type;
  for (int s = 0; s < b->max_slots; ++s) {
    plbm_lattice* L = b->lat[s];
    if (!L) {
      b->slots_host[s] = KParams{};  // no lattice: ntiles = 0, never dereferenced
      continue;
    }
    KParams k = L->kp;
    k.parity = (int)(L->t & 1);
    b->slots_host[s] = k;
    by_type[std::make_tuple(L->desc.lattice, L->desc.collision, L->desc.storage, L->kp.bb_z, L->kp.aa, L->kp.wb)]
        .push_back(s);
  }
  for (auto& kv : by_type) {
    plbm_batch::Group gr;
    gr.lattice = std::get<0>(kv.first);
    gr.coll = std::get<1>(kv.first);
    gr.storage = std::get<2>(kv.first);
    gr.walls = std::get<3>(kv.first);
    gr.aa = std::get<4>(kv.first);
    gr.wb = std::get<5>(kv.first);
    gr.offset = (int)b->work_host.size();
    for (int s : kv.second)
      for (int t = 0; t < b->lat[s]->lay.ntiles; ++t) b->work_host.push_back(WorkItem{s, t});
    gr.count = (int)b->work_host.size() - gr.offset;
    b->groups.push_back(gr);
  }
  if ((int64_t)b->work_host.size() > b->max_tiles)
    return set_error(PLBM_E_NOMEM, "batch work table holds %lld tiles, %zu needed", (long long)b->max_tiles,
                     b->work_host.size());
  HIPCHK(hipMemcpyAsync(b->slots_dev, b->slots_host.data(), sizeof(KParams) * b->max_slots, hipMemcpyHostToDevice,
                        b->stream));
  if (!b->work_host.empty())
    HIPCHK(hipMemcpyAsync(b->work_dev, b->work_host.data(), sizeof(WorkItem) * b->work_host.size(),
                          hipMemcpyHostToDevice, b->stream));
  HIPCHK(hipStreamSynchronize(b->stream));
  b->g = 0;
  b->dirty = false;
  return PLBM_OK;
}

int batch_launch(plbm_batch* b, int mode, int phase) {
  for (auto& gr : b->groups) {
    StepLaunch a{};
    a.lattice = gr.lattice;
    a.coll = gr.coll;
    a.mode = mode;
    a.walls = gr.walls;
    a.aa = gr.aa;
    a.wb = gr.wb;
    a.psplit = psi_split(gr.storage);
    a.nblocks = gr.count;
    a.stream = b->stream;
    a.P = b->slots_dev;
    a.work = b->work_dev + gr.offset;
    a.nwork = gr.count;
    a.phase = phase;
    plbm_lattice_desc d{};
    d.storage = gr.storage;
    HIPCHK(launch_step(d, a));
  }
  return PLBM_OK;
}

}  // namespace

extern "C" {

int plbm_batch_bytes(int32_t max_slots, int64_t max_tiles, uint64_t* bytes) {
  if (max_slots < 1 || max_tiles < 1 || !bytes) return set_error(PLBM_E_INVALID, "bad batch sizes");
  uint64_t ow, orr;
  *bytes = batch_layout(max_slots, max_tiles, &ow, &orr);
  return PLBM_OK;
}

int plbm_batch_create(int32_t max_slots, int64_t max_tiles, void* dev_mem, uint64_t dev_bytes, void* hip_stream,
                      plbm_batch** out) {
  if (!out || max_slots < 1 || max_tiles < 1 || !dev_mem) return set_error(PLBM_E_INVALID, "bad batch arguments");
  if (((uintptr_t)dev_mem) % kAlign) return set_error(PLBM_E_INVALID, "device memory must be 256-byte aligned");
  uint64_t ow, orr;
  uint64_t need = batch_layout(max_slots, max_tiles, &ow, &orr);
  if (dev_bytes < need) return set_error(PLBM_E_NOMEM, "batch needs %llu bytes", (unsigned long long)need);
  plbm_batch* b = new plbm_batch();
  b->max_slots = max_slots;
  b->max_tiles = max_tiles;
  b->mem = static_cast<char*>(dev_mem);
  b->stream = static_cast<hipStream_t>(hip_stream);
  b->slots_dev = reinterpret_cast<KParams*>(b->mem);
  b->work_dev = reinterpret_cast<WorkItem*>(b->mem + ow);
  b->red_dev = b->mem + orr;
  b->lat.assign(max_slots, nullptr);
  b->slots_host.assign(max_slots, KParams{});
  b->g = 0;
  b->dirty = true;
  b->has_graph = false;
  *out = b;
  return PLBM_OK;
}

int plbm_batch_attach(plbm_batch* b, plbm_lattice* L, int32_t* slot) {
  if (!b || !L || !slot) return set_error(PLBM_E_INVALID, "null argument");
  if (L->batch) return set_error(PLBM_E_INVALID, "lattice already attached to a batch");
  for (int s = 0; s < b->max_slots; ++s) {
    if (!b->lat[s]) {
      b->lat[s] = L;
      b->dirty = true;
      L->batch = b;
      L->slot = s;
      *slot = s;
      return PLBM_OK;
    }
  }
  return set_error(PLBM_E_NOMEM, "no free batch slot");
}

int plbm_batch_detach(plbm_batch* b, int32_t slot) {
  if (!b || slot < 0 || slot >= b->max_slots || !b->lat[slot]) return set_error(PLBM_E_INVALID, "bad slot");
  // the lattice keeps its own time; its standalone kernel block has parity 0
  b->lat[slot]->batch = nullptr;
  b->lat[slot]->slot = -1;
  b->lat[slot] = nullptr;
  b->dirty = true;
  return PLBM_OK;
}

int plbm_batch_step(plbm_batch* b, int64_t n) {
  if (!b || n < 0) return set_error(PLBM_E_INVALID, "bad batch step");
  int st = batch_rebuild(b);
  if (st) return st;
  if (b->groups.empty()) return PLBM_OK;
  const int64_t n0 = n;
  if (n >= 4 && b->stream != nullptr && graphs_enabled()) {
    if (!b->has_graph) {
      auto launch = [b](int phase) { return batch_launch(b, MODE_STEP, phase); };
      int s1 = capture_steps(b->stream, 2, launch, &b->graph2);
      if (s1) return s1;
      if (long_steps() > 0) {
        s1 = capture_steps(b->stream, long_steps(), launch, &b->graphL);
        if (s1) {
          (void)hipGraphExecDestroy(b->graph2);
          return s1;
        }
      }
      b->has_graph = true;
    }
    if (b->g & 1) {
      st = batch_launch(b, MODE_STEP, 1);
      if (st) return st;
      ++b->g;
      --n;
    }
    for (const int m = long_steps(); m > 0 && n >= m; n -= m) {
      HIPCHK(hipGraphLaunch(b->graphL, b->stream));
      b->g += m;
    }
    for (; n >= 2; n -= 2) {
      HIPCHK(hipGraphLaunch(b->graph2, b->stream));
      b->g += 2;
    }
  }
  for (; n > 0; --n) {
    st = batch_launch(b, MODE_STEP, (int)(b->g & 1));
    if (st) return st;
    ++b->g;
  }
  for (int s = 0; s < b->max_slots; ++s)
    if (b->lat[s]) b->lat[s]->t += n0;
  return PLBM_OK;
}

int plbm_batch_diag(plbm_batch* b, plbm_diag* per_slot) {
  if (!b || !per_slot) return set_error(PLBM_E_INVALID, "null argument");
  int st = batch_rebuild(b);
  if (st) return st;
  std::memset(per_slot, 0, sizeof(plbm_diag) * b->max_slots);
  st = batch_launch(b, MODE_REDUCE, (int)(b->g & 1));
  if (st) return st;
  // one launch combines every slot's tile records, one copy brings them back
  std::vector<RedRec> recs(b->max_slots);
  HIPCHK(launch_reduce_final_batch(b->stream, b->slots_dev, b->max_slots, b->red_dev));
  HIPCHK(hipMemcpyAsync(recs.data(), b->red_dev, sizeof(RedRec) * b->max_slots, hipMemcpyDeviceToHost, b->stream));
  HIPCHK(hipStreamSynchronize(b->stream));
  for (int s = 0; s < b->max_slots; ++s)
    if (b->lat[s]) fill_diag(b->lat[s], recs[s], &per_slot[s]);
  return PLBM_OK;
}

void plbm_batch_destroy(plbm_batch* b) {
  if (!b) return;
  for (int s = 0; s < b->max_slots; ++s)
    if (b->lat[s]) {
      b->lat[s]->batch = nullptr;
      b->lat[s]->slot = -1;
    }
  if (b->has_graph) {
    (void)hipGraphExecDestroy(b->graph2);
    if (long_steps() > 0) (void)hipGraphExecDestroy(b->graphL);
  }
  delete b;
}

}  // extern "C"
