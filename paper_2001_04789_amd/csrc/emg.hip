// Host runtime and C ABI of the gfx950 multigrid elasticity solver.
//
// A problem owns its multigrid hierarchy in HBM (levels 0, -1, -2, ... of
// Sec. 3.1), one HIP stream, and HIP graphs of whole cycles.  The solve loop
// replays a graph of `check_every` cycles; the first Jacobi sweep of each
// cycle also produces the residual norm of the incoming iterate, and a
// one-block check kernel decides convergence on the device, so cycles queued
// after convergence return at once and the host reads a 64-byte control
// block once per replay.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <type_traits>
#include <utility>
#include <vector>

#include "../../include/emg.h"
#include "emg_kernels.hpp"

using namespace emg;

// Device scratch of the allocation-free batched solve: the work lists of one
// batch.  Each GPU holds its own copy from module load to process end.  In
// host code `scratch` only names the symbol; its device address on the
// current GPU comes from hipGetSymbolAddress (see noalloc_scratch below).
static __device__ __align__(256) unsigned char scratch[EMG_NOALLOC_SCRATCH_BYTES];

namespace {

thread_local std::string g_err;

emg_status fail(emg_status s, const std::string &msg) {
  g_err = msg;
  return s;
}

#define HIPCK(call)                                                                                  \
  do {                                                                                               \
    hipError_t e_ = (call);                                                                          \
    if (e_ != hipSuccess)                                                                            \
      return fail(EMG_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_));                   \
  } while (0)

constexpr int kMaxBottom = 1536;
// Stored nodes per level (box) at most: the interior kernels index nodes and
// form byte offsets of 8-byte values in 32 bits.
constexpr long long kMaxNodes = 1LL << 29;

template <class F>
void dispatch(int D, int K, F &&f) {
  if (D == 2 && K == MOD_ISO) f(std::integral_constant<int, 2>{}, std::integral_constant<int, MOD_ISO>{});
  else if (D == 2) f(std::integral_constant<int, 2>{}, std::integral_constant<int, MOD_ANISO>{});
  else if (K == MOD_ISO) f(std::integral_constant<int, 3>{}, std::integral_constant<int, MOD_ISO>{});
  else f(std::integral_constant<int, 3>{}, std::integral_constant<int, MOD_ANISO>{});
}

dim3 grid_of(const Geom &g) { return dim3((g.m[0] + BX - 1) / BX, (g.m[1] + BY - 1) / BY, g.m[2]); }
const dim3 kBlock(BX, BY, 1);

struct Level {
  Geom g{};
  double *C64 = nullptr;
  float *C32 = nullptr;
  double *u64[2] = {nullptr, nullptr};
  double *f64 = nullptr, *r64 = nullptr;
  float *u32[2] = {nullptr, nullptr};
  float *f32 = nullptr, *r32 = nullptr;
  const unsigned char *vm = nullptr;   // refined AMR level: valid-node mask (masked tile passes)
  const int *act_st = nullptr;         //   interior tiles of the stencil split holding valid nodes or ghosts
  long long nact_st = 0;
  const int *act_gr = nullptr;         //   grid_of tiles holding valid nodes or ghosts
  long long nact_gr = 0;
};

// One refined AMR level: valid nodes = the union of `boxes`, stored over
// their bounding box b grown by one node, with the valid-node mask vm.
struct Fine {
  Geom g{};
  Box b{};
  std::vector<Box> boxes;
  std::vector<unsigned char> hmask;   // host copy of vm (nesting checks of the next level)
  unsigned char *vm = nullptr;
  int *act_st = nullptr, *act_gr = nullptr;   // active tiles (see Level)
  long long nact_st = 0, nact_gr = 0;
  double *sig = nullptr;              // stress output buffer (allocated on first use)
  long long nvalid = 0, ncov = 0;     // valid nodes; coarse nodes they cover
  double *C = nullptr, *eps = nullptr, *body = nullptr;
  double *f = nullptr, *u = nullptr, *rr = nullptr, *t = nullptr;
  double *e[2] = {nullptr, nullptr};
  // FP32 correction cycle of mixed precision: moduli copy, residual, scratch, corrections
  float *C32 = nullptr, *rr32 = nullptr, *t32 = nullptr;
  float *e32[2] = {nullptr, nullptr};
  bool moduli_set = false;
};

}  // namespace

struct emg_ctx {
  int device = 0;
  size_t budget = 0;
  size_t in_use = 0;
  int live = 0;            // problems and servers created on this context and not yet destroyed
  bool closing = false;    // emg_ctx_destroy called while some were live: freed with the last one
  std::mutex mu;
};

namespace {
// Drop one live object of the context; frees it if it was closed meanwhile.
void ctx_release(emg_ctx *c) {
  bool last = false;
  {
    std::lock_guard<std::mutex> lk(c->mu);
    last = --c->live == 0 && c->closing;
  }
  if (last) delete c;
}
}  // namespace

struct emg_problem {
  emg_ctx *ctx = nullptr;
  emg_domain dom{};
  int D = 3, K = MOD_ISO, nc = 2, ne = 6;
  std::vector<Level> lv;
  double *eps = nullptr, *body = nullptr, *face[6] = {nullptr};
  double *Ainv = nullptr;
  int nbot = 0;
  double *partial = nullptr;
  long long npartial = 0;
  Ctl *ctl = nullptr;
  Ctl *ctl_host = nullptr;
  int *status = nullptr;
  double *sig = nullptr, *svm = nullptr;   // stress (Voigt) and von Mises output buffers
  hipStream_t own = nullptr, stream = nullptr;
  bool moduli_set = false, setup_done = false, mixed_ready = false, rhs_ready = false;
  // launch variants under measurement by emg_autotune (-1: none): stencil
  // pass (z-march chunks > 0, tile kernel 0, other tile shapes -shape),
  // restriction and interpolation tile shapes
  bool force_stencil = false;
  int force_v = 0, force_rs = -1, force_ps = -1;
  int force_tail = -1;   // fused-tail depth under measurement (-1: none)
  int inner = 1;        // FP32 cycles per mixed refinement step (set by emg_solve for its duration)
  std::vector<void *> allocs;
  size_t bytes = 0;
  size_t accounted = 0;   // bytes charged to the context's HBM budget
  bool counted = false;   // counted in the context's live objects
  // graph cache: key = (precision, cycles per replay, nu1, nu2, cycle type, omega)
  struct GraphEntry {
    int prec, k, nu1, nu2, fcyc, inner;
    double omega;
    hipGraphExec_t exec;
  };
  std::vector<GraphEntry> graphs;
  // step lists of the fused coarse tail (device BLists, one per precision,
  // smoothing counts, cycle type and first tail level; kept until destroy:
  // captured graphs hold their addresses)
  struct TailList {
    int rbytes, nu1, nu2, fcyc, start, res;
    const BList *dev;
  };
  std::vector<TailList> tails;
  // block-structured AMR: refined levels 1.. (empty = single level)
  std::vector<Fine> fine;
  double *amr_u0 = nullptr, *amr_f0 = nullptr, *amr_partial = nullptr;
  long long amr_nparts = 0;
};

namespace {

template <typename T>
emg_status dalloc(emg_problem *p, T **out, size_t count) {
  void *ptr = nullptr;
  const size_t b = std::max<size_t>(count, 1) * sizeof(T);
  hipError_t e = hipMalloc(&ptr, b);
  if (e != hipSuccess) return fail(EMG_ENOMEM, std::string("hipMalloc failed: ") + hipGetErrorString(e));
  p->allocs.push_back(ptr);
  p->bytes += b;
  *out = static_cast<T *>(ptr);
  return EMG_OK;
}

#define TRY(x)                    \
  do {                            \
    emg_status s_ = (x);          \
    if (s_ != EMG_OK) return s_;  \
  } while (0)

bool can_coarsen(const Geom &g) {
  for (int a = 0; a < g.dim; a++) {
    if (g.per[a]) {
      if (g.m[a] % 2 || g.m[a] < 8) return false;
    } else {
      const int cells = g.m[a] - 1;
      if (cells % 2 || cells < 8) return false;
    }
  }
  return true;
}

Geom coarse_of(const Geom &g) {
  Geom c = g;
  for (int a = 0; a < g.dim; a++) {
    c.m[a] = g.per[a] ? g.m[a] / 2 : (g.m[a] - 1) / 2 + 1;
    c.h[a] = 2.0 * g.h[a];
  }
  c.N = (long long)c.m[0] * c.m[1] * c.m[2];
  c.SC = moduli_stride(c.N);
  return c;
}

// workgroups of a grid_of launch / of a stencil pass (one norm partial each)
long long grid_blocks(const Geom &g) {
  dim3 gr = grid_of(g);
  return (long long)gr.x * gr.y * gr.z;
}
long long stencil_blocks(const Geom &g) { return split_of(g).blocks; }

// ---- kernel launch helpers (all on the problem's stream) ----

template <typename R>
const R *moduli(const Level &L) {
  if constexpr (std::is_same<R, double>::value) return L.C64;
  else return L.C32;
}

// ---- autotuner table ----
// Measured stencil-pass choice per device architecture, precision, level
// extents and periodic axes: chunks per column of the z-marching pass, 0 for
// the tile kernel.  emg_autotune fills it; zm_plan reads it before the cost
// model.  With EMG_TUNE_CACHE naming a file, the table is read from it at
// first use and written back after each tuning call (a flat JSON object).
struct TuneTable {
  std::mutex mu;
  std::map<std::string, int> table;
  std::map<int, std::string> arch;   // device -> architecture name
  bool loaded = false;               // EMG_TUNE_CACHE read (or absent)
};
TuneTable &tune_table() {
  static TuneTable t;
  return t;
}

// Architecture name of a device ("gfx950"), queried once; caller holds the
// table's lock.  Contexts query it at creation, so lookups made while a
// stream is being captured find it cached.
const std::string &tune_arch_locked(TuneTable &t, int device) {
  auto it = t.arch.find(device);
  if (it == t.arch.end()) {
    hipDeviceProp_t prop;
    std::string name = "unknown";
    if (hipGetDeviceProperties(&prop, device) == hipSuccess) {
      name = prop.gcnArchName;
      const size_t colon = name.find(':');   // "gfx950:sramecc+:xnack-" -> "gfx950"
      if (colon != std::string::npos) name.resize(colon);
    }
    it = t.arch.emplace(device, name).first;
  }
  return it->second;
}

// Key of a level; caller holds the table's lock.  what: "" for the stencil
// pass, "/r" for the restriction from the level, "/i" for the interpolation
// onto it; isotropic levels carry "/iso".
std::string tune_key_locked(TuneTable &t, int device, int rbytes, const Geom &g, int kind = MOD_ANISO,
                            const char *what = "") {
  const std::string &arch = tune_arch_locked(t, device);
  char buf[192];
  snprintf(buf, sizeof buf, "%s/%s/%dx%dx%d/p%d%s%s", arch.c_str(), rbytes == 8 ? "fp64" : "fp32", g.m[0], g.m[1],
           g.m[2], g.per[0] | (g.per[1] << 1) | (g.per[2] << 2), kind == MOD_ISO ? "/iso" : "", what);
  return buf;
}

// Reads EMG_TUNE_CACHE once: every "key": integer pair of the file (keys
// hold no quotes); anything else is skipped.  Caller holds the lock.
void tune_load_locked(TuneTable &t) {
  if (t.loaded) return;
  t.loaded = true;
  const char *path = getenv("EMG_TUNE_CACHE");
  if (!path || !*path) return;
  FILE *fp = fopen(path, "r");
  if (!fp) return;
  std::string s;
  char buf[4096];
  size_t n;
  while ((n = fread(buf, 1, sizeof buf, fp)) > 0) s.append(buf, n);
  fclose(fp);
  size_t i = 0;
  while ((i = s.find('"', i)) != std::string::npos) {
    const size_t j = s.find('"', i + 1);
    if (j == std::string::npos) break;
    const std::string key = s.substr(i + 1, j - i - 1);
    size_t k = j + 1;
    while (k < s.size() && (s[k] == ' ' || s[k] == '\t' || s[k] == '\n' || s[k] == '\r')) k++;
    i = j + 1;
    if (k < s.size() && s[k] == ':') {
      const char *a = s.c_str() + k + 1;
      char *end = nullptr;
      const long v = strtol(a, &end, 10);
      if (end != a && v >= -(TS_COUNT - 1) && v <= 4096) t.table[key] = (int)v;
    }
  }
}

// Writes the table to EMG_TUNE_CACHE (through a temporary file renamed over
// it); false if the file cannot be written.  Caller holds the lock.
bool tune_save_locked(const TuneTable &t) {
  const char *path = getenv("EMG_TUNE_CACHE");
  if (!path || !*path) return true;
  const std::string tmp = std::string(path) + ".tmp";
  FILE *fp = fopen(tmp.c_str(), "w");
  if (!fp) return false;
  fputs("{\n", fp);
  size_t i = 0;
  for (const auto &e : t.table)
    fprintf(fp, "  \"%s\": %d%s\n", e.first.c_str(), e.second, ++i < t.table.size() ? "," : "");
  fputs("}\n", fp);
  const bool ok = fclose(fp) == 0;
  return ok && rename(tmp.c_str(), path) == 0;
}

// Stencil-pass variants: the z-marching pass needs a workgroup row of
// interior nodes (64 x 4 tiles fully inside the level in x and y) and at
// least 8 planes per chunk; tile shapes -1..-3; a table value outside that
// range is ignored.
bool zm_valid(const Geom &g, int nzc) {
  const Split sp = split_of(g);
  if (nzc <= 0) return nzc > -TS_COUNT;
  return g.dim == 3 && sp.inner > 0 && g.m[0] >= BX && g.m[1] >= BY && nzc >= 1 && nzc <= sp.ntz / 8;
}

bool tune_find(int device, int rbytes, const Geom &g, int *nzc, int kind = MOD_ANISO, const char *what = "") {
  TuneTable &t = tune_table();
  std::lock_guard<std::mutex> lk(t.mu);
  tune_load_locked(t);
  auto it = t.table.find(tune_key_locked(t, device, rbytes, g, kind, what));
  if (it == t.table.end()) return false;
  const bool ok = strcmp(what, "/tail") == 0 ? it->second >= 0
                 : *what                    ? (it->second >= 0 && it->second < TS_COUNT)
                                            : zm_valid(g, it->second);
  if (!ok) return false;
  *nzc = it->second;
  return true;
}

// Chunks per column of the z-marching pass for a level (0: tile kernel): the
// variant under measurement, else the tuned choice, else the cost model,
// which takes 3D levels with enough columns x chunks of >= 8 planes to give
// every CU its resident workgroups (anisotropic FP64: one per CU, FP32: two;
// isotropic, with a third of the LDS and fewer registers: twice that);
// smaller levels keep the tile kernel, which spreads them over more
// workgroups.
// The stencil-pass variant of a level: > 0 z-march chunks, 0 the tile
// kernel in 64 x 4 tiles, < 0 the tile kernel in tile shape -v.
template <typename R>
int stencil_plan(const emg_problem *p, const Geom &g) {
  if (p->force_stencil) return p->force_v;
  int tuned;
  if (tune_find(p->ctx->device, (int)sizeof(R), g, &tuned, p->K)) return tuned;
  if (p->D != 3) return 0;
  const int target = (sizeof(R) == 8 ? 256 : 512) * (p->K == MOD_ISO ? 2 : 1);
  const int nzc = zm_chunks(g, target);
  if (nzc == 0) return 0;
  const Split sp = split_of(g);
  return (long long)sp.ntx * sp.nty * nzc >= target / 2 ? nzc : 0;
}
template <typename R>
int zm_plan(const emg_problem *p, const Geom &g) {
  return std::max(0, stencil_plan<R>(p, g));
}
// Tile shape of a stencil pass on the tile kernel (TS_64x4 when z-marched).
template <typename R>
int tile_plan(const emg_problem *p, const Geom &g) {
  return std::max(0, -stencil_plan<R>(p, g));
}
// Norm-partial slots of the first sweep of a level: the tile kernel's blocks
// in its tile shape (the z-marching pass fills the 64 x 4 slots).
template <typename R>
long long plan_blocks(const emg_problem *p, const Geom &g) {
  return split_shape(g, tile_plan<R>(p, g)).blocks;
}
// Tile shape of the restriction from a level (what "/r") or of the
// interpolation onto it ("/i").
template <typename R>
int xfer_plan(const emg_problem *p, const Geom &g, bool restriction) {
  const int forced = restriction ? p->force_rs : p->force_ps;
  if (forced >= 0) return forced;
  int tuned;
  if (tune_find(p->ctx->device, (int)sizeof(R), g, &tuned, p->K, restriction ? "/r" : "/i")) return tuned;
  return TS_64x4;
}
dim3 grid_shape(const Geom &g, int s) {
  return dim3((g.m[0] + ts_x(s) - 1) / ts_x(s), (g.m[1] + ts_y(s) - 1) / ts_y(s), g.m[2]);
}
dim3 block_shape(int s) { return dim3(ts_x(s), ts_y(s), 1); }
// Calls f(integral_constant<TX>, integral_constant<TY>) for tile shape s.
template <class F>
void dispatch_shape(int s, F &&f) {
  switch (s) {
    case TS_64x2: f(std::integral_constant<int, 64>{}, std::integral_constant<int, 2>{}); break;
    case TS_128x2: f(std::integral_constant<int, 128>{}, std::integral_constant<int, 2>{}); break;
    case TS_32x8: f(std::integral_constant<int, 32>{}, std::integral_constant<int, 8>{}); break;
    default: f(std::integral_constant<int, 64>{}, std::integral_constant<int, 4>{}); break;
  }
}

template <typename R, int MODE, typename TO>
void launch_stencil(emg_problem *p, const Level &L, const R *u, const R *f, TO *out, R omega, double *partial,
                    const Ctl *ctl) {
  if constexpr (MODE != MODE_APPLY) {
    if (L.vm) {   // refined AMR level: tile kernel with the valid-node mask (no norm partials)
      dispatch(p->D, p->K, [&](auto Dc, auto Kc) {
        constexpr int D = decltype(Dc)::value, K = decltype(Kc)::value;
        const Split sp = split_of(L.g);
        hipLaunchKernelGGL((k_stencil_mask<D, K, R, MODE, TO>), dim3((unsigned)(sp.sblocks + L.nact_st)), kBlock, 0,
                           p->stream, L.g, moduli<R>(L), u, f, out, omega, L.vm, L.act_st, sp.sblocks, ctl);
      });
      return;
    }
  }
  const int nzc = zm_plan<R>(p, L.g);
  if (nzc > 0) {
    const Split sp = split_of(L.g);
    const unsigned blocks = (unsigned)((long long)sp.ntx * sp.nty * nzc + sp.sblocks);
    if (p->K == MOD_ISO)
      hipLaunchKernelGGL((k_stencil_zm<R, MODE, TO, MOD_ISO>), dim3(blocks), kBlock, 0, p->stream, L.g, moduli<R>(L),
                         u, f, out, omega, partial, ctl, nzc, (float *)nullptr, 0.0f);
    else
      hipLaunchKernelGGL((k_stencil_zm<R, MODE, TO>), dim3(blocks), kBlock, 0, p->stream, L.g, moduli<R>(L), u, f,
                         out, omega, partial, ctl, nzc, (float *)nullptr, 0.0f);
    return;
  }
  const int ts = MODE == MODE_APPLY ? TS_64x4 : tile_plan<R>(p, L.g);
  dispatch(p->D, p->K, [&](auto Dc, auto Kc) {
    constexpr int D = decltype(Dc)::value, K = decltype(Kc)::value;
    if constexpr (MODE == MODE_APPLY) {
      hipLaunchKernelGGL((k_stencil<D, K, R, MODE, TO>), dim3((unsigned)stencil_blocks(L.g)), kBlock, 0, p->stream,
                         L.g, moduli<R>(L), u, f, out, omega, partial, ctl);
    } else {
      dispatch_shape(ts, [&](auto Xc, auto Yc) {
        constexpr int TX = decltype(Xc)::value, TY = decltype(Yc)::value;
        hipLaunchKernelGGL((k_stencil<D, K, R, MODE, TO, TX, TY>), dim3((unsigned)split_tiles<TX, TY>(L.g).blocks),
                           dim3(TX, TY, 1), 0, p->stream, L.g, moduli<R>(L), u, f, out, omega, partial, ctl);
      });
    }
  });
}

template <typename R>
void launch_jacobi_zero(emg_problem *p, const Level &L, const R *f, R *out, R omega, const Ctl *ctl) {
  dispatch(p->D, p->K, [&](auto Dc, auto Kc) {
    constexpr int D = decltype(Dc)::value, K = decltype(Kc)::value;
    hipLaunchKernelGGL((k_jacobi_zero<D, K, R>), L.act_gr ? dim3((unsigned)L.nact_gr) : grid_of(L.g), kBlock, 0,
                       p->stream, L.g, moduli<R>(L), f, out, omega, ctl, L.vm, L.act_gr);
  });
}

template <typename RI, typename RO>
void launch_restrict(emg_problem *p, const Level &Lf, const Level &Lc, const RI *rf, RO *fc, const Ctl *ctl) {
  const int s = xfer_plan<RI>(p, Lf.g, true);
  dispatch_shape(s, [&](auto Xc, auto Yc) {
    constexpr int TX = decltype(Xc)::value, TY = decltype(Yc)::value;
    if (p->D == 2)
      hipLaunchKernelGGL((k_restrict<2, RI, RO, TX, TY>), grid_shape(Lc.g, s), block_shape(s), 0, p->stream, Lf.g,
                         Lc.g, rf, fc, ctl);
    else
      hipLaunchKernelGGL((k_restrict<3, RI, RO, TX, TY>), grid_shape(Lc.g, s), block_shape(s), 0, p->stream, Lf.g,
                         Lc.g, rf, fc, ctl);
  });
}

template <typename RC, typename RF>
void launch_prolong(emg_problem *p, const Level &Lc, const Level &Lf, const RC *ec, RF *uf, const Ctl *ctl) {
  const int s = xfer_plan<RF>(p, Lf.g, false);
  dispatch_shape(s, [&](auto Xc, auto Yc) {
    constexpr int TX = decltype(Xc)::value, TY = decltype(Yc)::value;
    if (p->D == 2)
      hipLaunchKernelGGL((k_prolong_add<2, RC, RF, TX, TY>), grid_shape(Lf.g, s), block_shape(s), 0, p->stream, Lc.g,
                         Lf.g, ec, uf, ctl);
    else
      hipLaunchKernelGGL((k_prolong3_lds<RC, RF, TX, TY>), grid_shape(Lf.g, s), block_shape(s), 0, p->stream, Lc.g,
                         Lf.g, ec, uf, ctl);
  });
}

template <typename RI, typename RO>
void launch_bottom(emg_problem *p, const RI *f, RO *e, const Ctl *ctl) {
  hipLaunchKernelGGL((k_bottom_solve<RI, RO>), dim3((p->nbot + 3) / 4), dim3(256), 0, p->stream, p->Ainv, p->nbot, f,
                     e, ctl);
}

template <typename A, typename B>
void launch_cast(emg_problem *p, long long n, const A *in, B *out, const Ctl *ctl) {
  const long long blocks = std::min<long long>((n + 255) / 256, 8192);
  hipLaunchKernelGGL((k_cast<A, B>), dim3((unsigned)std::max<long long>(blocks, 1)), dim3(256), 0, p->stream, n, in,
                     out, ctl);
}

template <typename T>
void launch_fill(emg_problem *p, long long n, T *out, T v) {
  const long long blocks = std::min<long long>((n + 255) / 256, 8192);
  hipLaunchKernelGGL((k_fill<T>), dim3((unsigned)std::max<long long>(blocks, 1)), dim3(256), 0, p->stream, n, out, v);
}

void launch_check(emg_problem *p, long long nparts, int ans) {
  hipLaunchKernelGGL(k_check, dim3(1), dim3(1024), 0, p->stream, p->partial, nparts, p->ctl, ans);
}

// ---- setup: coarse moduli, coarsest inverse, right-hand side ----

emg_status setup(emg_problem *p) {
  if (!p->moduli_set) return fail(EMG_ESTATE, "moduli not set");
  if (p->setup_done) return EMG_OK;
  for (auto &F : p->fine)
    if (!F.moduli_set) return fail(EMG_ESTATE, "moduli of a refined level not set");
  // coarse levels carry the average of the finer level where it exists (finest first)
  for (int k = (int)p->fine.size(); k >= 1; k--) {
    Fine &F = p->fine[k - 1];
    const Geom gc = k == 1 ? p->lv[0].g : p->fine[k - 2].g;
    const int3 co = k == 1 ? make_int3(0, 0, 0)
                           : make_int3(p->fine[k - 2].b.lo[0] - 1, p->fine[k - 2].b.lo[1] - 1,
                                       p->D == 3 ? p->fine[k - 2].b.lo[2] - 1 : 0);
    double *Cc = k == 1 ? p->lv[0].C64 : p->fine[k - 2].C;
    double *Ec = k == 1 ? p->eps : p->fine[k - 2].eps;
    const dim3 gr((F.b.hi[0] / 2 - F.b.lo[0] / 2 + BX) / BX, (F.b.hi[1] / 2 - F.b.lo[1] / 2 + BY) / BY,
                  p->D == 3 ? F.b.hi[2] / 2 - F.b.lo[2] / 2 + 1 : 1);
    if (p->D == 2) {
      hipLaunchKernelGGL((k_average_cf<2>), gr, kBlock, 0, p->stream, gc, co, F.g, F.b, F.vm, F.C, Cc, p->nc, F.g.SC, gc.SC);
      if (Ec && F.eps)
        hipLaunchKernelGGL((k_average_cf<2>), gr, kBlock, 0, p->stream, gc, co, F.g, F.b, F.vm, F.eps, Ec, p->ne, F.g.N, gc.N);
    } else {
      hipLaunchKernelGGL((k_average_cf<3>), gr, kBlock, 0, p->stream, gc, co, F.g, F.b, F.vm, F.C, Cc, p->nc, F.g.SC, gc.SC);
      if (Ec && F.eps)
        hipLaunchKernelGGL((k_average_cf<3>), gr, kBlock, 0, p->stream, gc, co, F.g, F.b, F.vm, F.eps, Ec, p->ne, F.g.N, gc.N);
    }
  }
  const int L = (int)p->lv.size();
  for (int l = 1; l < L; l++) {
    const Geom &gc = p->lv[l].g;
    const dim3 gr((gc.m[0] + BX - 1) / BX, (gc.m[1] + BY - 1) / BY, (unsigned)(gc.m[2] * p->nc));
    hipLaunchKernelGGL((k_coarsen<double>), gr, kBlock, 0, p->stream, p->lv[l - 1].g, gc, p->nc, p->lv[l - 1].C64,
                       p->lv[l].C64);
  }
  HIPCK(hipGetLastError());
  // coarsest operator: assemble [A | I], invert by blocked Gauss-Jordan with partial pivoting
  const Level &B = p->lv[L - 1];
  const int n = p->nbot;
  const int pb = n * 16 <= GJB_LDS ? 16 : 12;   // panel width (n <= kMaxBottom = GJB_LDS / 12)
  static_assert(kMaxBottom * 12 <= GJB_LDS, "coarsest level too large for a 12-column panel in LDS");
  double *M = nullptr;   // two n x 2n buffers (panels go back and forth), the panel transform, the permutation
  HIPCK(hipMallocAsync((void **)&M, sizeof(double) * (4 * (size_t)n * n + (size_t)n * pb + (n + 1) / 2), p->stream));
  double *Mb[2] = {M, M + 2 * (size_t)n * n};
  double *Np = M + 4 * (size_t)n * n;
  int *pi = (int *)(Np + (size_t)n * pb);
  dispatch(p->D, p->K, [&](auto Dc, auto Kc) {
    constexpr int D = decltype(Dc)::value, K = decltype(Kc)::value;
    hipLaunchKernelGGL((k_bottom_assemble<D, K>), dim3((n + 255) / 256, n), dim3(256), 0, p->stream, B.g, B.C64, Mb[0],
                       n);
  });
  hipLaunchKernelGGL((k_fill<int>), dim3(1), dim3(256), 0, p->stream, 1LL, p->status, 0);
  int cur = 0;
  for (int k = 0; k < n; k += pb) {
    const int b = std::min(pb, n - k);
    if (pb == 16)
      hipLaunchKernelGGL(k_gjb_panel<16>, dim3(1), dim3(1024), 0, p->stream, (const double *)Mb[cur], n, k, b, Np, pi,
                         p->status);
    else
      hipLaunchKernelGGL(k_gjb_panel<12>, dim3(1), dim3(1024), 0, p->stream, (const double *)Mb[cur], n, k, b, Np, pi,
                         p->status);
    const long long cols = 2LL * n - k - b;   // columns right of the panel
    hipLaunchKernelGGL(k_gjb_update, dim3((unsigned)((cols + 255) / 256), (unsigned)((n + GJB_ROWS - 1) / GJB_ROWS)),
                       dim3(256), 0,
                       p->stream, (const double *)Mb[cur], Mb[cur ^ 1], n, k, b, (const double *)Np, (const int *)pi);
    cur ^= 1;
  }
  hipLaunchKernelGGL(k_gj_extract, dim3((unsigned)(((long long)n * n + 255) / 256)), dim3(256), 0, p->stream,
                     Mb[cur], n, p->Ainv);
  HIPCK(hipGetLastError());
  int st = 0;
  HIPCK(hipMemcpyAsync(&st, p->status, sizeof(int), hipMemcpyDeviceToHost, p->stream));
  HIPCK(hipFreeAsync(M, p->stream));
  HIPCK(hipStreamSynchronize(p->stream));
  if (st) return fail(EMG_EINVAL, "coarsest-level operator is singular");
  p->setup_done = true;
  p->mixed_ready = false;   // the FP32 copies follow the moduli setup just wrote
  return EMG_OK;
}

emg_status ensure_mixed(emg_problem *p) {
  if (p->mixed_ready) return EMG_OK;
  size_t extra = 0;   // first use: charge the FP32 copies to the context's budget
  if (!p->lv[0].C32)
    for (auto &L : p->lv) extra += ((size_t)L.g.SC * p->nc + (size_t)L.g.N * 4 * p->D) * sizeof(float);
  for (auto &F : p->fine)
    if (!F.C32) extra += ((size_t)F.g.SC * p->nc + (size_t)F.g.N * 4 * p->D) * sizeof(float);
  if (extra && p->ctx) {
    std::lock_guard<std::mutex> lk(p->ctx->mu);
    if (p->ctx->budget && p->ctx->in_use + extra > p->ctx->budget)
      return fail(EMG_ENOMEM, "HBM budget exceeded by the FP32 copies of mixed precision");
    p->ctx->in_use += extra;
    p->accounted += extra;
  }
  for (auto &L : p->lv) {
    const long long nd = (long long)p->D * L.g.N;
    if (!L.C32) {
      TRY(dalloc(p, &L.C32, (size_t)p->nc * L.g.SC));
      TRY(dalloc(p, &L.u32[0], nd));
      TRY(dalloc(p, &L.u32[1], nd));
      TRY(dalloc(p, &L.f32, nd));
      TRY(dalloc(p, &L.r32, nd));
    }
    launch_cast<double, float>(p, (long long)p->nc * L.g.SC, L.C64, L.C32, nullptr);
  }
  for (auto &F : p->fine) {   // refined boxes: their moduli after setup's averaging
    const long long nd = (long long)p->D * F.g.N;
    if (!F.C32) {
      TRY(dalloc(p, &F.C32, (size_t)p->nc * F.g.SC));
      TRY(dalloc(p, &F.rr32, nd));
      TRY(dalloc(p, &F.t32, nd));
      TRY(dalloc(p, &F.e32[0], nd));
      TRY(dalloc(p, &F.e32[1], nd));
      for (float *a : {F.rr32, F.t32, F.e32[0], F.e32[1]}) launch_fill<float>(p, (long long)nd, a, 0.0f);
    }
    launch_cast<double, float>(p, (long long)p->nc * F.g.SC, F.C, F.C32, nullptr);
  }
  HIPCK(hipGetLastError());
  p->mixed_ready = true;
  return EMG_OK;
}

emg_status assemble_rhs(emg_problem *p) {
  if (p->rhs_ready) return EMG_OK;
  const Level &L0 = p->lv[0];
  Faces F;
  for (int f = 0; f < 6; f++) F.p[f] = p->face[f];
  Faces none;
  for (int f = 0; f < 6; f++) none.p[f] = nullptr;
  double *f0 = p->fine.empty() ? L0.f64 : p->amr_f0;
  dispatch(p->D, p->K, [&](auto Dc, auto Kc) {
    constexpr int D = decltype(Dc)::value, K = decltype(Kc)::value;
    hipLaunchKernelGGL((k_rhs<D, K>), grid_of(L0.g), kBlock, 0, p->stream, L0.g, L0.C64, p->eps, p->body, F, f0);
    for (auto &Fn : p->fine)
      hipLaunchKernelGGL((k_rhs<D, K>), grid_of(Fn.g), kBlock, 0, p->stream, Fn.g, Fn.C, Fn.eps, Fn.body, none, Fn.f);
  });
  HIPCK(hipGetLastError());
  p->rhs_ready = true;
  return EMG_OK;
}

// ---- cycles ----

template <typename R>
R *vbuf(Level &L, int b) {
  if constexpr (std::is_same<R, double>::value) return L.u64[b];
  else return L.u32[b];
}
template <typename R>
R *fbuf(Level &L) {
  if constexpr (std::is_same<R, double>::value) return L.f64;
  else return L.f32;
}
template <typename R>
R *rbuf(Level &L) {
  if constexpr (std::is_same<R, double>::value) return L.r64;
  else return L.r32;
}

template <typename R>
int coarse_correction(emg_problem *p, int l, int nu1, int nu2, R omega, bool fcyc, bool jz_done = false);

// Restriction of level l's residual to f_{l+1}; when level l+1 is not the
// bottom, fused with its first Jacobi sweep from zero (into buffer 0), and
// the callee's cycle from zero starts after that sweep.  Returns whether it
// was fused.
template <typename R>
bool restrict_down(emg_problem *p, int l, R omega, const Ctl *ctl, bool plain = false) {
  Level &Lv = p->lv[l], &Lc = p->lv[l + 1];
  if (plain || l + 1 == (int)p->lv.size() - 1) {
    launch_restrict<R, R>(p, Lv, Lc, rbuf<R>(Lv), fbuf<R>(Lc), ctl);
    return false;
  }
  const int s = xfer_plan<R>(p, Lv.g, true);
  dispatch(p->D, p->K, [&](auto Dc, auto Kc) {
    constexpr int D = decltype(Dc)::value, K = decltype(Kc)::value;
    dispatch_shape(s, [&](auto Xc, auto Yc) {
      constexpr int TX = decltype(Xc)::value, TY = decltype(Yc)::value;
      hipLaunchKernelGGL((k_restrict_jz<D, K, R, TX, TY>), grid_shape(Lc.g, s), block_shape(s), 0, p->stream, Lv.g,
                         Lc.g, (const R *)rbuf<R>(Lv), fbuf<R>(Lc), moduli<R>(Lc), vbuf<R>(Lc, 0), omega, ctl);
    });
  });
  return true;
}
template <typename R>
bool restrict_down(emg_problem *p, int l, R omega, bool plain = false) {
  return restrict_down<R>(p, l, omega, p->ctl, plain);
}

// ---- fused coarse tail (k_tail) ----
constexpr long long kTailNodes = 1024;   // levels of at most this many nodes go into the tail
constexpr int kTailGrid = 64;            // workgroups of a batched tail launch (problems grid-strided)

// Candidate depth of the fused tail: the levels below level 0 with at most
// kTailNodes nodes each, counted from the bottom, if there are at least two
// (a bottom solve alone gains nothing from fusing), else 0.
int tail_candidate(const emg_problem *p) {
  const int L = (int)p->lv.size();
  int k = 0;
  while (k < L - 1 && p->lv[L - 1 - k].g.N <= kTailNodes) k++;
  return k >= 2 ? k : 0;
}

// Levels in the fused coarse tail of a problem's cycles (0: none): the depth
// under measurement, else the table's (key of level 0 with "/tail"), else 0.
// The default is no fusion: on MI355X one workgroup walking the small levels
// (about 17 us per step, its loads not hidden by other wavefronts) is slower
// than a launch per pass spread over many CUs (5-10 us each), at every size
// measured; emg_autotune times both for a problem and records the faster.
template <typename R>
int tail_levels(const emg_problem *p) {
  const int L = (int)p->lv.size();
  if (p->force_tail >= 0) return std::min(p->force_tail, L - 1);
  int tuned;
  if (tune_find(p->ctx->device, (int)sizeof(R), p->lv[0].g, &tuned, p->K, "/tail")) return std::min(tuned, L - 1);
  return 0;
}

// Step list of the cycle on levels l.. (from zero; buffers as coarse_cycle /
// coarse_correction use them, restrictions unfused), appended to v; returns
// the buffer holding the result, as they do.
template <typename R>
int tail_cycle(emg_problem *p, int l, int nu1, int nu2, bool fcyc, int cur, std::vector<BEnt> &v);
template <typename R>
int tail_correction(emg_problem *p, int l, int nu1, int nu2, bool fcyc, std::vector<BEnt> &v) {
  if (!fcyc) return tail_cycle<R>(p, l, nu1, nu2, false, -1, v);
  const int b = tail_cycle<R>(p, l, nu1, nu2, true, -1, v);
  if (l == (int)p->lv.size() - 1) return b;
  return tail_cycle<R>(p, l, nu1, nu2, false, b, v);
}
template <typename R>
int tail_cycle(emg_problem *p, int l, int nu1, int nu2, bool fcyc, int cur, std::vector<BEnt> &v) {
  const int L = (int)p->lv.size();
  Level &Lv = p->lv[l];
  auto ent = [&](int kind, const void *a, const void *b, void *out) {
    BEnt e{};
    e.kind = kind;
    e.g = Lv.g;
    e.C = moduli<R>(Lv);
    e.a = a;
    e.b = b;
    e.out = out;
    e.ctl = p->ctl;
    return e;
  };
  if (l == L - 1) {
    BEnt e = ent(BK_BOTTOM, fbuf<R>(Lv), nullptr, vbuf<R>(Lv, 0));
    e.Ainv = p->Ainv;
    e.nbot = p->nbot;
    v.push_back(e);
    return 0;
  }
  int s0 = 0;
  if (cur < 0) {
    v.push_back(ent(BK_JZERO, fbuf<R>(Lv), nullptr, vbuf<R>(Lv, 0)));
    cur = 0;
    s0 = 1;
  }
  for (int s = s0; s < nu1; s++, cur ^= 1) v.push_back(ent(BK_JACOBI, vbuf<R>(Lv, cur), fbuf<R>(Lv), vbuf<R>(Lv, cur ^ 1)));
  v.push_back(ent(BK_RESID, vbuf<R>(Lv, cur), fbuf<R>(Lv), rbuf<R>(Lv)));
  Level &Lc = p->lv[l + 1];
  BEnt r = ent(BK_RESTRICT, rbuf<R>(Lv), nullptr, fbuf<R>(Lc));
  r.g2 = Lc.g;
  v.push_back(r);
  const int cb = tail_correction<R>(p, l + 1, nu1, nu2, fcyc, v);
  BEnt q = ent(BK_PROLONG, vbuf<R>(Lc, cb), nullptr, vbuf<R>(Lv, cur));
  q.g2 = Lc.g;
  v.push_back(q);
  for (int s = 0; s < nu2; s++, cur ^= 1) v.push_back(ent(BK_JACOBI, vbuf<R>(Lv, cur), fbuf<R>(Lv), vbuf<R>(Lv, cur ^ 1)));
  return cur;
}

// The problem's tail list for the current choice if the cycle's level l
// starts the tail and the list was prepared, else null (per-launch path).
template <typename R>
const emg_problem::TailList *tail_at(const emg_problem *p, int l, int nu1, int nu2, bool fcyc) {
  const int k = tail_levels<R>(p);
  if (k == 0 || l != (int)p->lv.size() - k) return nullptr;
  for (auto &t : p->tails)
    if (t.rbytes == (int)sizeof(R) && t.start == l && t.nu1 == nu1 && t.nu2 == nu2 && t.fcyc == (int)fcyc) return &t;
  return nullptr;
}

// Builds and uploads the tail list for the current choice (not while a
// stream is captured: it allocates and copies).
template <typename R>
emg_status prepare_tail(emg_problem *p, int nu1, int nu2, bool fcyc) {
  const int k = tail_levels<R>(p);
  if (k == 0) return EMG_OK;
  const int start = (int)p->lv.size() - k;
  if (tail_at<R>(p, start, nu1, nu2, fcyc)) return EMG_OK;
  std::vector<BEnt> v;
  const int res = tail_correction<R>(p, start, nu1, nu2, fcyc, v);
  std::vector<char> host(blist_bytes((int)v.size()), 0);
  BList *h = (BList *)host.data();
  h->n = (int)v.size();
  h->total = 1;   // one problem, tile0 = 0
  for (size_t j = 0; j < v.size(); j++) h->e[j] = v[j];
  char *dev = nullptr;
  TRY(dalloc(p, &dev, host.size()));
  HIPCK(hipMemcpyAsync(dev, host.data(), host.size(), hipMemcpyHostToDevice, p->stream));
  HIPCK(hipStreamSynchronize(p->stream));
  p->tails.push_back({(int)sizeof(R), nu1, nu2, (int)fcyc, start, res, (const BList *)dev});
  return EMG_OK;
}

template <typename R>
void launch_tail(emg_problem *p, const BList *L, R omega, unsigned grid) {
  dispatch(p->D, p->K, [&](auto Dc, auto Kc) {
    constexpr int D = decltype(Dc)::value, K = decltype(Kc)::value;
    hipLaunchKernelGGL((k_tail<D, K, R>), dim3(grid), dim3(TL_THREADS), 0, p->stream, L, omega);
  });
}

// Cycle on level l for the correction of the right-hand side f_l: from zero
// (cur < 0; the first sweep is the zero-start sweep) or from the iterate in
// ping-pong buffer cur.  The coarse correction is a V-cycle from zero, or
// with fcyc an F-cycle from zero followed by a V-cycle from its result, so
// with fcyc and cur < 0 this is the F-cycle on level l.  The bottom level is
// solved exactly whatever the start.  Returns the buffer holding the result.
template <typename R>
int coarse_cycle(emg_problem *p, int l, int nu1, int nu2, R omega, bool fcyc, int cur = -1, bool jz_done = false) {
  const int L = (int)p->lv.size();
  Level &Lv = p->lv[l];
  if (l == L - 1) {
    launch_bottom<R, R>(p, fbuf<R>(Lv), vbuf<R>(Lv, 0), p->ctl);
    return 0;
  }
  int s0 = 0;
  if (cur < 0) {
    if (!jz_done) launch_jacobi_zero<R>(p, Lv, fbuf<R>(Lv), vbuf<R>(Lv, 0), omega, p->ctl);
    cur = 0;
    s0 = 1;
  }
  for (int s = s0; s < nu1; s++) {
    launch_stencil<R, MODE_JACOBI, R>(p, Lv, vbuf<R>(Lv, cur), fbuf<R>(Lv), vbuf<R>(Lv, cur ^ 1), omega, nullptr, p->ctl);
    cur ^= 1;
  }
  launch_stencil<R, MODE_RESID, R>(p, Lv, vbuf<R>(Lv, cur), fbuf<R>(Lv), rbuf<R>(Lv), omega, nullptr, p->ctl);
  const bool jz = restrict_down<R>(p, l, omega, tail_at<R>(p, l + 1, nu1, nu2, fcyc) != nullptr);
  const int cb = coarse_correction<R>(p, l + 1, nu1, nu2, omega, fcyc, jz);
  launch_prolong<R, R>(p, p->lv[l + 1], Lv, vbuf<R>(p->lv[l + 1], cb), vbuf<R>(Lv, cur), p->ctl);
  for (int s = 0; s < nu2; s++) {
    launch_stencil<R, MODE_JACOBI, R>(p, Lv, vbuf<R>(Lv, cur), fbuf<R>(Lv), vbuf<R>(Lv, cur ^ 1), omega, nullptr, p->ctl);
    cur ^= 1;
  }
  return cur;
}

// Correction on level l >= 1 for the restricted residual in f_l: a V-cycle
// from zero, or an F-cycle from zero then a V-cycle from its result (the
// V-cycle's restriction overwrites f_{l+1}, which the F-cycle no longer
// needs; f_l itself is only read).
template <typename R>
int coarse_correction(emg_problem *p, int l, int nu1, int nu2, R omega, bool fcyc, bool jz_done) {
  if (const auto *t = tail_at<R>(p, l, nu1, nu2, fcyc)) {   // the whole correction in one launch
    launch_tail<R>(p, t->dev, omega, 1);
    return t->res;
  }
  if (!fcyc) return coarse_cycle<R>(p, l, nu1, nu2, omega, false, -1, jz_done);
  const int b = coarse_cycle<R>(p, l, nu1, nu2, omega, true, -1, jz_done);
  if (l == (int)p->lv.size() - 1) return b;   // exact bottom solve: the V-cycle would repeat it
  return coarse_cycle<R>(p, l, nu1, nu2, omega, false, b);
}

// One FP64 V-cycle on level 0 for u (buffer 0 in and out).  The first sweep
// also sums the squared residual of the incoming iterate; the check kernel
// stops the solve before the cycle changes anything if it has converged.
void record_fp64_cycle(emg_problem *p, int nu1, int nu2, double omega, bool fcyc) {
  Level &L0 = p->lv[0];
  int cur = 0;
  launch_stencil<double, MODE_JACOBI, double>(p, L0, L0.u64[0], L0.f64, L0.u64[1], omega, p->partial, p->ctl);
  launch_check(p, plan_blocks<double>(p, L0.g), 0);
  cur = 1;
  for (int s = 1; s < nu1; s++) {
    launch_stencil<double, MODE_JACOBI, double>(p, L0, L0.u64[cur], L0.f64, L0.u64[cur ^ 1], omega, nullptr, p->ctl);
    cur ^= 1;
  }
  launch_stencil<double, MODE_RESID, double>(p, L0, L0.u64[cur], L0.f64, L0.r64, omega, nullptr, p->ctl);
  const bool jz = restrict_down<double>(p, 0, omega, tail_at<double>(p, 1, nu1, nu2, fcyc) != nullptr);
  const int cb = coarse_correction<double>(p, 1, nu1, nu2, omega, fcyc, jz);
  launch_prolong<double, double>(p, p->lv[1], L0, p->lv[1].u64[cb], L0.u64[cur], p->ctl);
  for (int s = 0; s < nu2; s++) {
    launch_stencil<double, MODE_JACOBI, double>(p, L0, L0.u64[cur], L0.f64, L0.u64[cur ^ 1], omega, nullptr, p->ctl);
    cur ^= 1;
  }
  if (cur != 0) launch_cast<double, double>(p, (long long)p->D * L0.g.N, L0.u64[cur], L0.u64[0], p->ctl);
}

// Level-0 buffer (u32[b]) in which the FP32 correction cycle from zero
// leaves its result: the zero-start sweep writes buffer 0 and every further
// sweep flips the buffer (a one-level hierarchy is solved exactly into 0).
int mixed_result_buf(const emg_problem *p, int nu1, int nu2) {
  return p->lv.size() == 1 ? 0 : (nu1 - 1 + nu2) & 1;
}

// One mixed-precision refinement step: u += e (the previous FP32
// correction, zero at the start), FP64 residual written as FP32 to the
// level-0 FP32 right-hand side with its norm, convergence check, then one
// FP32 V-cycle (F-cycle with fcyc) for the new correction e, left in
// u32[mixed_result_buf()] of level 0 where the next step reads it.  With
// p->inner > 1 the further cycles continue from that correction (same FP32
// right-hand side) before the step ends.
void record_mixed_iter(emg_problem *p, int nu1, int nu2, float omega, bool fcyc) {
  Level &L0 = p->lv[0];
  const long long nd0 = (long long)p->D * L0.g.N;
  const int eb = mixed_result_buf(p, nu1, nu2);
  hipLaunchKernelGGL(k_add_correction, dim3((unsigned)std::min<long long>((nd0 + 255) / 256, 8192)), dim3(256), 0,
                     p->stream, nd0, L0.u64[0], L0.u32[eb], p->ctl);
  // on z-marching levels the residual pass also writes the FP32 cycle's
  // first sweep from zero (into u32[0]), which the cycle then skips
  const int nzc = zm_plan<double>(p, L0.g);
  if (nzc > 0) {
    const Split sp = split_of(L0.g);
    const unsigned blocks = (unsigned)((long long)sp.ntx * sp.nty * nzc + sp.sblocks);
    if (p->K == MOD_ISO)
      hipLaunchKernelGGL((k_stencil_zm<double, MODE_RESID, float, MOD_ISO>), dim3(blocks), kBlock, 0, p->stream,
                         L0.g, (const double *)L0.C64, (const double *)L0.u64[0], (const double *)L0.f64, L0.f32, 0.0,
                         p->partial, p->ctl, nzc, L0.u32[0], omega);
    else
      hipLaunchKernelGGL((k_stencil_zm<double, MODE_RESID, float>), dim3(blocks), kBlock, 0, p->stream, L0.g,
                         (const double *)L0.C64, (const double *)L0.u64[0], (const double *)L0.f64, L0.f32, 0.0,
                         p->partial, p->ctl, nzc, L0.u32[0], omega);
  } else {
    launch_stencil<double, MODE_RESID, float>(p, L0, L0.u64[0], L0.f64, L0.f32, 0.0, p->partial, p->ctl);
  }
  launch_check(p, plan_blocks<double>(p, L0.g), 0);
  int cb = coarse_cycle<float>(p, 0, nu1, nu2, omega, fcyc, -1, nzc > 0);
  for (int i = 1; i < p->inner; i++) cb = coarse_cycle<float>(p, 0, nu1, nu2, omega, fcyc, cb);
  // a continuing cycle flips the buffer nu1 + nu2 times: with an odd count
  // the correction ends in the other buffer and is moved back to u32[eb]
  if (cb != eb) launch_cast<float, float>(p, nd0, L0.u32[cb], L0.u32[eb], p->ctl);
}

// ---- AMR helpers ----
int3 parent_origin(emg_problem *p, int k) {
  if (k == 1) return make_int3(0, 0, 0);
  const Box &b = p->fine[k - 2].b;
  return make_int3(b.lo[0] - 1, b.lo[1] - 1, p->D == 3 ? b.lo[2] - 1 : 0);
}
const Geom &parent_geom(emg_problem *p, int k) { return k == 1 ? p->lv[0].g : p->fine[k - 2].g; }
dim3 covered_grid(emg_problem *p, const Box &b, int grow) {
  return dim3((b.hi[0] / 2 - b.lo[0] / 2 + 1 + 2 * grow + BX - 1) / BX,
              (b.hi[1] / 2 - b.lo[1] / 2 + 1 + 2 * grow + BY - 1) / BY,
              p->D == 3 ? b.hi[2] / 2 - b.lo[2] / 2 + 1 + 2 * grow : 1);
}
// launch grid of a refined level's active tiles (grid_of order, 1D)
dim3 act_grid(const Fine &F) { return dim3((unsigned)std::max<long long>(F.nact_gr, 1)); }
// a box level seen through the single-level launch helpers
Level box_level(const Fine &F) {
  Level L;
  L.g = F.g;
  L.C64 = F.C;
  L.C32 = F.C32;
  L.vm = F.vm;
  L.act_st = F.act_st;
  L.nact_st = F.nact_st;
  L.act_gr = F.act_gr;
  L.nact_gr = F.nact_gr;
  return L;
}

template <int D>
void amr_sync(emg_problem *p, double *u0, const Ctl *ctl) {
  const int Lf = (int)p->fine.size();
  for (int k = Lf; k >= 1; k--) {
    Fine &F = p->fine[k - 1];
    double *uc = k == 1 ? u0 : p->fine[k - 2].u;
    hipLaunchKernelGGL((k_inject<D, double>), covered_grid(p, F.b, 0), kBlock, 0, p->stream, parent_geom(p, k),
                       parent_origin(p, k), F.g, F.b, F.vm, F.u, uc, D, ctl);
  }
  for (int k = 1; k <= Lf; k++) {
    Fine &F = p->fine[k - 1];
    const double *uc = k == 1 ? u0 : p->fine[k - 2].u;
    hipLaunchKernelGGL((k_interp<D, double>), act_grid(F), kBlock, 0, p->stream, parent_geom(p, k), parent_origin(p, k),
                       F.g, F.b, F.vm, F.act_gr, uc, F.u, (double *)nullptr, 1, ctl);
  }
}

// Composite residual of the (synced) state: base rows into L0.f64, refined
// rows into each level's rr, squared-norm partials of the composite rows.
template <int D>
void amr_residual(emg_problem *p, const Ctl *ctl) {
  Level &L0 = p->lv[0];
  const int Lf = (int)p->fine.size();
  launch_stencil<double, MODE_RESID, double>(p, L0, p->amr_u0, p->amr_f0, L0.f64, 0.0, nullptr, ctl);
  long long off = 0;
  for (int k = 0; k <= Lf; k++) {
    const Geom &g = k == 0 ? L0.g : p->fine[k - 1].g;
    const double *r = k == 0 ? L0.f64 : p->fine[k - 1].rr;
    const unsigned char *own = k == 0 ? nullptr : p->fine[k - 1].vm;
    const int3 co = k == 0 ? make_int3(0, 0, 0) : parent_origin(p, k + 1);
    Geom cg{};
    Box cb{};
    const unsigned char *cvm = nullptr;
    if (k < Lf) {
      cg = p->fine[k].g;
      cb = p->fine[k].b;
      cvm = p->fine[k].vm;
    }
    if (k > 0) {
      Fine &F = p->fine[k - 1];
      launch_stencil<double, MODE_RESID, double>(p, box_level(F), F.u, F.f, F.rr, 0.0, nullptr, ctl);
    }
    hipLaunchKernelGGL((k_masked_norm<D>), grid_of(g), kBlock, 0, p->stream, g, r, own, co, cg, cb, cvm,
                       p->amr_partial + off, ctl);
    off += grid_blocks(g);
  }
}

// One composite correction cycle (Sec. 3.2): sync, composite residual and
// convergence check; down the levels: fine corrections relaxed with zero
// ghosts (the coarse/fine boundary acting as Dirichlet), coarse residual
// updated for the injected correction, fine residual restricted onto the
// covered coarse nodes; one V-cycle on the base grid; up the levels:
// interpolation onto valid and ghost nodes, relaxation with the
// interpolated ghosts as Dirichlet values; update.
template <int D>
void record_amr_cycle(emg_problem *p, int nu1, int nu2, double omega, bool fcyc) {
  Level &L0 = p->lv[0];
  const int Lf = (int)p->fine.size();
  amr_sync<D>(p, p->amr_u0, p->ctl);
  amr_residual<D>(p, p->ctl);
  hipLaunchKernelGGL(k_check, dim3(1), dim3(1024), 0, p->stream, p->amr_partial, p->amr_nparts, p->ctl, 0);
  std::vector<int> cur(Lf + 1, 0);
  for (int k = Lf; k >= 1; k--) {
    Fine &F = p->fine[k - 1];
    Level B = box_level(F);
    hipLaunchKernelGGL((k_ghost_fill<D, double>), act_grid(F), kBlock, 0, p->stream, F.g, F.vm, F.act_gr, F.rr, 0.0,
                       p->ctl);
    launch_jacobi_zero<double>(p, B, F.rr, F.e[0], omega, p->ctl);
    int c = 0;
    for (int s = 1; s < nu1; s++) {
      launch_stencil<double, MODE_JACOBI, double>(p, B, F.e[c], F.rr, F.e[c ^ 1], omega, nullptr, p->ctl);
      c ^= 1;
    }
    cur[k] = c;
    launch_stencil<double, MODE_RESID, double>(p, B, F.e[c], F.rr, F.t, 0.0, nullptr, p->ctl);
    const Geom &gc = parent_geom(p, k);
    const int3 co = parent_origin(p, k);
    double *rrc = k == 1 ? L0.f64 : p->fine[k - 2].rr;
    const double *Cc = k == 1 ? L0.C64 : p->fine[k - 2].C;
    dispatch(p->D, p->K, [&](auto Dc, auto Kc) {
      constexpr int DD = decltype(Dc)::value, K = decltype(Kc)::value;
      hipLaunchKernelGGL((k_cf_update<DD, K, double>), covered_grid(p, F.b, 1), kBlock, 0, p->stream, gc, co, F.g, F.b,
                         F.vm, Cc, (const double *)F.e[c], rrc, p->ctl);
    });
    hipLaunchKernelGGL((k_restrict_cf<D, double>), covered_grid(p, F.b, 0), kBlock, 0, p->stream, F.g, F.b, F.vm,
                       (const double *)F.t, gc, co, rrc, p->ctl);
  }
  const int cb = coarse_cycle<double>(p, 0, nu1, nu2, omega, fcyc);
  for (int k = 1; k <= Lf; k++) {
    Fine &F = p->fine[k - 1];
    Level B = box_level(F);
    const double *ec = k == 1 ? L0.u64[cb] : p->fine[k - 2].e[cur[k - 1]];
    int c = cur[k];
    hipLaunchKernelGGL((k_interp<D, double>), act_grid(F), kBlock, 0, p->stream, parent_geom(p, k), parent_origin(p, k),
                       F.g, F.b, F.vm, F.act_gr, ec, F.e[c], F.rr, 2, p->ctl);
    for (int s = 0; s < nu2; s++) {
      launch_stencil<double, MODE_JACOBI, double>(p, B, F.e[c], F.rr, F.e[c ^ 1], omega, nullptr, p->ctl);
      c ^= 1;
    }
    cur[k] = c;
  }
  const long long nd0 = (long long)p->D * L0.g.N;
  hipLaunchKernelGGL((k_axpy<double>), dim3((unsigned)std::min<long long>((nd0 + 255) / 256, 8192)), dim3(256), 0,
                     p->stream, nd0, p->amr_u0, (const double *)L0.u64[cb], p->ctl);
  for (int k = 1; k <= Lf; k++) {
    Fine &F = p->fine[k - 1];
    const long long nd = (long long)p->D * F.g.N;
    hipLaunchKernelGGL((k_axpy<double>), dim3((unsigned)std::min<long long>((nd + 255) / 256, 8192)), dim3(256), 0,
                       p->stream, nd, F.u, (const double *)F.e[cur[k]], p->ctl);
  }
}

// Mixed-precision composite cycle: the state, its sync, the composite
// residual and convergence check and the final update stay FP64; the
// correction (fine relaxations, coarse/fine residual transfer, base V-cycle
// with its FP64 bottom solve, interpolation) runs in FP32 from the residuals
// rounded to FP32 -- the iterative-refinement split of the single-level
// mixed iteration applied to the composite system.
template <int D>
void record_amr_cycle_mixed(emg_problem *p, int nu1, int nu2, float omega, bool fcyc) {
  Level &L0 = p->lv[0];
  const int Lf = (int)p->fine.size();
  amr_sync<D>(p, p->amr_u0, p->ctl);
  amr_residual<D>(p, p->ctl);
  hipLaunchKernelGGL(k_check, dim3(1), dim3(1024), 0, p->stream, p->amr_partial, p->amr_nparts, p->ctl, 0);
  launch_cast<double, float>(p, (long long)p->D * L0.g.N, L0.f64, L0.f32, p->ctl);
  for (auto &F : p->fine) launch_cast<double, float>(p, (long long)p->D * F.g.N, F.rr, F.rr32, p->ctl);
  std::vector<int> cur(Lf + 1, 0);
  for (int k = Lf; k >= 1; k--) {
    Fine &F = p->fine[k - 1];
    Level B = box_level(F);
    hipLaunchKernelGGL((k_ghost_fill<D, float>), act_grid(F), kBlock, 0, p->stream, F.g, F.vm, F.act_gr, F.rr32, 0.0f,
                       p->ctl);
    launch_jacobi_zero<float>(p, B, F.rr32, F.e32[0], omega, p->ctl);
    int c = 0;
    for (int s = 1; s < nu1; s++) {
      launch_stencil<float, MODE_JACOBI, float>(p, B, F.e32[c], F.rr32, F.e32[c ^ 1], omega, nullptr, p->ctl);
      c ^= 1;
    }
    cur[k] = c;
    launch_stencil<float, MODE_RESID, float>(p, B, F.e32[c], F.rr32, F.t32, 0.0f, nullptr, p->ctl);
    const Geom &gc = parent_geom(p, k);
    const int3 co = parent_origin(p, k);
    float *rrc = k == 1 ? L0.f32 : p->fine[k - 2].rr32;
    const float *Cc = k == 1 ? L0.C32 : p->fine[k - 2].C32;
    dispatch(p->D, p->K, [&](auto Dc, auto Kc) {
      constexpr int DD = decltype(Dc)::value, K = decltype(Kc)::value;
      hipLaunchKernelGGL((k_cf_update<DD, K, float>), covered_grid(p, F.b, 1), kBlock, 0, p->stream, gc, co, F.g, F.b,
                         F.vm, Cc, (const float *)F.e32[c], rrc, p->ctl);
    });
    hipLaunchKernelGGL((k_restrict_cf<D, float>), covered_grid(p, F.b, 0), kBlock, 0, p->stream, F.g, F.b, F.vm,
                       (const float *)F.t32, gc, co, rrc, p->ctl);
  }
  const int cb = coarse_cycle<float>(p, 0, nu1, nu2, omega, fcyc);
  for (int k = 1; k <= Lf; k++) {
    Fine &F = p->fine[k - 1];
    Level B = box_level(F);
    const float *ec = k == 1 ? L0.u32[cb] : p->fine[k - 2].e32[cur[k - 1]];
    int c = cur[k];
    hipLaunchKernelGGL((k_interp<D, float>), act_grid(F), kBlock, 0, p->stream, parent_geom(p, k), parent_origin(p, k),
                       F.g, F.b, F.vm, F.act_gr, ec, F.e32[c], F.rr32, 2, p->ctl);
    for (int s = 0; s < nu2; s++) {
      launch_stencil<float, MODE_JACOBI, float>(p, B, F.e32[c], F.rr32, F.e32[c ^ 1], omega, nullptr, p->ctl);
      c ^= 1;
    }
    cur[k] = c;
  }
  const long long nd0 = (long long)p->D * L0.g.N;
  hipLaunchKernelGGL(k_add_correction, dim3((unsigned)std::min<long long>((nd0 + 255) / 256, 8192)), dim3(256), 0,
                     p->stream, nd0, p->amr_u0, (const float *)L0.u32[cb], p->ctl);
  for (int k = 1; k <= Lf; k++) {
    Fine &F = p->fine[k - 1];
    const long long nd = (long long)p->D * F.g.N;
    hipLaunchKernelGGL(k_add_correction, dim3((unsigned)std::min<long long>((nd + 255) / 256, 8192)), dim3(256), 0,
                       p->stream, nd, F.u, (const float *)F.e32[cur[k]], p->ctl);
  }
}

void record_cycles(emg_problem *p, int prec, int k, int nu1, int nu2, double omega, bool fcyc) {
  if (!p->fine.empty()) {
    for (int c = 0; c < k; c++) {
      if (prec == EMG_MIXED) {
        if (p->D == 2) record_amr_cycle_mixed<2>(p, nu1, nu2, (float)omega, fcyc);
        else record_amr_cycle_mixed<3>(p, nu1, nu2, (float)omega, fcyc);
      } else {
        if (p->D == 2) record_amr_cycle<2>(p, nu1, nu2, omega, fcyc);
        else record_amr_cycle<3>(p, nu1, nu2, omega, fcyc);
      }
    }
    return;
  }
  if (prec == EMG_FP64) {
    for (int c = 0; c < k; c++) record_fp64_cycle(p, nu1, nu2, omega, fcyc);
  } else {
    for (int c = 0; c < k; c++) record_mixed_iter(p, nu1, nu2, (float)omega, fcyc);
  }
}

emg_status get_graph(emg_problem *p, int prec, int k, int nu1, int nu2, double omega, bool fcyc,
                     hipGraphExec_t *out) {
  for (auto &g : p->graphs)
    if (g.prec == prec && g.k == k && g.nu1 == nu1 && g.nu2 == nu2 && g.omega == omega && g.fcyc == (int)fcyc &&
        g.inner == p->inner) {
      *out = g.exec;
      return EMG_OK;
    }
  hipGraph_t graph;
  HIPCK(hipStreamBeginCapture(p->stream, hipStreamCaptureModeThreadLocal));
  record_cycles(p, prec, k, nu1, nu2, omega, fcyc);
  HIPCK(hipStreamEndCapture(p->stream, &graph));
  hipGraphExec_t exec;
  HIPCK(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
  HIPCK(hipGraphDestroy(graph));
  p->graphs.push_back({prec, k, nu1, nu2, (int)fcyc, p->inner, omega, exec});
  *out = exec;
  return EMG_OK;
}

emg_status validate_level(emg_problem *p, int level) {
  if (level < 0 || level >= (int)p->lv.size()) return fail(EMG_EINVAL, "level out of range");
  return EMG_OK;
}

emg_status copy_in(emg_problem *p, double *dst, const double *src, size_t count, int on_device) {
  HIPCK(hipMemcpyAsync(dst, src, count * sizeof(double), on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                       p->stream));
  HIPCK(hipStreamSynchronize(p->stream));
  return EMG_OK;
}

// ncomp component planes of `count` elements: source planes `src_ld` apart,
// destination planes `dst_ld` apart (count defaults to src_ld).
emg_status copy_planes(emg_problem *p, double *dst, long long dst_ld, const double *src, long long src_ld, int ncomp,
                       hipMemcpyKind kind, long long count = -1) {
  if (count < 0) count = src_ld;
  HIPCK(hipMemcpy2DAsync(dst, dst_ld * sizeof(double), src, src_ld * sizeof(double), count * sizeof(double), ncomp,
                         kind, p->stream));
  HIPCK(hipStreamSynchronize(p->stream));
  return EMG_OK;
}

emg_status copy_out(emg_problem *p, double *dst, const double *src, size_t count, int on_device) {
  HIPCK(hipMemcpyAsync(dst, src, count * sizeof(double), on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                       p->stream));
  HIPCK(hipStreamSynchronize(p->stream));
  return EMG_OK;
}

void destroy_graphs(emg_problem *p) {
  for (auto &g : p->graphs) (void)hipGraphExecDestroy(g.exec);
  p->graphs.clear();
}

}  // namespace

// ============================ ragged batching ============================
namespace {

constexpr int kBatchGrid = 2048;   // workgroups of a batched launch (grid-strided over the work list)

struct Step {
  int kind, D, K;
  bool f32;
  int list;
  bool zm = false;   // list of z-marching entries (k_batch_zm)
};

struct BatchPlan {
  std::vector<Step> steps;
  std::vector<std::vector<BEnt>> lists;
  std::vector<char> tail;          // per list: a coarse-tail list (several entries per problem)
  std::vector<int> sig;            // step sequence signature (graph reuse)
};

BEnt ent_level(const Geom &g) {
  BEnt e{};
  e.g = g;
  e.gx = (g.m[0] + BX - 1) / BX;
  e.gy = (g.m[1] + BY - 1) / BY;
  e.gz = g.m[2];
  return e;
}

struct Planner {
  std::vector<emg_problem *> probs;
  BatchPlan plan;
  std::vector<std::pair<int, int>> groups;
  int maxdepth = 0;

  explicit Planner(const std::vector<emg_problem *> &ps) : probs(ps) {
    for (auto *p : probs) {
      std::pair<int, int> g{p->D, p->K};
      if (std::find(groups.begin(), groups.end(), g) == groups.end()) groups.push_back(g);
      maxdepth = std::max(maxdepth, (int)p->lv.size());
    }
    std::sort(groups.begin(), groups.end());
  }

  // one launch per group, entries from `make(p)` for the problems it returns true for;
  // stencil passes over levels the z-marching pass takes go to a second list
  // of the step, launched with k_batch_zm
  template <class F>
  void step(int kind, bool f32, F make) {
    const bool stencil = kind == BK_JACOBI || kind == BK_JACOBI_NORM || kind == BK_RESID || kind == BK_RESID_F32;
    for (auto &gr : groups) {
      std::vector<BEnt> es, zs;
      for (auto *p : probs) {
        if (p->D != gr.first || p->K != gr.second) continue;
        BEnt e{};
        if (!make(p, e)) continue;
        if (stencil) {
          const int nzc = (f32 && kind != BK_RESID_F32) ? zm_plan<float>(p, e.g) : zm_plan<double>(p, e.g);
          if (nzc > 0) {
            const Split sp = split_of(e.g);
            e.nzc = nzc;
            e.gx = (int)((long long)sp.ntx * sp.nty * nzc + sp.sblocks);   // tasks
            e.gy = e.gz = 1;
            zs.push_back(e);
            continue;
          }
          e.gx = (int)stencil_blocks(e.g);   // stencil passes walk the interior/shell split
          e.gy = e.gz = 1;
        }
        es.push_back(e);
      }
      for (int z = 0; z < 2; z++) {
        auto &v = z ? zs : es;
        if (v.empty()) continue;
        long long t = 0;
        for (auto &e : v) {
          e.tile0 = t;
          t += (long long)e.gx * e.gy * e.gz;
        }
        plan.steps.push_back({kind, gr.first, gr.second, f32, (int)plan.lists.size(), z == 1});
        plan.lists.push_back(std::move(v));
        plan.tail.push_back(0);
        plan.sig.push_back((kind * 64 + gr.first * 8 + gr.second * 2 + (f32 ? 1 : 0)) * 2 + z);
      }
    }
  }

  template <typename R>
  static R *U(Level &L, int b) { return vbuf<R>(L, b); }

  // first level of a problem's fused coarse tail (its level count if none)
  template <typename R>
  static int tstart(const emg_problem *p) {
    const int k = tail_levels<R>(p);
    return (int)p->lv.size() - k;
  }

  // one launch per group: every problem's fused coarse tail (a V-cycle from
  // zero on its tail levels), entries grouped by problem
  template <typename R>
  void tail(int nu1, int nu2) {
    constexpr bool F = std::is_same<R, float>::value;
    for (auto &gr : groups) {
      std::vector<BEnt> es;
      long long q = 0;
      for (auto *p : probs) {
        if (p->D != gr.first || p->K != gr.second) continue;
        const int T = tstart<R>(p);
        if (T >= (int)p->lv.size()) continue;
        std::vector<BEnt> v;
        (void)tail_correction<R>(p, T, nu1, nu2, false, v);
        v[0].gx = v[0].gy = v[0].gz = 1;   // list total = problems
        for (auto &e : v) {
          e.tile0 = q;
          es.push_back(e);
        }
        q++;
      }
      if (es.empty()) continue;
      plan.steps.push_back({BK_TAIL, gr.first, gr.second, F, (int)plan.lists.size()});
      plan.lists.push_back(std::move(es));
      plan.tail.push_back(1);
      plan.sig.push_back((BK_TAIL * 64 + gr.first * 8 + gr.second * 2 + (F ? 1 : 0)) * 2);
    }
  }

  // coarse levels l >= 1 of the correction V-cycle (all problems with l < L_p),
  // down to each problem's fused tail, which runs between the two sweeps
  template <typename R>
  void down_up(int nu1, int nu2) {
    constexpr bool F = std::is_same<R, float>::value;
    for (int d = 1; d < maxdepth; d++) {
      step(BK_BOTTOM, F, [&](emg_problem *p, BEnt &e) {
        if (d != (int)p->lv.size() - 1 || d >= tstart<R>(p)) return false;
        Level &L = p->lv[d];
        e = BEnt{};
        e.g = L.g;
        e.gx = (p->nbot + 3) / 4;
        e.gy = e.gz = 1;
        e.Ainv = p->Ainv;
        e.nbot = p->nbot;
        e.a = fbuf<R>(L);
        e.out = U<R>(L, 0);
        e.ctl = p->ctl;
        return true;
      });
      step(BK_JZERO, F, [&](emg_problem *p, BEnt &e) {
        if (d >= (int)p->lv.size() - 1 || d >= tstart<R>(p)) return false;
        Level &L = p->lv[d];
        e = ent_level(L.g);
        e.C = moduli<R>(L);
        e.a = fbuf<R>(L);
        e.out = U<R>(L, 0);
        e.ctl = p->ctl;
        return true;
      });
      int cur = 0;
      for (int s2 = 1; s2 < nu1; s2++, cur ^= 1)
        step(BK_JACOBI, F, [&](emg_problem *p, BEnt &e) {
          if (d >= (int)p->lv.size() - 1 || d >= tstart<R>(p)) return false;
          Level &L = p->lv[d];
          e = ent_level(L.g);
          e.C = moduli<R>(L);
          e.a = U<R>(L, cur);
          e.b = fbuf<R>(L);
          e.out = U<R>(L, cur ^ 1);
          e.ctl = p->ctl;
          return true;
        });
      step(BK_RESID, F, [&](emg_problem *p, BEnt &e) {
        if (d >= (int)p->lv.size() - 1 || d >= tstart<R>(p)) return false;
        Level &L = p->lv[d];
        e = ent_level(L.g);
        e.C = moduli<R>(L);
        e.a = U<R>(L, cur);
        e.b = fbuf<R>(L);
        e.out = rbuf<R>(L);
        e.ctl = p->ctl;
        return true;
      });
      step(BK_RESTRICT, F, [&](emg_problem *p, BEnt &e) {
        if (d >= (int)p->lv.size() - 1 || d >= tstart<R>(p)) return false;
        Level &L = p->lv[d], &Lc = p->lv[d + 1];
        e = ent_level(Lc.g);
        e.g = L.g;
        e.g2 = Lc.g;
        e.a = rbuf<R>(L);
        e.out = fbuf<R>(Lc);
        e.ctl = p->ctl;
        return true;
      });
    }
    tail<R>(nu1, nu2);
    // up: deepest first
    const int post_cur = (nu1 - 1) & 1;   // buffer after the pre-sweeps of a coarse level
    const int end_cur = (nu1 - 1 + nu2) & 1;
    for (int d = maxdepth - 2; d >= 1; d--) {
      step(BK_PROLONG, F, [&](emg_problem *p, BEnt &e) {
        if (d >= (int)p->lv.size() - 1 || d >= tstart<R>(p)) return false;
        Level &L = p->lv[d], &Lc = p->lv[d + 1];
        const int cb = (d + 1 == (int)p->lv.size() - 1) ? 0 : end_cur;
        e = ent_level(L.g);
        e.g2 = Lc.g;
        e.a = U<R>(Lc, cb);
        e.out = U<R>(L, post_cur);
        e.ctl = p->ctl;
        return true;
      });
      int cur = post_cur;
      for (int s2 = 0; s2 < nu2; s2++, cur ^= 1)
        step(BK_JACOBI, F, [&](emg_problem *p, BEnt &e) {
          if (d >= (int)p->lv.size() - 1 || d >= tstart<R>(p)) return false;
          Level &L = p->lv[d];
          e = ent_level(L.g);
          e.C = moduli<R>(L);
          e.a = U<R>(L, cur);
          e.b = fbuf<R>(L);
          e.out = U<R>(L, cur ^ 1);
          e.ctl = p->ctl;
          return true;
        });
    }
  }

  // level 0 of the correction cycle for the mixed path (from zero) / the
  // FP64 path (on the iterate); ends with the result in buffer 0
  template <typename R>
  // Level-0 cycle: from zero (FP32 correction), or from the iterate in
  // buffer 0 with the residual norm and convergence check of its first sweep
  // (norm; FP64), or without them (a continuing FP32 correction cycle).
  void level0(int nu1, int nu2, bool from_zero, bool norm = true) {
    constexpr bool F = std::is_same<R, float>::value;
    int cur;
    if (from_zero) {
      step(BK_JZERO, F, [&](emg_problem *p, BEnt &e) {
        Level &L = p->lv[0];
        e = ent_level(L.g);
        e.C = moduli<R>(L);
        e.a = fbuf<R>(L);
        e.out = U<R>(L, 0);
        e.ctl = p->ctl;
        return true;
      });
      cur = 0;
    } else if (!norm) {
      step(BK_JACOBI, F, [&](emg_problem *p, BEnt &e) {
        Level &L = p->lv[0];
        e = ent_level(L.g);
        e.C = moduli<R>(L);
        e.a = U<R>(L, 0);
        e.b = fbuf<R>(L);
        e.out = U<R>(L, 1);
        e.ctl = p->ctl;
        return true;
      });
      cur = 1;
    } else {
      step(BK_JACOBI_NORM, F, [&](emg_problem *p, BEnt &e) {
        Level &L = p->lv[0];
        e = ent_level(L.g);
        e.C = moduli<R>(L);
        e.a = U<R>(L, 0);
        e.b = fbuf<R>(L);
        e.out = U<R>(L, 1);
        e.partial = p->partial;
        e.ctl = p->ctl;
        return true;
      });
      check(0);
      cur = 1;
    }
    for (int s2 = 1; s2 < nu1; s2++, cur ^= 1)
      step(BK_JACOBI, F, [&](emg_problem *p, BEnt &e) {
        Level &L = p->lv[0];
        e = ent_level(L.g);
        e.C = moduli<R>(L);
        e.a = U<R>(L, cur);
        e.b = fbuf<R>(L);
        e.out = U<R>(L, cur ^ 1);
        e.ctl = p->ctl;
        return true;
      });
    step(BK_RESID, F, [&](emg_problem *p, BEnt &e) {
      Level &L = p->lv[0];
      e = ent_level(L.g);
      e.C = moduli<R>(L);
      e.a = U<R>(L, cur);
      e.b = fbuf<R>(L);
      e.out = rbuf<R>(L);
      e.ctl = p->ctl;
      return true;
    });
    step(BK_RESTRICT, F, [&](emg_problem *p, BEnt &e) {
      Level &L = p->lv[0], &Lc = p->lv[1];
      e = ent_level(Lc.g);
      e.g = L.g;
      e.g2 = Lc.g;
      e.a = rbuf<R>(L);
      e.out = fbuf<R>(Lc);
      e.ctl = p->ctl;
      return true;
    });
    down_up<R>(nu1, nu2);
    const int end_cur = (nu1 - 1 + nu2) & 1;
    step(BK_PROLONG, F, [&](emg_problem *p, BEnt &e) {
      Level &L = p->lv[0], &Lc = p->lv[1];
      const int cb = ((int)p->lv.size() == 2) ? 0 : end_cur;
      e = ent_level(L.g);
      e.g2 = Lc.g;
      e.a = U<R>(Lc, cb);
      e.out = U<R>(L, cur);
      e.ctl = p->ctl;
      return true;
    });
    for (int s2 = 0; s2 < nu2; s2++, cur ^= 1)
      step(BK_JACOBI, F, [&](emg_problem *p, BEnt &e) {
        Level &L = p->lv[0];
        e = ent_level(L.g);
        e.C = moduli<R>(L);
        e.a = U<R>(L, cur);
        e.b = fbuf<R>(L);
        e.out = U<R>(L, cur ^ 1);
        e.ctl = p->ctl;
        return true;
      });
    if (cur != 0)
      step(BK_COPY, F, [&](emg_problem *p, BEnt &e) {
        Level &L = p->lv[0];
        e = ent_level(L.g);
        e.a = U<R>(L, cur);
        e.out = U<R>(L, 0);
        e.ctl = p->ctl;
        return true;
      });
  }

  void check(int ans) {
    for (auto &gr : groups) {
      (void)gr;
    }
    std::vector<BEnt> es;
    for (auto *p : probs) {
      BEnt e{};
      e.partial = p->partial;
      e.nparts = stencil_blocks(p->lv[0].g);
      e.ctl = p->ctl;
      e.ans = ans;
      e.gx = e.gy = e.gz = 1;
      es.push_back(e);
    }
    long long t = 0;
    for (auto &e : es) e.tile0 = t++;
    plan.steps.push_back({-1, 0, 0, false, (int)plan.lists.size()});
    plan.lists.push_back(std::move(es));
    plan.tail.push_back(0);
    plan.sig.push_back(-1);
  }

  void mixed_outer() {
    step(BK_ADDC, false, [&](emg_problem *p, BEnt &e) {
      Level &L = p->lv[0];
      e = ent_level(L.g);
      e.a = L.u32[0];
      e.out = L.u64[0];
      e.ctl = p->ctl;
      return true;
    });
    step(BK_RESID_F32, false, [&](emg_problem *p, BEnt &e) {
      Level &L = p->lv[0];
      e = ent_level(L.g);
      e.C = L.C64;
      e.a = L.u64[0];
      e.b = L.f64;
      e.out = L.f32;
      e.partial = p->partial;
      e.ctl = p->ctl;
      return true;
    });
    check(0);
  }

  void cycles(int prec, int k, int nu1, int nu2, int inner) {
    for (int c = 0; c < k; c++) {
      if (prec == EMG_FP64) {
        level0<double>(nu1, nu2, false);
      } else {
        mixed_outer();
        level0<float>(nu1, nu2, true);
        for (int i = 1; i < inner; i++) level0<float>(nu1, nu2, false, false);
      }
    }
  }
};

template <int D, int K>
void launch_batch_kind(hipStream_t st, int kind, bool f32, const BList *L, double omega) {
#define EMG_BK(KIND)                                                                                         \
  case KIND:                                                                                                 \
    if (f32)                                                                                                 \
      hipLaunchKernelGGL((k_batch<D, K, float, KIND>), dim3(kBatchGrid), dim3(BX, BY, 1), 0, st, L, (float)omega); \
    else                                                                                                     \
      hipLaunchKernelGGL((k_batch<D, K, double, KIND>), dim3(kBatchGrid), dim3(BX, BY, 1), 0, st, L, omega); \
    break;
  switch (kind) {
    EMG_BK(BK_JACOBI)
    EMG_BK(BK_JACOBI_NORM)
    EMG_BK(BK_RESID)
    EMG_BK(BK_JZERO)
    EMG_BK(BK_RESTRICT)
    EMG_BK(BK_PROLONG)
    EMG_BK(BK_BOTTOM)
    EMG_BK(BK_COPY)
    case BK_ADDC:
      hipLaunchKernelGGL((k_batch<D, K, double, BK_ADDC>), dim3(kBatchGrid), dim3(BX, BY, 1), 0, st, L, omega);
      break;
    case BK_RESID_F32:
      hipLaunchKernelGGL((k_batch<D, K, double, BK_RESID_F32>), dim3(kBatchGrid), dim3(BX, BY, 1), 0, st, L, omega);
      break;
  }
#undef EMG_BK
}

// Batched z-marching pass: FP64 fills the CUs with one workgroup each, FP32
// with two, isotropic levels with twice that (LDS and registers); tasks are
// taken grid-strided.
template <int K>
void launch_batch_zm_k(hipStream_t st, int kind, bool f32, const BList *L, double omega) {
  constexpr int mul = K == MOD_ISO ? 2 : 1;
  const dim3 g64(256 * mul), g32(512 * mul), blk(BX, BY, 1);
  switch (kind) {
    case BK_JACOBI:
    case BK_JACOBI_NORM:
      if (f32) hipLaunchKernelGGL((k_batch_zm<float, MODE_JACOBI, float, K>), g32, blk, 0, st, L, (float)omega);
      else hipLaunchKernelGGL((k_batch_zm<double, MODE_JACOBI, double, K>), g64, blk, 0, st, L, omega);
      break;
    case BK_RESID:
      if (f32) hipLaunchKernelGGL((k_batch_zm<float, MODE_RESID, float, K>), g32, blk, 0, st, L, 0.0f);
      else hipLaunchKernelGGL((k_batch_zm<double, MODE_RESID, double, K>), g64, blk, 0, st, L, 0.0);
      break;
    case BK_RESID_F32:
      hipLaunchKernelGGL((k_batch_zm<double, MODE_RESID, float, K>), g64, blk, 0, st, L, 0.0);
      break;
  }
}
void launch_batch_zm(hipStream_t st, int kind, bool f32, int K, const BList *L, double omega) {
  if (K == MOD_ISO) launch_batch_zm_k<MOD_ISO>(st, kind, f32, L, omega);
  else launch_batch_zm_k<MOD_ANISO>(st, kind, f32, L, omega);
}

// Device copy of a plan's work lists (capacity-sized, fixed addresses): the
// one-entry-per-problem lists at one stride, then the coarse-tail lists
// (several entries per problem) at their own, so that neither inflates the
// other.  A plan's i-th list of each kind always sits at the same address
// while the pool keeps its size, which is what captured graphs rely on.
struct BatchDev {
  char *buf = nullptr;
  size_t bytes = 0;
  int nlists = 0, cap = 0;     // regular lists: count and entries each
  int ntails = 0, tcap = 0;    // tail lists
  std::vector<const BList *> addr;   // per plan list
  std::vector<char> host;
  const BList *list(int i) const { return addr[i]; }
};

struct ListSizes {
  int nl = 0, cap = 1, nt = 0, tcap = 1;
};
ListSizes list_sizes(const BatchPlan &plan) {
  ListSizes z;
  for (size_t i = 0; i < plan.lists.size(); i++) {
    const int n = (int)plan.lists[i].size();
    if (plan.tail[i]) {
      z.nt++;
      z.tcap = std::max(z.tcap, n);
    } else {
      z.nl++;
      z.cap = std::max(z.cap, n);
    }
  }
  return z;
}

// Lays the plan's lists out in dev (its sizes already large enough) and
// copies them to the device.
emg_status write_lists(const BatchPlan &plan, BatchDev &dev, hipStream_t st) {
  const size_t stride = blist_bytes(dev.cap), tstride = blist_bytes(dev.tcap);
  const size_t toff = (size_t)dev.nlists * stride;
  dev.addr.assign(plan.lists.size(), nullptr);
  int il = 0, it = 0;
  for (size_t i = 0; i < plan.lists.size(); i++) {
    const size_t off = plan.tail[i] ? toff + (size_t)it++ * tstride : (size_t)il++ * stride;
    BList *h = (BList *)(dev.host.data() + off);
    const auto &es = plan.lists[i];
    h->n = (int)es.size();
    h->total = 0;
    for (size_t j = 0; j < es.size(); j++) {
      h->e[j] = es[j];
      h->total += (long long)es[j].gx * es[j].gy * es[j].gz;
    }
    dev.addr[i] = (const BList *)(dev.buf + off);
  }
  if (il) HIPCK(hipMemcpyAsync(dev.buf, dev.host.data(), (size_t)il * stride, hipMemcpyHostToDevice, st));
  if (it) HIPCK(hipMemcpyAsync(dev.buf + toff, dev.host.data() + toff, (size_t)it * tstride, hipMemcpyHostToDevice, st));
  return EMG_OK;
}

// Writes the plan's lists into the device pool (reallocated, and *grew set,
// only if it is too small: list addresses are what captured graphs hold).
emg_status upload_plan(const BatchPlan &plan, BatchDev &dev, hipStream_t st, int min_cap = 16, int min_lists = 1,
                       bool *grew = nullptr) {
  const ListSizes z = list_sizes(plan);
  if (grew) *grew = false;
  if (!dev.buf || z.nl > dev.nlists || z.cap > dev.cap || z.nt > dev.ntails || z.tcap > dev.tcap) {
    if (grew) *grew = dev.buf != nullptr;
    if (dev.buf) {
      HIPCK(hipStreamSynchronize(st));
      HIPCK(hipFree(dev.buf));
      dev.buf = nullptr;
    }
    dev.nlists = std::max(std::max(z.nl, 1), std::max(min_lists, dev.nlists));
    dev.cap = std::max(std::max(z.cap, min_cap), dev.cap);
    dev.ntails = std::max(std::max(z.nt, 1), dev.ntails);
    dev.tcap = std::max(z.tcap, dev.tcap);
    dev.bytes = (size_t)dev.nlists * blist_bytes(dev.cap) + (size_t)dev.ntails * blist_bytes(dev.tcap);
    HIPCK(hipMalloc((void **)&dev.buf, dev.bytes));
    dev.host.assign(dev.bytes, 0);
  }
  return write_lists(plan, dev, st);
}

// Writes the plan's lists into fixed device memory of `bytes` bytes (no
// allocation); EMG_EINVAL if they do not fit.
emg_status upload_plan_fixed(const BatchPlan &plan, void *base, size_t bytes, BatchDev &dev, hipStream_t st) {
  const ListSizes z = list_sizes(plan);
  dev.nlists = std::max(1, z.nl);
  dev.cap = z.cap;
  dev.ntails = z.nt;
  dev.tcap = z.tcap;
  const size_t need = (size_t)dev.nlists * blist_bytes(dev.cap) + (size_t)dev.ntails * blist_bytes(dev.tcap);
  if (need > bytes)
    return fail(EMG_EINVAL, "the batch's work lists need " + std::to_string(need) + " bytes, more than the " +
                                std::to_string(bytes) + " of the allocation-free scratch");
  dev.buf = (char *)base;
  dev.bytes = need;
  dev.host.assign(need, 0);
  return write_lists(plan, dev, st);
}

// check_grid: workgroups of the batched convergence checks (grid-strided
// over the problems), fixed so a captured graph serves any batch size
void launch_plan(const BatchPlan &plan, const BatchDev &dev, hipStream_t st, double omega, int check_grid) {
  for (auto &s : plan.steps) {
    const BList *L = dev.list(s.list);
    if (s.kind < 0) {
      hipLaunchKernelGGL(k_batch_check, dim3((unsigned)std::max(check_grid, 1)), dim3(1024), 0, st, L);
      continue;
    }
    if (s.zm) {
      launch_batch_zm(st, s.kind, s.f32, s.K, L, omega);
      continue;
    }
    if (s.kind == BK_TAIL) {
      dispatch(s.D, s.K, [&](auto Dc, auto Kc) {
        constexpr int D = decltype(Dc)::value, K = decltype(Kc)::value;
        if (s.f32) hipLaunchKernelGGL((k_tail<D, K, float>), dim3(kTailGrid), dim3(TL_THREADS), 0, st, L, (float)omega);
        else hipLaunchKernelGGL((k_tail<D, K, double>), dim3(kTailGrid), dim3(TL_THREADS), 0, st, L, omega);
      });
      continue;
    }
    if (s.D == 2 && s.K == MOD_ISO) launch_batch_kind<2, MOD_ISO>(st, s.kind, s.f32, L, omega);
    else if (s.D == 2) launch_batch_kind<2, MOD_ANISO>(st, s.kind, s.f32, L, omega);
    else if (s.K == MOD_ISO) launch_batch_kind<3, MOD_ISO>(st, s.kind, s.f32, L, omega);
    else launch_batch_kind<3, MOD_ANISO>(st, s.kind, s.f32, L, omega);
  }
}

// ---- allocation-free batches: the per-GPU scratch array ----
constexpr int kMaxDevices = 64;
struct NoAllocSlot {
  void *ptr = nullptr;              // device address of `scratch` on this GPU
  std::atomic<bool> busy{false};    // held by a running emg_solve_batch_noalloc
};
NoAllocSlot g_noalloc[kMaxDevices];
std::mutex g_noalloc_mu;

// Called with `dev` current (context creation): looks up this GPU's copy of
// the scratch array once.
emg_status noalloc_scratch_init(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return fail(EMG_EINVAL, "device index beyond the library's table");
  std::lock_guard<std::mutex> lk(g_noalloc_mu);
  if (g_noalloc[dev].ptr) return EMG_OK;
  void *ptr = nullptr;
  hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr)
    return fail(EMG_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
  g_noalloc[dev].ptr = ptr;
  return EMG_OK;
}

// Per-problem preparation before joining a batch: hierarchy, right-hand
// side, Dirichlet lift, control block.
emg_status prepare(emg_problem *p, const emg_solve_opts &opt, hipStream_t st) {
  if (!p->fine.empty()) return fail(EMG_EINVAL, "problems with refined levels are not batched");
  hipStream_t keep = p->stream;
  p->stream = st;
  emg_status s = setup(p);
  if (s == EMG_OK && opt.precision == EMG_MIXED) s = ensure_mixed(p);
  if (s == EMG_OK) s = assemble_rhs(p);
  if (s == EMG_OK) {
    Level &L0 = p->lv[0];
    if (p->D == 2) hipLaunchKernelGGL((k_lift<2>), grid_of(L0.g), kBlock, 0, st, L0.g, L0.f64, L0.u64[0]);
    else hipLaunchKernelGGL((k_lift<3>), grid_of(L0.g), kBlock, 0, st, L0.g, L0.f64, L0.u64[0]);
    if (opt.precision == EMG_MIXED) launch_fill<float>(p, (long long)p->D * L0.g.N, L0.u32[0], 0.0f);
    Ctl c0{};
    c0.r0sq = -1.0;
    c0.tol2 = opt.rtol * opt.rtol;
    c0.max_cycles = (opt.max_cycles + opt.inner_cycles - 1) / opt.inner_cycles;   // refinement steps
    *p->ctl_host = c0;
    if (hipMemcpyAsync(p->ctl, p->ctl_host, sizeof(Ctl), hipMemcpyHostToDevice, st) != hipSuccess)
      s = fail(EMG_EDEVICE, "control block upload failed");
  }
  p->stream = keep;
  return s;
}

void fill_stats(emg_problem *p, const Ctl &c, int steps_per, emg_solve_stats *st) {
  emg_solve_stats s{};
  s.cycles = c.cycles * steps_per;   // V-cycles: inner_cycles per refinement step
  s.rel_res = c.r0sq > 0 ? std::sqrt(c.rsq / c.r0sq) : 0.0;
  s.converged = c.done == 1;
  s.conv_factor = (s.cycles > 0 && s.rel_res > 0) ? std::pow(s.rel_res, 1.0 / s.cycles) : 0.0;
  const Geom &g = p->lv[0].g;
  long long inner = 1;
  for (int a = 0; a < g.dim; a++) {
    int cut = 0;
    if (!g.per[a]) cut = (g.bc[2 * a] == EMG_BC_DIRICHLET) + (g.bc[2 * a + 1] == EMG_BC_DIRICHLET);
    inner *= (g.m[a] - cut);
  }
  s.dofs = (long long)p->D * inner;
  *st = s;
}

}  // namespace

namespace {

// Validate a domain and build its multigrid level shapes.
emg_status level_chain(const emg_domain *dom, std::vector<Geom> &gs) {
  if (dom->dim != 2 && dom->dim != 3) return fail(EMG_EINVAL, "dim must be 2 or 3");
  if (dom->kind != EMG_MOD_ISO && dom->kind != EMG_MOD_ANISO) return fail(EMG_EINVAL, "bad moduli kind");
  Geom g{};
  g.dim = dom->dim;
  bool any_dir = false;
  for (int a = 0; a < 3; a++) {
    if (a < dom->dim) {
      const int b0 = dom->bc[2 * a], b1 = dom->bc[2 * a + 1];
      for (int b : {b0, b1})
        if (b != EMG_BC_DIRICHLET && b != EMG_BC_TRACTION && b != EMG_BC_PERIODIC && b != EMG_BC_NEUMANN)
          return fail(EMG_EINVAL, "bad boundary type");
      if ((b0 == EMG_BC_PERIODIC) != (b1 == EMG_BC_PERIODIC))
        return fail(EMG_EINVAL, "both faces of a periodic axis must be periodic");
      any_dir = any_dir || b0 == EMG_BC_DIRICHLET || b1 == EMG_BC_DIRICHLET;
      if (dom->n[a] < 5 || dom->n[a] > (1 << 20)) return fail(EMG_EINVAL, "every axis needs 5..2^20 nodes");
      if (!(dom->hi[a] > dom->lo[a])) return fail(EMG_EINVAL, "empty domain extent");
      g.per[a] = b0 == EMG_BC_PERIODIC;
      g.m[a] = (int)(g.per[a] ? dom->n[a] - 1 : dom->n[a]);
      g.h[a] = (dom->hi[a] - dom->lo[a]) / double(dom->n[a] - 1);
      g.bc[2 * a] = b0;
      g.bc[2 * a + 1] = b1;
    } else {
      if (dom->n[a] != 1) return fail(EMG_EINVAL, "n[2] must be 1 in 2D");
      g.m[a] = 1;
      g.per[a] = 1;
      g.h[a] = 1.0;
      g.bc[2 * a] = g.bc[2 * a + 1] = EMG_BC_PERIODIC;
    }
  }
  if (!any_dir) return fail(EMG_EINVAL, "at least one Dirichlet face is required (rigid-body null space)");
  g.N = (long long)g.m[0] * g.m[1] * g.m[2];
  if (g.N >= kMaxNodes) return fail(EMG_EINVAL, "grid too large (2^29 stored nodes per level at most)");
  g.SC = moduli_stride(g.N);
  gs.assign(1, g);
  while (can_coarsen(gs.back())) gs.push_back(coarse_of(gs.back()));
  if (gs.size() < 2) return fail(EMG_EINVAL, "grid does not coarsen (need even cell counts >= 8)");
  const long long nbot = (long long)dom->dim * gs.back().N;
  if (nbot > kMaxBottom) return fail(EMG_EINVAL, "coarsest level too large (" + std::to_string(nbot) + " unknowns)");
  return EMG_OK;
}

// Device bytes a problem on this level chain holds (FP64 arrays; FP32
// copies for mixed precision when `mixed`).
size_t footprint_of(const std::vector<Geom> &gs, int dim, int kind, bool mixed) {
  const int nc = kind == MOD_ISO ? 2 : (dim == 3 ? 21 : 6), ne = dim == 3 ? 6 : 3;
  const long long nbot = (long long)dim * gs.back().N;
  size_t b = 0;
  for (auto &g : gs) {
    b += (g.SC * nc + g.N * 4 * dim) * sizeof(double);
    if (mixed) b += (g.SC * nc + g.N * 4 * dim) * sizeof(float);
  }
  return b + gs[0].N * (ne + dim) * sizeof(double) + sizeof(double) * (size_t)nbot * nbot;
}

}  // namespace


// ============================ serving ============================
namespace {

struct Served {
  uint64_t ticket = 0;
  emg_domain dom{};
  std::vector<double> C, eps, body, face[6];   // owned copies of host inputs
  const double *pC = nullptr, *peps = nullptr, *pbody = nullptr, *pface[6] = {};
  int on_device = 0;
  double *u_out = nullptr;
  emg_problem *p = nullptr;
  size_t need = 0;
  double t_submit = 0, t_admit = 0, t_ready = 0, t_done = 0;
  bool done = false;
  emg_status status = EMG_OK;
  emg_solve_stats stats{};
};

std::vector<long long> dom_key(const emg_domain &d) {
  std::vector<long long> k = {d.dim, d.kind};
  for (int a = 0; a < 3; a++) {
    k.push_back(d.n[a]);
    long long lo, hi;
    std::memcpy(&lo, &d.lo[a], 8);
    std::memcpy(&hi, &d.hi[a], 8);
    k.push_back(lo);
    k.push_back(hi);
  }
  for (int f = 0; f < 6; f++) k.push_back(d.bc[f]);
  return k;
}

}  // namespace

// Two threads: the preparation thread takes queued requests in order, finds
// room for them (pooled hierarchy of the same domain, else a new one after
// freeing idle pooled ones), uploads their inputs and builds hierarchy, RHS
// and lift on its own stream; the scheduler thread moves prepared requests
// into free slots at cycle boundaries, replays the batched cycles of the
// active set and retires converged requests.  Preparation thus overlaps the
// running batch on the device.
struct emg_server {
  emg_ctx *ctx = nullptr;
  int slots = 8;
  emg_solve_opts opt{};
  hipStream_t stream = nullptr, prep_stream = nullptr;
  std::thread th, prep;
  std::mutex mu;                            // guards everything below but `active`
  std::condition_variable cv, cv_prep, cv_done;
  bool stop = false;
  int preparing = 0, nactive = 0;
  uint64_t next = 1;
  std::deque<Served *> pending, ready;
  std::vector<Served *> active;             // scheduler thread only
  std::map<uint64_t, Served *> all;
  std::multimap<std::vector<long long>, emg_problem *> pool;   // idle resident hierarchies
  std::map<std::vector<int>, hipGraphExec_t> graphs;          // scheduler thread only
  BatchDev dev;                                               // scheduler thread only
  std::chrono::steady_clock::time_point t0;
  double now() const { return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count(); }
};

namespace {

// Upload a request's inputs into problem p and prepare it on the
// preparation stream.
emg_status admit(emg_server *S, Served *r, emg_problem *p) {
  TRY(emg_set_moduli(p, r->pC, r->on_device));
  TRY(emg_set_eigenstrain(p, r->peps, r->on_device));
  TRY(emg_set_body_force(p, r->pbody, r->on_device));
  for (int f = 0; f < 2 * r->dom.dim; f++)
    if (r->dom.bc[f] != EMG_BC_PERIODIC) TRY(emg_set_face(p, f, r->pface[f], r->on_device));
  TRY(prepare(p, S->opt, S->prep_stream));
  HIPCK(hipStreamSynchronize(S->prep_stream));
  return EMG_OK;
}

// With S->mu held: free idle pooled problems until `need` more bytes fit.
bool make_room_locked(emg_server *S, size_t need) {
  emg_ctx *c = S->ctx;
  auto fits = [&]() {
    std::lock_guard<std::mutex> lk(c->mu);
    return c->budget == 0 || c->in_use + need <= c->budget;
  };
  while (!fits()) {
    if (S->pool.empty()) return false;
    auto it = S->pool.begin();
    emg_problem_destroy(it->second);
    S->pool.erase(it);
  }
  return true;
}

void release_inputs(Served *r) {
  r->C = std::vector<double>();
  r->eps = std::vector<double>();
  r->body = std::vector<double>();
  for (auto &f : r->face) f = std::vector<double>();
  r->pC = r->peps = r->pbody = nullptr;
  for (auto &f : r->pface) f = nullptr;
}

// Complete a request: copy its result out, return its hierarchy to the pool.
void finish(emg_server *S, Served *r, emg_status st) {
  r->status = st;
  r->t_done = S->now();
  if (r->p && (st == EMG_OK || st == EMG_ENOTCONV)) {
    if (r->u_out)
      (void)copy_out(r->p, r->u_out, r->p->lv[0].u64[0], (size_t)r->p->D * r->p->lv[0].g.N, r->on_device);
    fill_stats(r->p, *r->p->ctl_host, S->opt.inner_cycles, &r->stats);
    r->stats.solve_seconds = r->t_done - r->t_ready;
    r->stats.setup_seconds = r->t_ready - r->t_admit;
  }
  release_inputs(r);
  std::lock_guard<std::mutex> lk(S->mu);
  if (r->p) S->pool.emplace(dom_key(r->dom), r->p);
  r->p = nullptr;
  r->done = true;
  S->cv_done.notify_all();
  S->cv_prep.notify_all();
}

void prep_loop(emg_server *S) {
  (void)hipSetDevice(S->ctx->device);
  const int cap = S->slots + std::max(1, S->slots / 2);   // prepared or active requests at most
  for (;;) {
    Served *r = nullptr;
    emg_problem *p = nullptr;
    {
      std::unique_lock<std::mutex> lk(S->mu);
      for (;;) {
        if (S->pending.empty()) {
          if (S->stop) return;
          S->cv_prep.wait(lk);
          continue;
        }
        if ((int)S->ready.size() + S->nactive >= cap) {
          S->cv_prep.wait(lk);
          continue;
        }
        r = S->pending.front();
        auto it = S->pool.find(dom_key(r->dom));
        if (it != S->pool.end()) {
          p = it->second;
          S->pool.erase(it);
          break;
        }
        if (make_room_locked(S, r->need) || ((int)S->ready.size() + S->nactive == 0)) break;
        S->cv_prep.wait(lk);   // wait for a running request to free memory
      }
      S->pending.pop_front();
      S->preparing = 1;
    }
    r->t_admit = S->now();
    emg_status st = EMG_OK;
    if (!p) st = emg_problem_create(S->ctx, &r->dom, &p);
    r->p = p;
    if (st == EMG_OK) st = admit(S, r, p);
    r->t_ready = S->now();
    if (st != EMG_OK) {
      finish(S, r, st);
      std::lock_guard<std::mutex> lk(S->mu);
      S->preparing = 0;
      S->cv.notify_all();
      continue;
    }
    std::lock_guard<std::mutex> lk(S->mu);
    S->ready.push_back(r);
    S->preparing = 0;
    S->cv.notify_all();
  }
}

// Scheduler: admit prepared requests at cycle boundaries (continuous
// batching), replay the batched cycle graph for the active slot set, retire
// converged requests.
void serve_loop(emg_server *S) {
  (void)hipSetDevice(S->ctx->device);
  hipGraphExec_t exec = nullptr;
  bool changed = true;
  BatchPlan plan;
  const int k = std::max(1, S->opt.check_every);
  for (;;) {
    {
      std::unique_lock<std::mutex> lk(S->mu);
      S->cv.wait(lk, [&] {
        return !S->ready.empty() || !S->active.empty() ||
               (S->stop && S->pending.empty() && S->preparing == 0);
      });
      if (S->active.empty() && S->ready.empty() && S->stop && S->pending.empty() && S->preparing == 0) break;
      while (!S->ready.empty() && (int)S->active.size() < S->slots) {
        S->active.push_back(S->ready.front());
        S->ready.pop_front();
        changed = true;
      }
      S->nactive = (int)S->active.size();
    }
    if (S->active.empty()) continue;
    if (changed) {
      std::vector<emg_problem *> ps;
      for (auto *r : S->active) ps.push_back(r->p);
      Planner pl(ps);
      pl.cycles(S->opt.precision, k, S->opt.nu1, S->opt.nu2, S->opt.inner_cycles);
      plan = std::move(pl.plan);
      bool grew = false;
      if (upload_plan(plan, S->dev, S->stream, S->slots, 256, &grew) != EMG_OK) {
        for (auto *r : S->active) finish(S, r, EMG_EDEVICE);
        S->active.clear();
        std::lock_guard<std::mutex> lk(S->mu);
        S->nactive = 0;
        continue;
      }
      if (grew) {
        for (auto &g : S->graphs) (void)hipGraphExecDestroy(g.second);
        S->graphs.clear();
      }
      auto it = S->graphs.find(plan.sig);
      if (it == S->graphs.end()) {
        hipGraph_t graph;
        exec = nullptr;
        if (hipStreamBeginCapture(S->stream, hipStreamCaptureModeThreadLocal) == hipSuccess) {
          launch_plan(plan, S->dev, S->stream, S->opt.omega, S->slots);
          if (hipStreamEndCapture(S->stream, &graph) == hipSuccess) {
            if (hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess) exec = nullptr;
            (void)hipGraphDestroy(graph);
          }
        }
        if (exec) S->graphs[plan.sig] = exec;
      } else {
        exec = it->second;
      }
      changed = false;
    }
    if (exec) (void)hipGraphLaunch(exec, S->stream);
    else launch_plan(plan, S->dev, S->stream, S->opt.omega, S->slots);
    for (auto *r : S->active)
      (void)hipMemcpyAsync(r->p->ctl_host, r->p->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, S->stream);
    const bool ok = hipStreamSynchronize(S->stream) == hipSuccess;
    std::vector<Served *> keep;
    for (auto *r : S->active) {
      const int d = ok ? r->p->ctl_host->done : 2;
      if (!ok) finish(S, r, EMG_EDEVICE);
      else if (d == 0) keep.push_back(r);
      else finish(S, r, d == 1 ? EMG_OK : (d == 2 ? EMG_EDIVERGED : EMG_ENOTCONV));
    }
    if (keep.size() != S->active.size()) {
      changed = true;
      S->active.swap(keep);
      std::lock_guard<std::mutex> lk(S->mu);
      S->nactive = (int)S->active.size();
      S->cv_prep.notify_all();
    }
  }
  for (auto &g : S->graphs) (void)hipGraphExecDestroy(g.second);
  S->graphs.clear();
}

}  // namespace

// ============================== C ABI ==============================

extern "C" {

const char *emg_last_error(void) { return g_err.c_str(); }

void emg_default_opts(emg_solve_opts *o) {
  o->rtol = 1e-10;
  o->max_cycles = 200;
  o->precision = EMG_FP64;
  o->nu1 = 2;
  o->nu2 = 2;
  o->omega = 2.0 / 3.0;
  o->warm_start = 0;
  o->check_every = 4;
  o->use_graph = 1;
  o->cycle = EMG_VCYCLE;
  o->stall_iters = 24;
  o->stall_factor = 0.5;
  o->inner_cycles = 1;
}

emg_status emg_ctx_create(int hip_device, size_t hbm_budget_bytes, emg_ctx **out) {
  if (!out) return fail(EMG_EINVAL, "null output pointer");
  int count = 0;
  HIPCK(hipGetDeviceCount(&count));
  if (hip_device < 0 || hip_device >= count) return fail(EMG_EINVAL, "no such HIP device");
  HIPCK(hipSetDevice(hip_device));
  {
    TuneTable &t = tune_table();
    std::lock_guard<std::mutex> lk(t.mu);
    (void)tune_arch_locked(t, hip_device);
  }
  TRY(noalloc_scratch_init(hip_device));
  emg_ctx *c = new emg_ctx;
  c->device = hip_device;
  c->budget = hbm_budget_bytes;
  *out = c;
  return EMG_OK;
}

emg_status emg_ctx_destroy(emg_ctx *ctx) {
  if (!ctx) return EMG_OK;
  {
    std::lock_guard<std::mutex> lk(ctx->mu);
    if (ctx->live > 0) {   // deferred: the last problem or server frees it
      ctx->closing = true;
      return EMG_OK;
    }
  }
  delete ctx;
  return EMG_OK;
}

emg_status emg_problem_create(emg_ctx *ctx, const emg_domain *dom, emg_problem **out) {
  if (!ctx || !dom || !out) return fail(EMG_EINVAL, "null argument");
  std::vector<Geom> gs;
  TRY(level_chain(dom, gs));
  const long long nbot = (long long)dom->dim * gs.back().N;

  emg_problem *p = new emg_problem;
  p->ctx = ctx;
  p->dom = *dom;
  p->D = dom->dim;
  p->K = dom->kind;
  p->nc = p->K == MOD_ISO ? 2 : (p->D == 3 ? 21 : 6);
  p->ne = p->D == 3 ? 6 : 3;
  p->nbot = (int)nbot;
  auto bail = [&](emg_status s) {
    std::string keep = g_err;
    emg_problem_destroy(p);
    g_err = keep;
    return s;
  };
  if (hipSetDevice(ctx->device) != hipSuccess) return bail(fail(EMG_EDEVICE, "hipSetDevice failed"));
  if (hipStreamCreateWithFlags(&p->own, hipStreamNonBlocking) != hipSuccess)
    return bail(fail(EMG_EDEVICE, "hipStreamCreate failed"));
  p->stream = p->own;
  // footprint check before allocating
  const size_t need = footprint_of(gs, p->D, p->K, false);
  {
    std::lock_guard<std::mutex> lk(ctx->mu);
    if (ctx->closing) return bail(fail(EMG_ESTATE, "context is being destroyed"));
    if (ctx->budget && ctx->in_use + need > ctx->budget) return bail(fail(EMG_ENOMEM, "HBM budget exceeded"));
    ctx->in_use += need;
    ctx->live += 1;
    p->accounted = need;
    p->counted = true;
  }
  p->lv.resize(gs.size());
  for (size_t l = 0; l < gs.size(); l++) {
    Level &L = p->lv[l];
    L.g = gs[l];
    const size_t nd = (size_t)p->D * L.g.N;
    emg_status s;
    if ((s = dalloc(p, &L.C64, (size_t)p->nc * L.g.SC)) != EMG_OK) return bail(s);
    if ((s = dalloc(p, &L.u64[0], nd)) != EMG_OK) return bail(s);
    if ((s = dalloc(p, &L.u64[1], nd)) != EMG_OK) return bail(s);
    if ((s = dalloc(p, &L.f64, nd)) != EMG_OK) return bail(s);
    if ((s = dalloc(p, &L.r64, nd)) != EMG_OK) return bail(s);
  }
  emg_status s;
  if ((s = dalloc(p, &p->Ainv, (size_t)nbot * nbot)) != EMG_OK) return bail(s);
  p->npartial = grid_blocks(gs[0]);   // room for the partials of every tile shape of the stencil pass
  for (int ts = 0; ts < TS_COUNT; ts++) p->npartial = std::max(p->npartial, split_shape(gs[0], ts).blocks);
  if ((s = dalloc(p, &p->partial, (size_t)p->npartial)) != EMG_OK) return bail(s);
  if ((s = dalloc(p, &p->ctl, 1)) != EMG_OK) return bail(s);
  if ((s = dalloc(p, &p->status, 4)) != EMG_OK) return bail(s);
  if (hipHostMalloc((void **)&p->ctl_host, sizeof(Ctl), hipHostMallocDefault) != hipSuccess)
    return bail(fail(EMG_ENOMEM, "hipHostMalloc failed"));
  const size_t nd0 = (size_t)p->D * gs[0].N;
  launch_fill<double>(p, (long long)nd0, p->lv[0].u64[0], 0.0);
  if (hipStreamSynchronize(p->stream) != hipSuccess) return bail(fail(EMG_EDEVICE, "initial fill failed"));
  *out = p;
  return EMG_OK;
}

emg_status emg_problem_destroy(emg_problem *p) {
  if (!p) return EMG_OK;
  if (p->stream) (void)hipStreamSynchronize(p->stream);
  destroy_graphs(p);
  for (void *a : p->allocs) (void)hipFree(a);
  if (p->ctl_host) (void)hipHostFree(p->ctl_host);
  if (p->own) (void)hipStreamDestroy(p->own);
  if (p->ctx && p->accounted) {
    std::lock_guard<std::mutex> lk(p->ctx->mu);
    p->ctx->in_use -= std::min(p->ctx->in_use, p->accounted);
  }
  emg_ctx *c = p->counted ? p->ctx : nullptr;
  delete p;
  if (c) ctx_release(c);
  return EMG_OK;
}

emg_status emg_set_stream(emg_problem *p, void *s) {
  if (!p) return fail(EMG_EINVAL, "null problem");
  HIPCK(hipStreamSynchronize(p->stream));
  destroy_graphs(p);
  p->stream = s ? (hipStream_t)s : p->own;
  return EMG_OK;
}

emg_status emg_footprint(const emg_problem *p, size_t *bytes) {
  if (!p || !bytes) return fail(EMG_EINVAL, "null argument");
  *bytes = p->bytes;
  return EMG_OK;
}

emg_status emg_set_moduli(emg_problem *p, const double *C, int on_device) {
  if (!p || !C) return fail(EMG_EINVAL, "null argument");
  TRY(copy_planes(p, p->lv[0].C64, p->lv[0].g.SC, C, p->lv[0].g.N, p->nc, on_device ? hipMemcpyDeviceToDevice
                                                                                         : hipMemcpyHostToDevice));
  p->moduli_set = true;
  p->setup_done = p->mixed_ready = p->rhs_ready = false;
  return EMG_OK;
}

emg_status emg_set_eigenstrain(emg_problem *p, const double *e, int on_device) {
  if (!p) return fail(EMG_EINVAL, "null problem");
  p->rhs_ready = false;
  if (!e) {
    p->eps = nullptr;
    return EMG_OK;
  }
  static_assert(sizeof(double) == 8, "");
  if (!p->eps) TRY(dalloc(p, &p->eps, (size_t)p->ne * p->lv[0].g.N));
  return copy_in(p, p->eps, e, (size_t)p->ne * p->lv[0].g.N, on_device);
}

emg_status emg_set_body_force(emg_problem *p, const double *b, int on_device) {
  if (!p) return fail(EMG_EINVAL, "null problem");
  p->rhs_ready = false;
  if (!b) {
    p->body = nullptr;
    return EMG_OK;
  }
  if (!p->body) TRY(dalloc(p, &p->body, (size_t)p->D * p->lv[0].g.N));
  return copy_in(p, p->body, b, (size_t)p->D * p->lv[0].g.N, on_device);
}

emg_status emg_set_face(emg_problem *p, int f, const double *v, int on_device) {
  if (!p) return fail(EMG_EINVAL, "null problem");
  if (f < 0 || f >= 2 * p->D) return fail(EMG_EINVAL, "face out of range");
  if (p->lv[0].g.per[f / 2]) return fail(EMG_EINVAL, "periodic faces carry no data");
  p->rhs_ready = false;
  if (!v) {
    p->face[f] = nullptr;
    return EMG_OK;
  }
  const Geom &g = p->lv[0].g;
  const size_t fn = (size_t)g.N / g.m[f / 2];
  if (!p->face[f]) TRY(dalloc(p, &p->face[f], (size_t)p->D * fn));
  return copy_in(p, p->face[f], v, (size_t)p->D * fn, on_device);
}

emg_status emg_solve(emg_problem *p, const emg_solve_opts *o, emg_solve_stats *st) {
  if (!p) return fail(EMG_EINVAL, "null problem");
  emg_solve_opts opt;
  emg_default_opts(&opt);
  if (o) opt = *o;
  if (opt.precision != EMG_FP64 && opt.precision != EMG_MIXED) return fail(EMG_EINVAL, "bad precision");
  if (opt.nu1 < 1 || opt.nu2 < 0 || opt.nu1 > 16 || opt.nu2 > 16) return fail(EMG_EINVAL, "bad sweep counts");
  if (!(opt.omega > 0.0 && opt.omega < 2.0)) return fail(EMG_EINVAL, "omega must lie in (0, 2)");
  if (!(opt.rtol >= 0.0) || opt.max_cycles < 0) return fail(EMG_EINVAL, "bad tolerance or cycle cap");
  if (opt.cycle != EMG_VCYCLE && opt.cycle != EMG_FCYCLE) return fail(EMG_EINVAL, "bad cycle type");
  if (opt.stall_iters < 0 || (opt.stall_iters > 0 && !(opt.stall_factor > 0.0 && opt.stall_factor < 1.0)))
    return fail(EMG_EINVAL, "bad stall test");
  if (opt.inner_cycles < 1 || opt.inner_cycles > 4) return fail(EMG_EINVAL, "inner_cycles must lie in 1..4");
  if (opt.inner_cycles > 1 && (opt.precision != EMG_MIXED || !p->fine.empty()))
    return fail(EMG_EINVAL, "inner_cycles > 1 needs a single-level mixed-precision solve");
  const int inner = opt.inner_cycles;
  p->inner = inner;
  struct InnerReset {
    emg_problem *p;
    ~InnerReset() { p->inner = 1; }
  } inner_reset{p};
  const int k = std::max(1, opt.check_every);
  const auto t0 = std::chrono::steady_clock::now();
  TRY(setup(p));
  if (opt.precision == EMG_MIXED) TRY(ensure_mixed(p));
  TRY(assemble_rhs(p));
  TRY(prepare_tail<double>(p, opt.nu1, opt.nu2, opt.cycle == EMG_FCYCLE));   // FP64 cycles (and fallback)
  if (opt.precision == EMG_MIXED) TRY(prepare_tail<float>(p, opt.nu1, opt.nu2, opt.cycle == EMG_FCYCLE));
  Level &L0 = p->lv[0];
  const long long nd0 = (long long)p->D * L0.g.N;
  Ctl c0{};
  c0.r0sq = -1.0;
  c0.tol2 = opt.rtol * opt.rtol;
  c0.max_cycles = (opt.max_cycles + inner - 1) / inner;   // refinement steps
  *p->ctl_host = c0;
  HIPCK(hipMemcpyAsync(p->ctl, p->ctl_host, sizeof(Ctl), hipMemcpyHostToDevice, p->stream));
  if (!p->fine.empty()) {
    // composite start: Dirichlet lift on the base grid (norm reference),
    // refined levels interpolated from it, coarsest first
    if (!opt.warm_start) {
      if (p->D == 2)
        hipLaunchKernelGGL((k_lift<2>), grid_of(L0.g), kBlock, 0, p->stream, L0.g, p->amr_f0, p->amr_u0);
      else
        hipLaunchKernelGGL((k_lift<3>), grid_of(L0.g), kBlock, 0, p->stream, L0.g, p->amr_f0, p->amr_u0);
      for (int k = 1; k <= (int)p->fine.size(); k++) {
        Fine &F = p->fine[k - 1];
        const double *uc = k == 1 ? p->amr_u0 : p->fine[k - 2].u;
        if (p->D == 2)
          hipLaunchKernelGGL((k_interp<2, double>), act_grid(F), kBlock, 0, p->stream, parent_geom(p, k),
                             parent_origin(p, k), F.g, F.b, F.vm, F.act_gr, uc, F.u, (double *)nullptr, 0, (const Ctl *)nullptr);
        else
          hipLaunchKernelGGL((k_interp<3, double>), act_grid(F), kBlock, 0, p->stream, parent_geom(p, k),
                             parent_origin(p, k), F.g, F.b, F.vm, F.act_gr, uc, F.u, (double *)nullptr, 0, (const Ctl *)nullptr);
      }
    }
    // with a warm start the reference norm is the warm iterate's composite residual
  }
  // the Dirichlet lift; with a warm start it goes to a scratch buffer and
  // only its residual norm is kept as the reference
  double *lift = opt.warm_start ? L0.u64[1] : L0.u64[0];
  if (p->fine.empty()) {
    if (p->D == 2)
      hipLaunchKernelGGL((k_lift<2>), grid_of(L0.g), kBlock, 0, p->stream, L0.g, L0.f64, lift);
    else
      hipLaunchKernelGGL((k_lift<3>), grid_of(L0.g), kBlock, 0, p->stream, L0.g, L0.f64, lift);
  }
  if (opt.warm_start && p->fine.empty()) {
    launch_stencil<double, MODE_RESID, double>(p, L0, lift, L0.f64, L0.r64, 0.0, p->partial, nullptr);
    hipLaunchKernelGGL(k_set_r0, dim3(1), dim3(1024), 0, p->stream, p->partial, plan_blocks<double>(p, L0.g), p->ctl);
  }
  if (opt.precision == EMG_MIXED) launch_fill<float>(p, nd0, L0.u32[mixed_result_buf(p, opt.nu1, opt.nu2)], 0.0f);
  HIPCK(hipGetLastError());
  HIPCK(hipStreamSynchronize(p->stream));
  const auto t1 = std::chrono::steady_clock::now();
  hipGraphExec_t exec = nullptr;
  const bool fcyc = opt.cycle == EMG_FCYCLE;
  if (opt.use_graph) TRY(get_graph(p, opt.precision, k, opt.nu1, opt.nu2, opt.omega, fcyc, &exec));
  const auto t2 = std::chrono::steady_clock::now();
  int prec = opt.precision;
  bool fell_back = false;
  double win_rsq = -1.0;   // stall test: residual at the start of the current window
  int win_start = 0;
  int fb_steps = -1;   // refinement steps done when FP64 cycles took over
  for (;;) {
    if (exec)
      HIPCK(hipGraphLaunch(exec, p->stream));
    else
      record_cycles(p, prec, k, opt.nu1, opt.nu2, opt.omega, fcyc);
    HIPCK(hipGetLastError());
    HIPCK(hipMemcpyAsync(p->ctl_host, p->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, p->stream));
    HIPCK(hipStreamSynchronize(p->stream));
    const Ctl &h = *p->ctl_host;
    if (h.done) break;
    if (prec == EMG_MIXED && opt.stall_iters > 0) {
      if (win_rsq < 0.0 || h.rsq <= win_rsq * opt.stall_factor * opt.stall_factor) {
        win_rsq = h.rsq;
        win_start = h.cycles;
      } else if (h.cycles - win_start >= opt.stall_iters) {
        // the FP32 corrections no longer reduce the FP64 residual: FP64
        // cycles take over from the current iterate (the FP64 state; a
        // pending FP32 correction is dropped), with the same reference norm,
        // cycle count and cap
        prec = EMG_FP64;
        fell_back = true;
        fb_steps = h.cycles;
        // the cap counts V-cycles: fb_steps steps used inner V-cycles each,
        // every FP64 cycle from here on counts one
        p->ctl_host->max_cycles = fb_steps + std::max(0, opt.max_cycles - fb_steps * inner);
        HIPCK(hipMemcpyAsync(p->ctl, p->ctl_host, sizeof(Ctl), hipMemcpyHostToDevice, p->stream));
        HIPCK(hipStreamSynchronize(p->stream));
        exec = nullptr;
        if (opt.use_graph) TRY(get_graph(p, EMG_FP64, k, opt.nu1, opt.nu2, opt.omega, fcyc, &exec));
      }
    }
  }
  const auto t3 = std::chrono::steady_clock::now();
  const Ctl c = *p->ctl_host;
  // the answer lives in buffer c.ans of level 0; keep it in buffer 0
  if (c.ans != 0 && p->fine.empty()) {
    HIPCK(hipMemcpyAsync(L0.u64[0], L0.u64[c.ans], sizeof(double) * nd0, hipMemcpyDeviceToDevice, p->stream));
    HIPCK(hipStreamSynchronize(p->stream));
  }
  emg_solve_stats s{};
  // V-cycles: inner per refinement step, one per FP64 cycle after a fallback
  s.cycles = fb_steps >= 0 ? fb_steps * inner + (c.cycles - fb_steps) : c.cycles * inner;
  s.rel_res = c.r0sq > 0 ? std::sqrt(c.rsq / c.r0sq) : 0.0;
  s.converged = c.done == 1;
  s.conv_factor = (s.cycles > 0 && s.rel_res > 0) ? std::pow(s.rel_res, 1.0 / s.cycles) : 0.0;
  s.solve_seconds = std::chrono::duration<double>(t3 - t2).count();
  s.setup_seconds = std::chrono::duration<double>(t1 - t0).count();
  long long dir_nodes = 0;
  {
    const Geom &g = L0.g;
    // count nodes on a Dirichlet face (inclusion-exclusion over the box)
    long long inner = 1;
    for (int a = 0; a < g.dim; a++) {
      int cut = 0;
      if (!g.per[a]) cut = (g.bc[2 * a] == EMG_BC_DIRICHLET) + (g.bc[2 * a + 1] == EMG_BC_DIRICHLET);
      inner *= (g.m[a] - cut);
    }
    dir_nodes = g.N - inner;
  }
  long long unknown_nodes = L0.g.N - dir_nodes;
  for (auto &F : p->fine) unknown_nodes += F.nvalid - F.ncov;
  s.dofs = (long long)p->D * unknown_nodes;
  s.fp64_fallback = fell_back ? 1 : 0;
  if (st) *st = s;
  if (c.done == 2) return fail(EMG_EDIVERGED, "residual norm is not finite");
  if (c.done == 3) return fail(EMG_ENOTCONV, "cycle cap reached before the tolerance");
  return EMG_OK;
}

static double *base_u(emg_problem *p) { return p->fine.empty() ? p->lv[0].u64[0] : p->amr_u0; }

emg_status emg_get_displacement(emg_problem *p, double *u, int on_device) {
  if (!p || !u) return fail(EMG_EINVAL, "null argument");
  return copy_out(p, u, base_u(p), (size_t)p->D * p->lv[0].g.N, on_device);
}

emg_status emg_set_displacement(emg_problem *p, const double *u, int on_device) {
  if (!p || !u) return fail(EMG_EINVAL, "null argument");
  return copy_in(p, base_u(p), u, (size_t)p->D * p->lv[0].g.N, on_device);
}

emg_status emg_get_rhs(emg_problem *p, double *f, int on_device) {
  if (!p || !f) return fail(EMG_EINVAL, "null argument");
  if (!p->moduli_set) return fail(EMG_ESTATE, "moduli not set");
  TRY(assemble_rhs(p));
  return copy_out(p, f, p->fine.empty() ? p->lv[0].f64 : p->amr_f0, (size_t)p->D * p->lv[0].g.N, on_device);
}

emg_status emg_get_stress(emg_problem *p, int level, double *sigma, int on_device) {
  if (!p || !sigma) return fail(EMG_EINVAL, "null argument");
  if (!p->moduli_set) return fail(EMG_ESTATE, "moduli not set");
  if (level < 0 || level > (int)p->fine.size()) return fail(EMG_EINVAL, "no such level");
  if (level == 0) {
    const Level &L0 = p->lv[0];
    if (!p->sig) TRY(dalloc(p, &p->sig, (size_t)p->ne * L0.g.N));
    dispatch(p->D, p->K, [&](auto Dc, auto Kc) {
      constexpr int D = decltype(Dc)::value, K = decltype(Kc)::value;
      hipLaunchKernelGGL((k_stress<D, K>), grid_of(L0.g), kBlock, 0, p->stream, L0.g, L0.C64, p->eps, base_u(p),
                         p->sig);
    });
    HIPCK(hipGetLastError());
    return copy_out(p, sigma, p->sig, (size_t)p->ne * L0.g.N, on_device);
  }
  TRY(setup(p));   // moduli of covered nodes averaged from the finer level, as in the solve
  Fine &F = p->fine[level - 1];
  if (!F.sig) TRY(dalloc(p, &F.sig, (size_t)p->ne * F.g.N));
  dispatch(p->D, p->K, [&](auto Dc, auto Kc) {
    constexpr int D = decltype(Dc)::value, K = decltype(Kc)::value;
    hipLaunchKernelGGL((k_stress<D, K>), grid_of(F.g), kBlock, 0, p->stream, F.g, (const double *)F.C,
                       (const double *)F.eps, (const double *)F.u, F.sig);
  });
  HIPCK(hipGetLastError());
  return copy_out(p, sigma, F.sig, (size_t)p->ne * F.g.N, on_device);
}

emg_status emg_get_von_mises(emg_problem *p, double *svm, int on_device) {
  if (!p || !svm) return fail(EMG_EINVAL, "null argument");
  if (p->D != 3) return fail(EMG_EINVAL, "von Mises stress is defined for 3D problems");
  if (!p->moduli_set) return fail(EMG_ESTATE, "moduli not set");
  const Level &L0 = p->lv[0];
  const long long N = L0.g.N;
  if (!p->sig) TRY(dalloc(p, &p->sig, (size_t)p->ne * N));
  if (!p->svm) TRY(dalloc(p, &p->svm, (size_t)N));
  dispatch(p->D, p->K, [&](auto Dc, auto Kc) {
    constexpr int D = decltype(Dc)::value, K = decltype(Kc)::value;
    hipLaunchKernelGGL((k_stress<D, K>), grid_of(L0.g), kBlock, 0, p->stream, L0.g, L0.C64, p->eps, base_u(p), p->sig);
  });
  hipLaunchKernelGGL(k_von_mises, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, p->stream, N, (const double *)p->sig,
                     p->svm);
  HIPCK(hipGetLastError());
  return copy_out(p, svm, p->svm, (size_t)N, on_device);
}

emg_status emg_level_zmarch(emg_problem *p, int level, int precision, int *chunks) {
  if (!p || !chunks) return fail(EMG_EINVAL, "null argument");
  TRY(validate_level(p, level));
  if (precision != EMG_FP64 && precision != EMG_MIXED) return fail(EMG_EINVAL, "bad precision");
  const Geom &g = p->lv[level].g;
  *chunks = precision == EMG_FP64 ? zm_plan<double>(p, g) : zm_plan<float>(p, g);
  return EMG_OK;
}

emg_status emg_tail_levels(emg_problem *p, int precision, int *levels) {
  if (!p || !levels) return fail(EMG_EINVAL, "null argument");
  if (precision != EMG_FP64 && precision != EMG_MIXED) return fail(EMG_EINVAL, "bad precision");
  *levels = precision == EMG_FP64 ? tail_levels<double>(p) : tail_levels<float>(p);
  return EMG_OK;
}

emg_status emg_num_levels(emg_problem *p, int *levels) {
  if (!p || !levels) return fail(EMG_EINVAL, "null argument");
  *levels = (int)p->lv.size();
  return EMG_OK;
}

emg_status emg_level_shape(emg_problem *p, int level, int64_t m[3], double h[3]) {
  if (!p) return fail(EMG_EINVAL, "null problem");
  TRY(validate_level(p, level));
  for (int a = 0; a < 3; a++) {
    if (m) m[a] = p->lv[level].g.m[a];
    if (h) h[a] = p->lv[level].g.h[a];
  }
  return EMG_OK;
}

emg_status emg_level_moduli(emg_problem *p, int level, double *C_dev) {
  if (!p || !C_dev) return fail(EMG_EINVAL, "null argument");
  TRY(validate_level(p, level));
  TRY(setup(p));
  return copy_planes(p, C_dev, p->lv[level].g.N, p->lv[level].C64, p->lv[level].g.SC, p->nc, hipMemcpyDeviceToDevice,
                     p->lv[level].g.N);
}

static emg_status level_prep(emg_problem *p, int level, int precision) {
  if (!p) return fail(EMG_EINVAL, "null problem");
  TRY(validate_level(p, level));
  if (precision != EMG_FP64 && precision != EMG_MIXED) return fail(EMG_EINVAL, "bad precision");
  TRY(setup(p));
  if (precision == EMG_MIXED) TRY(ensure_mixed(p));
  return EMG_OK;
}

static emg_status finish(emg_problem *p) {
  HIPCK(hipGetLastError());
  HIPCK(hipStreamSynchronize(p->stream));
  return EMG_OK;
}

emg_status emg_level_apply(emg_problem *p, int level, int precision, const void *u, void *out) {
  TRY(level_prep(p, level, precision));
  const Level &L = p->lv[level];
  if (precision == EMG_FP64)
    launch_stencil<double, MODE_APPLY, double>(p, L, (const double *)u, nullptr, (double *)out, 0.0, nullptr, nullptr);
  else
    launch_stencil<float, MODE_APPLY, float>(p, L, (const float *)u, nullptr, (float *)out, 0.0f, nullptr, nullptr);
  return finish(p);
}

emg_status emg_level_residual(emg_problem *p, int level, int precision, const void *u, const void *f, void *out) {
  TRY(level_prep(p, level, precision));
  const Level &L = p->lv[level];
  if (precision == EMG_FP64)
    launch_stencil<double, MODE_RESID, double>(p, L, (const double *)u, (const double *)f, (double *)out, 0.0, nullptr,
                                               nullptr);
  else
    launch_stencil<float, MODE_RESID, float>(p, L, (const float *)u, (const float *)f, (float *)out, 0.0f, nullptr,
                                             nullptr);
  return finish(p);
}

emg_status emg_level_jacobi(emg_problem *p, int level, int precision, double omega, const void *u, const void *f,
                            void *out) {
  TRY(level_prep(p, level, precision));
  const Level &L = p->lv[level];
  if (precision == EMG_FP64)
    launch_stencil<double, MODE_JACOBI, double>(p, L, (const double *)u, (const double *)f, (double *)out, omega,
                                                nullptr, nullptr);
  else
    launch_stencil<float, MODE_JACOBI, float>(p, L, (const float *)u, (const float *)f, (float *)out, (float)omega,
                                              nullptr, nullptr);
  return finish(p);
}

emg_status emg_level_restrict(emg_problem *p, int level, int precision, const void *r, void *fc) {
  TRY(level_prep(p, level, precision));
  if (level + 1 >= (int)p->lv.size()) return fail(EMG_EINVAL, "no coarser level");
  if (precision == EMG_FP64)
    launch_restrict<double, double>(p, p->lv[level], p->lv[level + 1], (const double *)r, (double *)fc, nullptr);
  else
    launch_restrict<float, float>(p, p->lv[level], p->lv[level + 1], (const float *)r, (float *)fc, nullptr);
  return finish(p);
}

emg_status emg_level_prolong_add(emg_problem *p, int level, int precision, const void *ec, void *uf) {
  TRY(level_prep(p, level, precision));
  if (level + 1 >= (int)p->lv.size()) return fail(EMG_EINVAL, "no coarser level");
  if (precision == EMG_FP64)
    launch_prolong<double, double>(p, p->lv[level + 1], p->lv[level], (const double *)ec, (double *)uf, nullptr);
  else
    launch_prolong<float, float>(p, p->lv[level + 1], p->lv[level], (const float *)ec, (float *)uf, nullptr);
  return finish(p);
}

emg_status emg_level_bottom_solve(emg_problem *p, int precision, const void *f, void *e) {
  TRY(level_prep(p, (int)p->lv.size() - 1, precision));
  if (precision == EMG_FP64)
    launch_bottom<double, double>(p, (const double *)f, (double *)e, nullptr);
  else
    launch_bottom<float, float>(p, (const float *)f, (float *)e, nullptr);
  return finish(p);
}

// Average duration of one level kernel (0 Jacobi sweep, 1 residual, 2
// interpolation) over reps launches captured into a graph; arguments checked
// by the caller, which also synchronises.
static emg_status time_level_kernel(emg_problem *p, int kernel, int level, int precision, int reps, double *avg_ms) {
  Level &L = p->lv[level];
  auto one = [&]() {
    if (precision == EMG_FP64) {
      if (kernel == 0)
        launch_stencil<double, MODE_JACOBI, double>(p, L, L.u64[0], L.f64, L.u64[1], 2.0 / 3.0, nullptr, nullptr);
      else if (kernel == 1)
        launch_stencil<double, MODE_RESID, double>(p, L, L.u64[0], L.f64, L.r64, 0.0, nullptr, nullptr);
      else if (kernel == 2)
        launch_prolong<double, double>(p, p->lv[level + 1], L, p->lv[level + 1].u64[0], L.u64[1], nullptr);
      else if (kernel == 3)
        (void)restrict_down<double>(p, level, 2.0 / 3.0, nullptr);
      else
        (void)coarse_correction<double>(p, level, 2, 2, 2.0 / 3.0, false, false);
    } else {
      if (kernel == 0)
        launch_stencil<float, MODE_JACOBI, float>(p, L, L.u32[0], L.f32, L.u32[1], 2.0f / 3.0f, nullptr, nullptr);
      else if (kernel == 1)
        launch_stencil<float, MODE_RESID, float>(p, L, L.u32[0], L.f32, L.r32, 0.0f, nullptr, nullptr);
      else if (kernel == 2)
        launch_prolong<float, float>(p, p->lv[level + 1], L, p->lv[level + 1].u32[0], L.u32[1], nullptr);
      else if (kernel == 3)
        (void)restrict_down<float>(p, level, 2.0f / 3.0f, nullptr);
      else
        (void)coarse_correction<float>(p, level, 2, 2, 2.0f / 3.0f, false, false);
    }
  };
  // The launches are captured into one graph, as the solve's cycles are, and
  // the graph is replayed once untimed and once between the two events.
  one();  // warm
  hipGraph_t graph;
  HIPCK(hipStreamBeginCapture(p->stream, hipStreamCaptureModeThreadLocal));
  for (int r = 0; r < reps; r++) one();
  HIPCK(hipStreamEndCapture(p->stream, &graph));
  hipGraphExec_t exec;
  const hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (ie != hipSuccess) return fail(EMG_EDEVICE, "graph instantiate");
  hipEvent_t e0 = nullptr, e1 = nullptr;
  float ms = 0.f;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e == hipSuccess) e = hipGraphLaunch(exec, p->stream);
  if (e == hipSuccess) e = hipEventRecord(e0, p->stream);
  if (e == hipSuccess) e = hipGraphLaunch(exec, p->stream);
  if (e == hipSuccess) e = hipEventRecord(e1, p->stream);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipGraphExecDestroy(exec);
  if (e != hipSuccess) return fail(EMG_EDEVICE, hipGetErrorString(e));
  *avg_ms = ms / reps;
  return EMG_OK;
}

emg_status emg_kernel_time(emg_problem *p, int kernel, int level, int precision, int reps, double *avg_ms) {
  TRY(level_prep(p, level, precision));
  if (reps < 1 || !avg_ms) return fail(EMG_EINVAL, "bad reps or output");
  if ((kernel == 2 || kernel == 3) && level + 1 >= (int)p->lv.size()) return fail(EMG_EINVAL, "no coarser level");
  if (kernel < 0 || kernel > 3) return fail(EMG_EINVAL, "unknown kernel id");
  TRY(time_level_kernel(p, kernel, level, precision, reps, avg_ms));
  return finish(p);
}

// ---- autotuner ----

emg_status emg_autotune(emg_problem *p, int precision, int reps, int retune, int *tuned) {
  if (tuned) *tuned = 0;
  TRY(level_prep(p, 0, precision));
  if (reps < 1 || reps > 1000) return fail(EMG_EINVAL, "bad reps");
  const int rb = precision == EMG_FP64 ? 8 : 4;
  TuneTable &t = tune_table();
  int count = 0;
  // best of two graph replays of `reps` launches of `kernel` on level l
  auto measure = [&](int kernel, int l, double *ms) -> emg_status {
    double a = 0.0, b = 0.0;
    TRY(time_level_kernel(p, kernel, l, precision, reps, &a));
    TRY(time_level_kernel(p, kernel, l, precision, reps, &b));
    *ms = std::min(a, b);
    return EMG_OK;
  };
  auto record = [&](const Geom &g, const char *what, int v) {
    std::lock_guard<std::mutex> lk(t.mu);
    tune_load_locked(t);
    t.table[tune_key_locked(t, p->ctx->device, rb, g, p->K, what)] = v;
  };
  const int L = (int)p->lv.size();
  for (int l = 0; l < L; l++) {
    const Geom &g = p->lv[l].g;
    const Split sp = split_of(g);
    int have;
    bool measured = false;
    // stencil pass: the tile kernel in each tile shape, the z-marching pass at each chunk count
    if (retune || !tune_find(p->ctx->device, rb, g, &have, p->K)) {
      std::vector<int> cands;
      for (int s = 0; s < TS_COUNT; s++) cands.push_back(-s);
      if (zm_valid(g, 1))
        for (int c = 1; c <= sp.ntz / 8; c++) cands.push_back(c);
      double best_ms = 0.0;
      int best = 0;
      for (size_t i = 0; i < cands.size(); i++) {
        double ms = 0.0;
        p->force_stencil = true;
        p->force_v = cands[i];
        const emg_status st = measure(0, l, &ms);
        p->force_stencil = false;
        if (st != EMG_OK) return st;
        if (i == 0 || ms < best_ms) {
          best = cands[i];
          best_ms = ms;
        }
      }
      record(g, "", best);
      measured = true;
    }
    // restriction from level l and interpolation onto it: tile shapes
    for (int xf = 0; xf < 2 && l + 1 < L; xf++) {
      const bool restriction = xf == 0;
      if (!retune && tune_find(p->ctx->device, rb, g, &have, p->K, restriction ? "/r" : "/i")) continue;
      double best_ms = 0.0;
      int best = 0;
      for (int s = 0; s < TS_COUNT; s++) {
        double ms = 0.0;
        (restriction ? p->force_rs : p->force_ps) = s;
        const emg_status st = measure(restriction ? 3 : 2, l, &ms);
        (restriction ? p->force_rs : p->force_ps) = -1;
        if (st != EMG_OK) return st;
        if (s == 0 || ms < best_ms) {
          best = s;
          best_ms = ms;
        }
      }
      record(g, restriction ? "/r" : "/i", best);
      measured = true;
    }
    if (measured) count++;
  }
  // fused coarse tail: the V(2,2) correction on the candidate levels as one
  // launch against a launch per pass (the control block is reset to running
  // so that every launch does its work)
  bool tail_measured = false;
  const int kc = tail_candidate(p);
  int have_tail;
  if (kc >= 2 && (retune || !tune_find(p->ctx->device, rb, p->lv[0].g, &have_tail, p->K, "/tail"))) {
    Ctl c0{};
    c0.r0sq = -1.0;
    c0.max_cycles = 1 << 30;
    *p->ctl_host = c0;
    HIPCK(hipMemcpyAsync(p->ctl, p->ctl_host, sizeof(Ctl), hipMemcpyHostToDevice, p->stream));
    struct TailReset {
      emg_problem *p;
      ~TailReset() { p->force_tail = -1; }
    } tail_reset{p};
    double sep = 0.0, fused = 0.0;
    p->force_tail = 0;
    TRY(measure(4, L - kc, &sep));
    p->force_tail = kc;
    TRY(precision == EMG_FP64 ? prepare_tail<double>(p, 2, 2, false) : prepare_tail<float>(p, 2, 2, false));
    TRY(measure(4, L - kc, &fused));
    record(p->lv[0].g, "/tail", fused < sep ? kc : 0);
    tail_measured = true;
  }
  destroy_graphs(p);   // recorded with the earlier plans
  if (tuned) *tuned = count;
  if (count > 0 || tail_measured) {
    std::lock_guard<std::mutex> lk(t.mu);
    if (!tune_save_locked(t)) return fail(EMG_EINVAL, "cannot write the EMG_TUNE_CACHE file");
  }
  return finish(p);
}

emg_status emg_level_tiles(emg_problem *p, int level, int precision, int *stencil, int *restriction,
                           int *interpolation) {
  if (!p) return fail(EMG_EINVAL, "null problem");
  if (level < 0 || level >= (int)p->lv.size()) return fail(EMG_EINVAL, "no such level");
  if (precision != EMG_FP64 && precision != EMG_MIXED) return fail(EMG_EINVAL, "bad precision");
  const Geom &g = p->lv[level].g;
  const bool last = level + 1 >= (int)p->lv.size();
  if (precision == EMG_FP64) {
    if (stencil) *stencil = tile_plan<double>(p, g);
    if (restriction) *restriction = last ? -1 : xfer_plan<double>(p, g, true);
    if (interpolation) *interpolation = last ? -1 : xfer_plan<double>(p, g, false);
  } else {
    if (stencil) *stencil = tile_plan<float>(p, g);
    if (restriction) *restriction = last ? -1 : xfer_plan<float>(p, g, true);
    if (interpolation) *interpolation = last ? -1 : xfer_plan<float>(p, g, false);
  }
  return EMG_OK;
}

emg_status emg_autotune_reset(void) {
  TuneTable &t = tune_table();
  std::lock_guard<std::mutex> lk(t.mu);
  t.table.clear();
  t.loaded = false;
  return EMG_OK;
}

// ---- ragged batches ----

static emg_status batch_args(emg_problem **probs, int n, const emg_solve_opts *o, emg_solve_opts &opt,
                             std::vector<emg_problem *> &ps) {
  if (!probs || n < 1) return fail(EMG_EINVAL, "empty batch");
  emg_default_opts(&opt);
  if (o) opt = *o;
  if (opt.precision != EMG_FP64 && opt.precision != EMG_MIXED) return fail(EMG_EINVAL, "bad precision");
  if (opt.nu1 < 1 || opt.nu2 < 0 || opt.nu1 > 16 || opt.nu2 > 16) return fail(EMG_EINVAL, "bad sweep counts");
  if (opt.inner_cycles < 1 || opt.inner_cycles > 4 || (opt.inner_cycles > 1 && opt.precision != EMG_MIXED))
    return fail(EMG_EINVAL, "inner_cycles must lie in 1..4 (above 1 in mixed precision only)");
  if (!(opt.omega > 0.0 && opt.omega < 2.0) || opt.warm_start) return fail(EMG_EINVAL, "bad omega or warm start");
  if (opt.cycle != EMG_VCYCLE) return fail(EMG_EINVAL, "batched solves run V-cycles only");
  ps.assign(probs, probs + n);
  for (auto *p : ps)
    if (!p || p->ctx != ps[0]->ctx) return fail(EMG_EINVAL, "null problem or problems of different contexts");
  for (size_t i = 0; i < ps.size(); i++)
    for (size_t j = 0; j < i; j++)
      if (ps[i] == ps[j]) return fail(EMG_EINVAL, "a problem appears twice in the batch");
  return EMG_OK;
}

// Per-problem statistics of a finished batch and the batch's status.
static emg_status batch_stats(const std::vector<emg_problem *> &ps, const emg_solve_opts &opt, double solve_s,
                              double setup_s, emg_solve_stats *stats) {
  emg_status worst = EMG_OK;
  for (size_t i = 0; i < ps.size(); i++) {
    const Ctl c = *ps[i]->ctl_host;
    emg_solve_stats one;
    fill_stats(ps[i], c, opt.inner_cycles, &one);
    one.solve_seconds = solve_s;
    one.setup_seconds = setup_s;
    if (stats) stats[i] = one;
    if (c.done == 2) worst = EMG_EDIVERGED;
    else if (c.done == 3 && worst == EMG_OK) worst = EMG_ENOTCONV;
  }
  if (worst == EMG_EDIVERGED) return fail(worst, "a problem of the batch diverged");
  if (worst == EMG_ENOTCONV) return fail(worst, "a problem of the batch hit the cycle cap");
  return EMG_OK;
}

emg_status emg_solve_batch(emg_problem **probs, int n, const emg_solve_opts *o, emg_solve_stats *stats) {
  emg_solve_opts opt;
  std::vector<emg_problem *> ps;
  TRY(batch_args(probs, n, o, opt, ps));
  hipStream_t st = ps[0]->stream;
  const auto t0 = std::chrono::steady_clock::now();
  for (auto *p : ps) {
    HIPCK(hipStreamSynchronize(p->stream));
    TRY(prepare(p, opt, st));
  }
  HIPCK(hipStreamSynchronize(st));
  const auto t1 = std::chrono::steady_clock::now();
  Planner pl(ps);
  pl.cycles(opt.precision, std::max(1, opt.check_every), opt.nu1, opt.nu2, opt.inner_cycles);
  BatchDev dev;
  emg_status s = upload_plan(pl.plan, dev, st);
  hipGraphExec_t exec = nullptr;
  if (s == EMG_OK && opt.use_graph) {
    hipGraph_t graph;
    if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess) s = fail(EMG_EDEVICE, "capture");
    if (s == EMG_OK) {
      launch_plan(pl.plan, dev, st, opt.omega, n);
      if (hipStreamEndCapture(st, &graph) != hipSuccess) s = fail(EMG_EDEVICE, "capture end");
      else {
        if (hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess) s = fail(EMG_EDEVICE, "instantiate");
        (void)hipGraphDestroy(graph);
      }
    }
  }
  const auto t2 = std::chrono::steady_clock::now();
  while (s == EMG_OK) {
    if (exec) {
      if (hipGraphLaunch(exec, st) != hipSuccess) { s = fail(EMG_EDEVICE, "graph launch"); break; }
    } else {
      launch_plan(pl.plan, dev, st, opt.omega, n);
    }
    for (auto *p : ps)
      if (hipMemcpyAsync(p->ctl_host, p->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, st) != hipSuccess)
        s = fail(EMG_EDEVICE, "control read");
    if (hipStreamSynchronize(st) != hipSuccess) s = fail(EMG_EDEVICE, "batch cycle failed");
    bool all = true;
    for (auto *p : ps) all = all && p->ctl_host->done;
    if (all) break;
  }
  const auto t3 = std::chrono::steady_clock::now();
  if (exec) (void)hipGraphExecDestroy(exec);
  if (dev.buf) (void)hipFree(dev.buf);
  if (s != EMG_OK) return s;
  return batch_stats(ps, opt, std::chrono::duration<double>(t3 - t2).count(),
                     std::chrono::duration<double>(t1 - t0).count(), stats);
}

// The work lists of one cycle are written once to the GPU's scratch array
// and the cycle's steps are launched check_every times between host reads
// of the control blocks: the same launches, in the same order and on the
// same lists' contents, as a graph of check_every cycles (every cycle of
// such a graph walks equal lists), so results match emg_solve_batch bit for
// bit.
emg_status emg_solve_batch_noalloc(emg_problem **probs, int n, const emg_solve_opts *o, emg_solve_stats *stats) {
  emg_solve_opts opt;
  std::vector<emg_problem *> ps;
  TRY(batch_args(probs, n, o, opt, ps));
  for (auto *p : ps) {
    if (!p->fine.empty()) return fail(EMG_EINVAL, "problems with refined levels are not batched");
    if (!p->setup_done)
      return fail(EMG_ESTATE, "a problem has no hierarchy yet: solve it once after setting its moduli");
    if (opt.precision == EMG_MIXED && !p->lv[0].C32)
      return fail(EMG_ESTATE, "a problem has no FP32 copies yet: solve it once in mixed precision");
  }
  const int dev_id = ps[0]->ctx->device;
  NoAllocSlot &slot = g_noalloc[dev_id];
  if (!slot.ptr) return fail(EMG_ESTATE, "the device's scratch array was not looked up");
  bool expected = false;
  if (!slot.busy.compare_exchange_strong(expected, true))
    return fail(EMG_EBUSY, "the device's allocation-free scratch is in use by another call");
  struct Release {
    NoAllocSlot &s;
    ~Release() { s.busy.store(false); }
  } release{slot};
  HIPCK(hipSetDevice(dev_id));
  hipStream_t st = ps[0]->stream;
  const auto t0 = std::chrono::steady_clock::now();
  for (auto *p : ps) {
    HIPCK(hipStreamSynchronize(p->stream));
    TRY(prepare(p, opt, st));
  }
  Planner pl(ps);
  pl.cycles(opt.precision, 1, opt.nu1, opt.nu2, opt.inner_cycles);
  BatchDev dev;
  emg_status s = upload_plan_fixed(pl.plan, slot.ptr, EMG_NOALLOC_SCRATCH_BYTES, dev, st);
  HIPCK(hipStreamSynchronize(st));
  const auto t1 = std::chrono::steady_clock::now();
  const int k = std::max(1, opt.check_every);
  while (s == EMG_OK) {
    for (int c = 0; c < k; c++) launch_plan(pl.plan, dev, st, opt.omega, n);
    if (hipGetLastError() != hipSuccess) { s = fail(EMG_EDEVICE, "batched launch failed"); break; }
    for (auto *p : ps)
      if (hipMemcpyAsync(p->ctl_host, p->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, st) != hipSuccess)
        s = fail(EMG_EDEVICE, "control read");
    if (hipStreamSynchronize(st) != hipSuccess) s = fail(EMG_EDEVICE, "batch cycle failed");
    bool all = true;
    for (auto *p : ps) all = all && p->ctl_host->done;
    if (all) break;
  }
  const auto t2 = std::chrono::steady_clock::now();
  if (s != EMG_OK) {
    (void)hipStreamSynchronize(st);
    return s;
  }
  return batch_stats(ps, opt, std::chrono::duration<double>(t2 - t1).count(),
                     std::chrono::duration<double>(t1 - t0).count(), stats);
}

// ---- serving ----

emg_status emg_server_create(emg_ctx *ctx, int max_slots, const emg_solve_opts *o, emg_server **out) {
  if (!ctx || !out || max_slots < 1 || max_slots > 1024) return fail(EMG_EINVAL, "bad context, slots or output");
  emg_server *S = new emg_server;
  S->ctx = ctx;
  S->slots = max_slots;
  emg_default_opts(&S->opt);
  if (o) S->opt = *o;
  if ((S->opt.precision != EMG_FP64 && S->opt.precision != EMG_MIXED) || S->opt.nu1 < 1 || S->opt.nu2 < 0 ||
      S->opt.nu1 > 16 || S->opt.nu2 > 16 || !(S->opt.omega > 0.0 && S->opt.omega < 2.0) || S->opt.warm_start ||
      S->opt.cycle != EMG_VCYCLE || S->opt.inner_cycles < 1 || S->opt.inner_cycles > 4 ||
      (S->opt.inner_cycles > 1 && S->opt.precision != EMG_MIXED)) {
    delete S;
    return fail(EMG_EINVAL, "bad solve options");
  }
  S->t0 = std::chrono::steady_clock::now();
  if (hipSetDevice(ctx->device) != hipSuccess || hipStreamCreateWithFlags(&S->stream, hipStreamNonBlocking) != hipSuccess) {
    delete S;
    return fail(EMG_EDEVICE, "stream creation failed");
  }
  if (hipStreamCreateWithFlags(&S->prep_stream, hipStreamNonBlocking) != hipSuccess) {
    (void)hipStreamDestroy(S->stream);
    delete S;
    return fail(EMG_EDEVICE, "stream creation failed");
  }
  {
    std::lock_guard<std::mutex> lk(ctx->mu);
    if (ctx->closing) {
      (void)hipStreamDestroy(S->stream);
      (void)hipStreamDestroy(S->prep_stream);
      delete S;
      return fail(EMG_ESTATE, "context is being destroyed");
    }
    ctx->live += 1;
  }
  S->th = std::thread(serve_loop, S);
  S->prep = std::thread(prep_loop, S);
  *out = S;
  return EMG_OK;
}

emg_status emg_server_submit(emg_server *S, const emg_request *req, uint64_t *ticket) {
  if (!S || !req || !ticket || !req->C) return fail(EMG_EINVAL, "null argument");
  std::vector<Geom> gs;
  TRY(level_chain(&req->dom, gs));
  Served *r = new Served;
  r->dom = req->dom;
  const Geom &g = gs[0];
  const int D = req->dom.dim, nc = req->dom.kind == EMG_MOD_ISO ? 2 : (D == 3 ? 21 : 6), ne = D == 3 ? 6 : 3;
  r->on_device = (req->flags & EMG_REQ_DEVICE) != 0;
  if (r->on_device) {   // borrowed device arrays
    r->pC = req->C;
    r->peps = req->eps0;
    r->pbody = req->body;
    for (int f = 0; f < 2 * D; f++) r->pface[f] = g.per[f / 2] ? nullptr : req->face[f];
  } else {              // host arrays are copied now
    r->C.assign(req->C, req->C + (size_t)nc * g.N);
    if (req->eps0) r->eps.assign(req->eps0, req->eps0 + (size_t)ne * g.N);
    if (req->body) r->body.assign(req->body, req->body + (size_t)D * g.N);
    for (int f = 0; f < 2 * D; f++)
      if (req->face[f] && !g.per[f / 2]) r->face[f].assign(req->face[f], req->face[f] + (size_t)D * (g.N / g.m[f / 2]));
    r->pC = r->C.data();
    r->peps = r->eps.empty() ? nullptr : r->eps.data();
    r->pbody = r->body.empty() ? nullptr : r->body.data();
    for (int f = 0; f < 2 * D; f++) r->pface[f] = r->face[f].empty() ? nullptr : r->face[f].data();
  }
  r->u_out = req->u_out;
  r->need = footprint_of(gs, D, req->dom.kind, S->opt.precision == EMG_MIXED);
  std::lock_guard<std::mutex> lk(S->mu);
  if (S->stop) {
    delete r;
    return fail(EMG_ESTATE, "server is shutting down");
  }
  r->ticket = S->next++;
  r->t_submit = S->now();
  S->all[r->ticket] = r;
  S->pending.push_back(r);
  S->cv_prep.notify_all();
  *ticket = r->ticket;
  return EMG_OK;
}

static void ticket_info(const Served *r, emg_ticket_info *info) {
  info->done = r->done;
  info->status = r->status;
  info->stats = r->stats;
  info->t_submit = r->t_submit;
  info->t_admit = r->t_admit;
  info->t_ready = r->t_ready;
  info->t_done = r->t_done;
}

emg_status emg_server_poll(emg_server *S, uint64_t ticket, emg_ticket_info *info) {
  if (!S || !info) return fail(EMG_EINVAL, "null argument");
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->all.find(ticket);
  if (it == S->all.end()) return fail(EMG_EINVAL, "unknown ticket");
  ticket_info(it->second, info);
  return EMG_OK;
}

emg_status emg_server_wait(emg_server *S, uint64_t ticket, emg_ticket_info *info) {
  if (!S || !info) return fail(EMG_EINVAL, "null argument");
  std::unique_lock<std::mutex> lk(S->mu);
  auto it = S->all.find(ticket);
  if (it == S->all.end()) return fail(EMG_EINVAL, "unknown ticket");
  Served *r = it->second;
  S->cv_done.wait(lk, [&] { return r->done; });
  ticket_info(r, info);
  return EMG_OK;
}

emg_status emg_server_now(emg_server *S, double *t) {
  if (!S || !t) return fail(EMG_EINVAL, "null argument");
  *t = S->now();
  return EMG_OK;
}

emg_status emg_server_destroy(emg_server *S) {
  if (!S) return EMG_OK;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
    S->cv.notify_all();
    S->cv_prep.notify_all();
  }
  if (S->prep.joinable()) S->prep.join();
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->cv.notify_all();
  }
  if (S->th.joinable()) S->th.join();
  for (auto &kv : S->pool) emg_problem_destroy(kv.second);
  for (auto &kv : S->all) delete kv.second;
  if (S->dev.buf) (void)hipFree(S->dev.buf);
  if (S->stream) (void)hipStreamDestroy(S->stream);
  if (S->prep_stream) (void)hipStreamDestroy(S->prep_stream);
  emg_ctx *c = S->ctx;
  delete S;
  ctx_release(c);
  return EMG_OK;
}

// ---- block-structured AMR ----

// Refined level `level` (the next one) as the union of `boxes`: checks
// bounds and nesting, builds the bounding array and its valid-node mask.
static emg_status add_refined_level(emg_problem *p, int level, const emg_box *boxes, int nbox) {
  if (!p || !boxes || nbox < 1) return fail(EMG_EINVAL, "null argument or no boxes");
  const int k = (int)p->fine.size() + 1;
  if (level != k)
    return fail(EMG_ESTATE, "refined levels are added in order; the next one is level " + std::to_string(k));
  const Geom &pg = parent_geom(p, k);
  const Fine *par = k == 1 ? nullptr : &p->fine[k - 2];
  Fine F;
  F.g.dim = p->D;
  for (int i = 0; i < nbox; i++) {
    Box bx{};
    for (int a = 0; a < 3; a++) {
      if (a >= p->D) continue;
      const int64_t lo = boxes[i].lo[a], hi = boxes[i].hi[a];
      if (lo % 2 || hi % 2 || hi <= lo) return fail(EMG_EINVAL, "box bounds must be even with hi > lo");
      if (lo < 0 || hi > (int64_t)1 << 30) return fail(EMG_EINVAL, "box bounds out of range");
      if (k == 1 && pg.per[a]) return fail(EMG_EINVAL, "refined boxes need non-periodic axes");
      if (k == 1 && (lo / 2 - 2 < 0 || hi / 2 + 2 > pg.m[a] - 1))
        return fail(EMG_EINVAL, "box must nest inside the base grid with two coarse cells to spare");
      bx.lo[a] = (int)lo;
      bx.hi[a] = (int)hi;
    }
    if (par) {   // every coarse node of the box grown by two coarse cells is a valid node of level k-1
      const int o[3] = {par->b.lo[0] - 1, par->b.lo[1] - 1, p->D == 3 ? par->b.lo[2] - 1 : 0};
      int q0[3] = {0, 0, 0}, q1[3] = {0, 0, 0};
      for (int a = 0; a < p->D; a++) {
        q0[a] = bx.lo[a] / 2 - 2 - o[a];
        q1[a] = bx.hi[a] / 2 + 2 - o[a];
        if (q0[a] < 0 || q1[a] > par->g.m[a] - 1)
          return fail(EMG_EINVAL, "box must nest inside the valid nodes of the coarser level with two coarse cells "
                                  "to spare");
      }
      for (int z = q0[2]; z <= q1[2]; z++)
        for (int y = q0[1]; y <= q1[1]; y++)
          for (int x = q0[0]; x <= q1[0]; x++)
            if (!par->hmask[((size_t)z * par->g.m[1] + y) * par->g.m[0] + x])
              return fail(EMG_EINVAL, "box must nest inside the valid nodes of the coarser level with two coarse "
                                      "cells to spare");
    }
    F.boxes.push_back(bx);
  }
  for (int a = 0; a < 3; a++) {
    if (a < p->D) {
      int lo = F.boxes[0].lo[a], hi = F.boxes[0].hi[a];
      for (auto &bx : F.boxes) {
        lo = std::min(lo, bx.lo[a]);
        hi = std::max(hi, bx.hi[a]);
      }
      F.b.lo[a] = lo;
      F.b.hi[a] = hi;
      F.g.m[a] = hi - lo + 3;
      F.g.per[a] = 0;
      F.g.h[a] = pg.h[a] / 2.0;
      F.g.bc[2 * a] = F.g.bc[2 * a + 1] = EMG_BC_DIRICHLET;
    } else {
      F.b.lo[a] = F.b.hi[a] = 0;
      F.g.m[a] = 1;
      F.g.per[a] = 1;
      F.g.h[a] = 1.0;
      F.g.bc[2 * a] = F.g.bc[2 * a + 1] = EMG_BC_PERIODIC;
    }
  }
  F.g.N = (long long)F.g.m[0] * F.g.m[1] * F.g.m[2];
  if (F.g.N >= kMaxNodes) return fail(EMG_EINVAL, "level too large (2^29 stored nodes at most in its bounding box)");
  F.g.SC = moduli_stride(F.g.N);
  // valid-node mask over the bounding array; counts of valid and covered-coarse nodes
  F.hmask.assign((size_t)F.g.N, 0);
  for (auto &bx : F.boxes) {
    const int z0 = p->D == 3 ? bx.lo[2] - F.b.lo[2] + 1 : 0, z1 = p->D == 3 ? bx.hi[2] - F.b.lo[2] + 1 : 0;
    for (int z = z0; z <= z1; z++)
      for (int y = bx.lo[1] - F.b.lo[1] + 1; y <= bx.hi[1] - F.b.lo[1] + 1; y++)
        for (int x = bx.lo[0] - F.b.lo[0] + 1; x <= bx.hi[0] - F.b.lo[0] + 1; x++)
          F.hmask[((size_t)z * F.g.m[1] + y) * F.g.m[0] + x] = 1;
  }
  for (long long n = 0; n < F.g.N; n++) {
    if (!F.hmask[n]) continue;
    F.nvalid++;
    const int x = int(n % F.g.m[0]), y = int((n / F.g.m[0]) % F.g.m[1]), z = int(n / ((long long)F.g.m[0] * F.g.m[1]));
    const bool even = (F.b.lo[0] - 1 + x) % 2 == 0 && (F.b.lo[1] - 1 + y) % 2 == 0 &&
                      (p->D == 2 || (F.b.lo[2] - 1 + z) % 2 == 0);
    if (even) F.ncov++;
  }
  // active tiles: those holding a valid node or a node next to one (a ghost);
  // passes over the level skip the others, whose nodes no valid row reads
  {
    std::vector<unsigned char> near((size_t)F.g.N, 0);
    const int m0 = F.g.m[0], m1 = F.g.m[1], m2 = F.g.m[2];
    const int zr = p->D == 3 ? 1 : 0;
    for (int z = 0; z < m2; z++)
      for (int y = 0; y < m1; y++)
        for (int x = 0; x < m0; x++) {
          if (!F.hmask[((size_t)z * m1 + y) * m0 + x]) continue;
          for (int dz = -zr; dz <= zr; dz++)
            for (int dy = -1; dy <= 1; dy++)
              for (int dx = -1; dx <= 1; dx++) {
                const int X = x + dx, Y = y + dy, Z = z + dz;
                if (X >= 0 && X < m0 && Y >= 0 && Y < m1 && Z >= 0 && Z < m2) near[((size_t)Z * m1 + Y) * m0 + X] = 1;
              }
        }
    auto any_near = [&](int x0, int x1, int y0, int y1, int z) {
      for (int y = y0; y <= std::min(y1, m1 - 1); y++)
        for (int x = x0; x <= std::min(x1, m0 - 1); x++)
          if (near[((size_t)z * m1 + y) * m0 + x]) return true;
      return false;
    };
    std::vector<int> gr, st;
    const int gx = (m0 + BX - 1) / BX, gy = (m1 + BY - 1) / BY;
    for (int z = 0; z < m2; z++)
      for (int ty = 0; ty < gy; ty++)
        for (int tx = 0; tx < gx; tx++)
          if (any_near(tx * BX, tx * BX + BX - 1, ty * BY, ty * BY + BY - 1, z)) gr.push_back((z * gy + ty) * gx + tx);
    const Split sp = split_of(F.g);
    for (int tz = 0; tz < sp.ntz; tz++)
      for (int ty = 0; ty < sp.nty; ty++)
        for (int tx = 0; tx < sp.ntx; tx++) {
          const int x0 = sp.lo[0] + tx * BX, y0 = sp.lo[1] + ty * BY;
          if (any_near(x0, std::min(x0 + BX - 1, sp.hi[0]), y0, std::min(y0 + BY - 1, sp.hi[1]), sp.lo[2] + tz))
            st.push_back((tz * sp.nty + ty) * sp.ntx + tx);
        }
    F.nact_gr = (long long)gr.size();
    F.nact_st = (long long)st.size();
    TRY(dalloc(p, &F.act_gr, std::max<size_t>(gr.size(), 1)));
    TRY(dalloc(p, &F.act_st, std::max<size_t>(st.size(), 1)));
    HIPCK(hipMemcpyAsync(F.act_gr, gr.data(), sizeof(int) * gr.size(), hipMemcpyHostToDevice, p->stream));
    HIPCK(hipMemcpyAsync(F.act_st, st.data(), sizeof(int) * st.size(), hipMemcpyHostToDevice, p->stream));
    HIPCK(hipStreamSynchronize(p->stream));   // the host vectors go out of scope
  }
  const size_t nd = (size_t)p->D * F.g.N;
  TRY(dalloc(p, &F.vm, (size_t)F.g.N));
  HIPCK(hipMemcpyAsync(F.vm, F.hmask.data(), (size_t)F.g.N, hipMemcpyHostToDevice, p->stream));
  TRY(dalloc(p, &F.C, (size_t)p->nc * F.g.SC));
  TRY(dalloc(p, &F.f, nd));
  TRY(dalloc(p, &F.u, nd));
  TRY(dalloc(p, &F.rr, nd));
  TRY(dalloc(p, &F.t, nd));
  TRY(dalloc(p, &F.e[0], nd));
  TRY(dalloc(p, &F.e[1], nd));
  // nodes outside the active tiles are never written by the cycle: start
  // every per-node array at zero so they stay finite
  for (double *a : {F.f, F.rr, F.t, F.e[0], F.e[1]}) launch_fill<double>(p, (long long)nd, a, 0.0);
  if (!p->amr_u0) {
    const size_t nd0 = (size_t)p->D * p->lv[0].g.N;
    TRY(dalloc(p, &p->amr_u0, nd0));
    TRY(dalloc(p, &p->amr_f0, nd0));
    launch_fill<double>(p, (long long)nd0, p->amr_u0, 0.0);
  }
  launch_fill<double>(p, (long long)nd, F.u, 0.0);
  p->fine.push_back(std::move(F));
  // norm partials of every level's composite rows
  long long parts = grid_blocks(p->lv[0].g);
  for (auto &G : p->fine) parts += grid_blocks(G.g);
  TRY(dalloc(p, &p->amr_partial, (size_t)parts));
  p->amr_nparts = parts;
  destroy_graphs(p);
  p->setup_done = p->rhs_ready = p->mixed_ready = false;
  HIPCK(hipStreamSynchronize(p->stream));
  return EMG_OK;
}

emg_status emg_set_level_boxes(emg_problem *p, int level, const emg_box *boxes, int nbox) {
  return add_refined_level(p, level, boxes, nbox);
}

emg_status emg_amr_add_level(emg_problem *p, const int64_t lo[3], const int64_t hi[3]) {
  if (!p || !lo || !hi) return fail(EMG_EINVAL, "null argument");
  emg_box b;
  for (int a = 0; a < 3; a++) {
    b.lo[a] = lo[a];
    b.hi[a] = hi[a];
  }
  return add_refined_level(p, (int)p->fine.size() + 1, &b, 1);
}

emg_status emg_amr_level_valid(emg_problem *p, int level, unsigned char *mask, int64_t *nvalid) {
  if (!p) return fail(EMG_EINVAL, "null problem");
  if (level < 1 || level > (int)p->fine.size()) return fail(EMG_EINVAL, "no such refined level");
  const Fine &F = p->fine[level - 1];
  if (mask) std::memcpy(mask, F.hmask.data(), F.hmask.size());
  if (nvalid) *nvalid = F.nvalid;
  return EMG_OK;
}

static emg_status fine_level(emg_problem *p, int level, Fine **F) {
  if (!p) return fail(EMG_EINVAL, "null problem");
  if (level < 1 || level > (int)p->fine.size()) return fail(EMG_EINVAL, "no such refined level");
  *F = &p->fine[level - 1];
  return EMG_OK;
}

emg_status emg_amr_num_levels(emg_problem *p, int *levels) {
  if (!p || !levels) return fail(EMG_EINVAL, "null argument");
  *levels = (int)p->fine.size();
  return EMG_OK;
}

emg_status emg_amr_level_shape(emg_problem *p, int level, int64_t m[3]) {
  Fine *F;
  TRY(fine_level(p, level, &F));
  for (int a = 0; a < 3; a++) m[a] = F->g.m[a];
  return EMG_OK;
}

emg_status emg_amr_set_moduli(emg_problem *p, int level, const double *C, int on_device) {
  Fine *F;
  TRY(fine_level(p, level, &F));
  if (!C) return fail(EMG_EINVAL, "null moduli");
  TRY(copy_planes(p, F->C, F->g.SC, C, F->g.N, p->nc, on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice));
  F->moduli_set = true;
  p->setup_done = p->rhs_ready = p->mixed_ready = false;
  return EMG_OK;
}

emg_status emg_amr_set_eigenstrain(emg_problem *p, int level, const double *e, int on_device) {
  Fine *F;
  TRY(fine_level(p, level, &F));
  p->rhs_ready = p->setup_done = false;
  if (!e) {
    F->eps = nullptr;
    return EMG_OK;
  }
  if (!F->eps) TRY(dalloc(p, &F->eps, (size_t)p->ne * F->g.N));
  return copy_in(p, F->eps, e, (size_t)p->ne * F->g.N, on_device);
}

emg_status emg_amr_set_body_force(emg_problem *p, int level, const double *b, int on_device) {
  Fine *F;
  TRY(fine_level(p, level, &F));
  p->rhs_ready = false;
  if (!b) {
    F->body = nullptr;
    return EMG_OK;
  }
  if (!F->body) TRY(dalloc(p, &F->body, (size_t)p->D * F->g.N));
  return copy_in(p, F->body, b, (size_t)p->D * F->g.N, on_device);
}

emg_status emg_amr_get_displacement(emg_problem *p, int level, double *u, int on_device) {
  Fine *F;
  TRY(fine_level(p, level, &F));
  if (!u) return fail(EMG_EINVAL, "null output");
  return copy_out(p, u, F->u, (size_t)p->D * F->g.N, on_device);
}

emg_status emg_amr_set_displacement(emg_problem *p, int level, const double *u, int on_device) {
  Fine *F;
  TRY(fine_level(p, level, &F));
  if (!u) return fail(EMG_EINVAL, "null input");
  return copy_in(p, F->u, u, (size_t)p->D * F->g.N, on_device);
}

emg_status emg_amr_residual(emg_problem *p, int level, double *r_dev, double *norm) {
  if (!p || !r_dev) return fail(EMG_EINVAL, "null argument");
  if (p->fine.empty()) return fail(EMG_ESTATE, "no refined levels");
  if (level < 0 || level > (int)p->fine.size()) return fail(EMG_EINVAL, "no such level");
  TRY(setup(p));
  TRY(assemble_rhs(p));
  if (p->D == 2) {
    amr_sync<2>(p, p->amr_u0, nullptr);
    amr_residual<2>(p, nullptr);
  } else {
    amr_sync<3>(p, p->amr_u0, nullptr);
    amr_residual<3>(p, nullptr);
  }
  HIPCK(hipGetLastError());
  if (norm) {
    std::vector<double> parts(p->amr_nparts);
    HIPCK(hipMemcpyAsync(parts.data(), p->amr_partial, sizeof(double) * parts.size(), hipMemcpyDeviceToHost,
                         p->stream));
    HIPCK(hipStreamSynchronize(p->stream));
    double s = 0.0;
    for (double v : parts) s += v;
    *norm = std::sqrt(s);
  }
  if (level == 0) return copy_out(p, r_dev, p->lv[0].f64, (size_t)p->D * p->lv[0].g.N, 1);
  return copy_out(p, r_dev, p->fine[level - 1].rr, (size_t)p->D * p->fine[level - 1].g.N, 1);
}

}  // extern "C"
