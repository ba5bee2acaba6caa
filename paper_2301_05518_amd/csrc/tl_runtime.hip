// Host runtime behind the C ABI of twolink.h: contexts, argument validation,
// resident plans (packing, work lists, tuning, HIP graph capture), reductions.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <list>
#include <map>
#include <new>
#include <sstream>
#include <string>
#include <utility>
#include <vector>

#include <unistd.h>

#include "tl_internal.h"
#include "twolink.h"

using tl::StepConfig;
using tl::StepGroup;

static_assert(TL_F64 == tl::F64 && TL_F32 == tl::F32 && TL_F16S == tl::F16S && TL_BF16 == tl::BF16,
              "precision codes");
static_assert((TL_W12 & 3) == 0 && (TL_ONELINK & 3) == 0 && TL_W12 != TL_ONELINK,
              "TL_W12 and TL_ONELINK are bits above the precision codes");

// A tuned step tiling: cfg, and when cfg runs two steps per launch (variant 8) the one-step
// tiling `single` that an odd step count ends with (single.variant < 0: none).
struct Tuned {
  StepConfig cfg{0, 256, 4, 0, 0, 0, 0};
  StepConfig single{-1, 0, 0, 0, 0, 0, 0};
};

struct tl_ctx {
  int device = -1;
  hipStream_t stream = nullptr;
  std::string err;
  int n_cu = 0;
  std::string arch;
  bool log = false;
  bool fault_alloc = false;   // TL_FAULT=alloc: internal allocations report failure
  bool fault_launch = false;  // TL_FAULT=launch: launches report failure without running
  bool big_lds = false;       // dynamic-LDS limit raised for the LDS-staged step kernels
  void* scratch = nullptr;
  size_t scratch_bytes = 0;
  double* noalloc = nullptr;  // this device's fixed partial-sum area of tl_reduce_noalloc
  std::string noalloc_err;    // why it is missing (lookup failed at tl_create)
  std::map<std::string, Tuned> tune;       // tuned step tilings by workload key
  std::string tune_file;                   // TL_TUNE_CACHE: tuning results persisted across processes
  std::list<std::pair<std::string, tl_plan*>> smear_plans;   // tl_smear(TL_GRAPH) plans, most recent first
  tl_ctx_stats stats{};
};

namespace {

thread_local std::string g_create_err;

int vfail(tl_ctx* c, int code, const char* fmt, va_list ap) {
  char buf[1024];
  vsnprintf(buf, sizeof buf, fmt, ap);
  if (c) c->err = buf; else g_create_err = buf;
  return code;
}

int fail(tl_ctx* c, int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vfail(c, code, fmt, ap);
  va_end(ap);
  return code;
}

// No C++ exception may cross the C interface: an entry point whose host-side bookkeeping
// throws (in practice a failed host allocation) reports TL_ERR_NOMEM instead.
int host_failure(tl_ctx* c) noexcept {
  try {
    if (c) c->err = "host allocation failed"; else g_create_err = "host allocation failed";
  } catch (...) {
  }
  return TL_ERR_NOMEM;
}

#define HIP_TRY(ctx, expr)                                                                     \
  do {                                                                                         \
    hipError_t e_ = (expr);                                                                    \
    if (e_ != hipSuccess) return fail((ctx), TL_ERR_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

#define TL_TRY(expr)            \
  do {                          \
    int rc_ = (expr);           \
    if (rc_ != TL_OK) return rc_; \
  } while (0)

// Makes the context's device current for the duration of a call.
struct DeviceGuard {
  int prev = -1;
  bool ok = true;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) ok = hipSetDevice(dev) == hipSuccess;
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

// Makes the context's device current for the rest of the enclosing entry point, or fails
// the call (nothing queued) when the runtime refuses to switch to it.
#define TL_ON_DEVICE(c)                                                                  \
  DeviceGuard dg_((c)->device);                                                          \
  if (!dg_.ok) return fail((c), TL_ERR_DEVICE, "hipSetDevice(%d) failed", (c)->device)

// Internal format code of a public precision argument (precision, optionally | TL_W12 and
// | TL_ONELINK), -1 if invalid.
int fmt_code(int p) {
  const int base = p & ~(TL_W12 | TL_ONELINK);
  if (base < TL_F64 || base > TL_BF16) return -1;
  return base | ((p & TL_W12) ? tl::W12 : 0) | ((p & TL_ONELINK) ? tl::ONE : 0);
}

bool valid_prec(int p) { return fmt_code(p) >= 0; }

int check_geom(tl_ctx* c, const tl_geom* g) {
  if (!g) return fail(c, TL_ERR_ARG, "geometry is NULL");
  for (int d = 0; d < 4; d++)
    if (g->L[d] < 1 || g->L[d] > 4096)
      return fail(c, TL_ERR_SHAPE, "extent L[%d] = %d outside [1, 4096]", d, g->L[d]);
  const int64_t v3 = (int64_t)g->L[0] * g->L[1] * g->L[2];
  if (v3 > (int64_t(1) << 27)) return fail(c, TL_ERR_SHAPE, "slice volume %lld exceeds 2^27 sites", (long long)v3);
  return TL_OK;
}

int64_t vol3(const tl_geom& g) { return (int64_t)g.L[0] * g.L[1] * g.L[2]; }

int need_device(tl_ctx* c) {
  if (c->device < 0) return fail(c, TL_ERR_DEVICE, "host-only context (created with device -1) cannot run device work");
  return TL_OK;
}

int dev_alloc(tl_ctx* c, void** p, size_t bytes) {
  *p = nullptr;
  if (bytes == 0) bytes = 256;
  if (c->fault_alloc) return fail(c, TL_ERR_NOMEM, "device allocation of %zu bytes failed (TL_FAULT=alloc)", bytes);
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    *p = nullptr;
    return fail(c, TL_ERR_NOMEM, "hipMalloc(%zu): %s", bytes, hipGetErrorString(e));
  }
  return TL_OK;
}

// Queue one library launch; TL_FAULT=launch makes it fail before anything is queued.
template <class F>
int launch(tl_ctx* c, const char* what, F&& f) {
  if (c->fault_launch) return fail(c, TL_ERR_HIP, "%s launch failed (TL_FAULT=launch)", what);
  const hipError_t e = f();
  if (e != hipSuccess) return fail(c, TL_ERR_HIP, "%s launch: %s", what, hipGetErrorString(e));
  return TL_OK;
}

// Context scratch: grows on demand; stream-ordered reuse is safe because every
// user queues on the context stream and waits before overwriting host tables.
int ctx_scratch(tl_ctx* c, size_t bytes, char** out) {
  if (bytes > c->scratch_bytes) {
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    if (c->scratch) HIP_TRY(c, hipFree(c->scratch));
    c->scratch = nullptr;
    c->scratch_bytes = 0;
    void* p = nullptr;
    TL_TRY(dev_alloc(c, &p, bytes));
    c->scratch = p;
    c->scratch_bytes = bytes;
  }
  *out = static_cast<char*>(c->scratch);
  return TL_OK;
}

// Synchronous upload of a small host table onto the context stream.
int upload(tl_ctx* c, void* dst, const void* src, size_t bytes) {
  if (bytes == 0) return TL_OK;
  HIP_TRY(c, hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return TL_OK;
}

size_t align256(size_t v) { return (v + 255) / 256 * 256; }

// Slot of slice t in a two-link field built for w_slices (NULL = all slices).
int slot_of(const tl_geom& g, const int32_t* w_slices, int n_w, int t) {
  if (t < 0 || t >= g.L[3]) return -1;
  if (!w_slices) return t;
  for (int j = 0; j < n_w; j++)
    if (w_slices[j] == t) return j;
  return -1;
}

int check_wslices(tl_ctx* c, const tl_geom& g, const int32_t* w_slices, int n_w) {
  if (!w_slices) return TL_OK;
  if (n_w < 1 || n_w > g.L[3]) return fail(c, TL_ERR_ARG, "n_w_slices = %d outside [1, Lt=%d]", n_w, g.L[3]);
  for (int j = 0; j < n_w; j++)
    if (w_slices[j] < 0 || w_slices[j] >= g.L[3])
      return fail(c, TL_ERR_SHAPE, "w_slices[%d] = %d outside [0, %d)", j, w_slices[j], g.L[3]);
  return TL_OK;
}

// Coefficients of one smearing step, out = alpha in + beta sum_hops:
//   two-link (eq. tlSmear with eq. tlLapl1): in + (s/4)(sum_hops - 6 in), s = sigma/n
//   one-link (Sec. 2, nabla^2 = H - 6):      in + s (sum_hops - 6 in)
void step_coeffs(bool one, int n_steps, double sigma, double* alpha, double* beta) {
  const double s = sigma / (double)n_steps;
  const double q = one ? s : 0.25 * s;
  *alpha = 1.0 - 6.0 * q;
  *beta = q;
}

// Largest sigma/n for which every step factor lies in [-1, 1] (a contraction for unitary links).
double max_step(bool one) { return one ? 1.0 / 6.0 : 2.0 / 3.0; }

// A step configuration a cache entry or TL_TILE may name.
bool valid_cfg(const StepConfig& g) {
  return g.variant >= 0 && g.variant <= 8 && g.block >= 64 && g.block <= (g.variant >= 5 ? 512 : 256) &&
         g.block % 64 == 0 && g.tz >= 1 && (g.nt == 0 || g.nt == 1) && (g.flip == 0 || g.flip == 1) &&
         g.width >= 0 && g.width <= 4;
}

// Up to 7 comma-separated integers "variant,block,tz,grid,nt,flip,width" at v into c (missing
// ones 0); returns how many were read and sets *end past them.
int parse_cfg(const char* v, StepConfig* c, const char** end) {
  int* f[7] = {&c->variant, &c->block, &c->tz, &c->grid, &c->nt, &c->flip, &c->width};
  *c = StepConfig{};
  int n = 0;
  const char* q = v;
  while (n < 7) {
    char* e = nullptr;
    const long x = strtol(q, &e, 10);
    if (e == q || x < -(1L << 30) || x > (1L << 30)) break;
    *f[n++] = (int)x;
    q = e;
    if (*q != ',') break;
    q++;
  }
  *end = q;
  return n;
}

// "variant,block,tz,grid[,nt[,flip[,width]]]" with an optional ";..." naming the one-step tiling
// of a two-step one (six or seven fields); n_min: fields the first part needs.
bool parse_tuned(const char* v, int n_min, Tuned* out) {
  Tuned t;
  const char* end = nullptr;
  const int n = parse_cfg(v, &t.cfg, &end);
  if (n < n_min || !valid_cfg(t.cfg)) return false;
  if (*end == ';') {
    if (n < 6 || parse_cfg(end + 1, &t.single, &end) < 6 || *end != '\0' || !valid_cfg(t.single) ||
        t.single.variant == 8)
      return false;
  } else if (*end != '\0') {
    return false;
  }
  if (t.cfg.variant != 8) t.single = StepConfig{-1, 0, 0, 0, 0, 0, 0};
  else if (t.single.variant < 0) t.single = StepConfig{0, 256, 4, 0, 0, 0, 0};
  *out = t;
  return true;
}

std::string cfg_text(const StepConfig& g) {
  return std::to_string(g.variant) + "," + std::to_string(g.block) + "," + std::to_string(g.tz) + "," +
         std::to_string(g.grid) + "," + std::to_string(g.nt) + "," + std::to_string(g.flip) +
         (g.width > 0 ? "," + std::to_string(g.width) : std::string());
}

// Tuning cache file (TL_TUNE_CACHE): a JSON object {"<workload key>": "variant,block,tz,grid,nt,flip[,width]",
// ...} (a two-step tiling followed by ";" and its one-step companion).  The keys (architecture,
// precision code, group width, launch mode, each group's dims and RHS) hold no quote or
// backslash, so the file is read and written with plain string handling; a missing,
// unreadable or malformed file is an empty cache.
void tune_file_load(tl_ctx* c) {
  std::ifstream in(c->tune_file);
  if (!in) return;
  std::stringstream ss;
  ss << in.rdbuf();
  const std::string t = ss.str();
  size_t pos = 0;
  while (true) {
    const size_t k0 = t.find('"', pos);
    if (k0 == std::string::npos) break;
    const size_t k1 = t.find('"', k0 + 1);
    const size_t v0 = k1 == std::string::npos ? k1 : t.find('"', k1 + 1);
    const size_t v1 = v0 == std::string::npos ? v0 : t.find('"', v0 + 1);
    if (v1 == std::string::npos) break;
    Tuned tu;
    const std::string val = t.substr(v0 + 1, v1 - v0 - 1);
    if (parse_tuned(val.c_str(), 6, &tu)) c->tune[t.substr(k0 + 1, k1 - k0 - 1)] = tu;
    pos = v1 + 1;
  }
}

// Rewrite the whole file (a temporary then a rename, so a reader never sees half a file).
void tune_file_save(const tl_ctx* c) {
  const std::string tmp = c->tune_file + ".tmp" + std::to_string((long)getpid());
  {
    std::ofstream out(tmp);
    if (!out) return;
    out << "{\n";
    size_t k = 0;
    for (const auto& kv : c->tune) {
      const Tuned& g = kv.second;
      out << "  \"" << kv.first << "\": \"" << cfg_text(g.cfg)
          << (g.cfg.variant == 8 ? ";" + cfg_text(g.single) : std::string()) << "\""
          << (++k < c->tune.size() ? ",\n" : "\n");
    }
    out << "}\n";
    if (!out) return;
  }
  (void)std::rename(tmp.c_str(), c->tune_file.c_str());
}

}  // namespace

// ====================================================================== plans

struct tl_plan {
  tl_ctx* ctx = nullptr;
  int prec = 0, n_steps = 0;     // prec: internal format code (tl::vprec(prec) for the vectors)
  double sigma = 0.0, alpha = 1.0, beta = 0.0;
  unsigned flags = 0;

  struct JobCopy {
    tl_job job;
    std::vector<int32_t> t_of_rhs, w_slices;
    int64_t V3 = 0, Vp = 0;
    std::vector<int> res_index;   // job RHS r -> resident RHS index
  };
  std::vector<JobCopy> jobs;

  struct Res {
    int job, r, slot;
    int64_t off;                  // byte offset in each resident buffer
  };
  std::vector<Res> res;           // resident order: grouped by (job, slot)

  struct Group {
    int job, slot, first, nr;     // resident RHS [first, first + nr)
  };
  std::vector<Group> groups;
  int width = 1;

  size_t buf_bytes = 0;
  char* buf[2] = {nullptr, nullptr};
  int cur = 0;

  // device tables: the step groups of both tilings (group_cap entries each), per-job pack
  // offsets, reduction fields, partials
  char* tables = nullptr;
  size_t group_cap = 0;
  int64_t* packoff_dev = nullptr;
  std::vector<int64_t> packoff_first;   // index of job j's first entry in packoff_dev
  tl::RedField* red_dev = nullptr;
  double* partials = nullptr;
  int64_t max_v3 = 0;

  // A step tiling and its work list (device table dev, host copy host).
  struct Tiling {
    StepConfig cfg{0, 256, 4, 0, 0, 0, 0};
    StepGroup* dev = nullptr;
    std::vector<StepGroup> host;
    int n_tiles = 0;
    int64_t lds = 0;                    // dynamic LDS bytes of its launches (variants 5-8)
  };
  Tiling tile;                          // the step tiling
  Tiling single;                        // when tile runs two steps per launch: the one-step
                                        // tiling of the last step of an odd count
  bool ready = false;                   // tuning done (or not requested) and tables uploaded

  hipGraphExec_t graph[2] = {nullptr, nullptr};

  tl_plan_info info{};
};

namespace {

// RHS per step group of a configuration: the plan's groups, or narrower ones (cfg.width).
int eff_width(const tl_plan* p, const StepConfig& cfg) {
  return cfg.width > 0 ? std::min(cfg.width, p->width) : p->width;
}

// Work list of a plan for one step configuration.
int make_groups(const tl_plan* p, const StepConfig& cfg, std::vector<StepGroup>* out) {
  out->clear();
  int tiles = 0;
  const int ew = eff_width(p, cfg);
  for (const auto& gr0 : p->groups) {
    for (int first = gr0.first; first < gr0.first + gr0.nr; first += ew) {   // the plan's group, or its parts
      const auto& jc = p->jobs[gr0.job];
      const tl_geom& g = jc.job.g;
      const int nr = std::min(ew, gr0.first + gr0.nr - first);
      StepGroup s{};
      const int64_t wslot = (int64_t)gr0.slot * 3 * jc.Vp * tl::kWBytes[p->prec];
      s.W = static_cast<const char*>(jc.job.W) + wslot;
      s.w_mu_stride = jc.Vp * tl::kWBytes[p->prec];
      s.psi_off = p->res[first].off;
      s.rhs_stride = nr > 1 ? p->res[first + 1].off - p->res[first].off : 0;
      s.Lx = g.L[0];
      s.Ly = g.L[1];
      s.Lz = g.L[2];
      s.Vp = (int32_t)jc.Vp;
      s.nr = nr;
      if (cfg.variant == 8) {   // two steps per launch: blocks of k rows of one y chain
        const int D = tl::hop_of(p->prec);
        const int R = (tl::vprec(p->prec) == tl::F64) ? 1 : ew;
        s.rows = tl::fuse_rows(p->prec, R, g.L[0], g.L[1], cfg.block, 160 * 1024);
        if (s.rows == 0) return TL_ERR_UNSUPPORTED;
        const int ychains = (D == 2 && !(g.L[1] & 1)) ? 2 : 1;
        s.n_xy_tiles = ychains * (g.L[1] / ychains / s.rows);
      } else if (cfg.variant >= 5) {   // full-row tiles
        s.rows = tl::lds_rows(g.L[0], g.L[1], cfg.block);
        if (s.rows == 0) return TL_ERR_UNSUPPORTED;
        s.n_xy_tiles = g.L[1] / s.rows;
      } else {
        s.rows = 0;
        s.n_xy_tiles = (int32_t)(((int64_t)g.L[0] * g.L[1] + cfg.block - 1) / cfg.block);
      }
      if (cfg.variant >= 6) {   // chains of planes z, z+2, ...: two for even Lz, one for odd (and for
        const int chains = (tl::is_one(p->prec) || (g.L[2] & 1)) ? 1 : 2;   // one-links: consecutive planes)
        const int clen = g.L[2] / chains;
        s.n_z_tiles = chains * ((clen + cfg.tz - 1) / cfg.tz);
      } else {
        s.n_z_tiles = (g.L[2] + cfg.tz - 1) / cfg.tz;
      }
      s.tile_begin = tiles;
      const int64_t nt = (int64_t)s.n_xy_tiles * s.n_z_tiles;
      if (tiles + nt > (int64_t)1 << 30) return TL_ERR_UNSUPPORTED;
      tiles += (int)nt;
      out->push_back(s);
    }
  }
  return TL_OK;
}

// Dynamic LDS bytes of a configuration (variants 5-8), -1 if it does not fit.
int64_t plan_lds(const tl_plan* p, const StepConfig& cfg, const std::vector<StepGroup>& gs) {
  if (cfg.variant < 5) return 0;
  int64_t mx = 0;
  const int R = (tl::vprec(p->prec) == tl::F64) ? 1 : eff_width(p, cfg);
  for (const auto& g : gs)
    mx = std::max(mx, cfg.variant == 8 ? tl::lds_bytes_fuse2(p->prec, R, g.Lx, g.rows)
                                       : tl::lds_bytes(p->prec, R, g.Lx, g.rows));
  return mx <= 160 * 1024 ? mx : -1;
}

// Whether cfg applies to this plan (its work list exists and fits in LDS); reason on failure.
bool tiling_applies(const tl_plan* p, const StepConfig& cfg, const char** reason) {
  if (tl::is_one(p->prec) && cfg.variant != 0 && cfg.variant != 4 && cfg.variant != 7 && cfg.variant != 8) {
    *reason = "one-link smearing runs the step variants 0, 4, 7 and 8 only";
    return false;
  }
  if (cfg.variant >= 5 && tl::vprec(p->prec) == tl::F64 && eff_width(p, cfg) > 1) {
    *reason = "the LDS-staged step kernels take FP64 groups of one RHS only";
    return false;
  }
  if (cfg.variant == 8 && (p->flags & TL_PLAIN)) {
    *reason = "TL_PLAIN runs one step per launch";
    return false;
  }
  std::vector<StepGroup> gs;
  if (make_groups(p, cfg, &gs) != TL_OK) {
    *reason = "work list too long, or tiling not applicable to these lattices";
    return false;
  }
  const int64_t lds = plan_lds(p, cfg, gs);
  if (lds < 0 || (lds > 0 && !p->ctx->big_lds)) {
    *reason = "tiling needs more LDS than this device allows";
    return false;
  }
  return true;
}

// Build cfg's work list and upload it into tiling t's device table.
int upload_tiling(tl_plan* p, const StepConfig& cfg, tl_plan::Tiling* t) {
  const char* why = nullptr;
  if (!tiling_applies(p, cfg, &why)) return fail(p->ctx, TL_ERR_UNSUPPORTED, "%s", why);
  std::vector<StepGroup> gs;
  (void)make_groups(p, cfg, &gs);
  if (gs.size() > p->group_cap)   // the device table holds one entry per RHS at most
    return fail(p->ctx, TL_ERR_UNSUPPORTED, "work list of %zu groups exceeds the table (%zu)", gs.size(), p->group_cap);
  TL_TRY(upload(p->ctx, t->dev, gs.data(), gs.size() * sizeof(StepGroup)));
  t->cfg = cfg;
  t->cfg.rows64 = std::all_of(gs.begin(), gs.end(), [](const StepGroup& g) { return g.Lx == 64; }) ? 1 : 0;
  t->lds = plan_lds(p, cfg, gs);
  t->host = gs;
  t->n_tiles = gs.empty() ? 0 : gs.back().tile_begin + gs.back().n_xy_tiles * gs.back().n_z_tiles;
  return TL_OK;
}

// The plan's tilings from a tuned pair.
int upload_tuned(tl_plan* p, const Tuned& tu) {
  TL_TRY(upload_tiling(p, tu.cfg, &p->tile));
  if (tu.cfg.variant == 8) TL_TRY(upload_tiling(p, tu.single, &p->single));
  return TL_OK;
}

// One launch of tiling t over every group (batched) or over one group (plain mode, g >= 0),
// from buffer `in` to buffer `out`: one step, or two for variant 8.  k: index of the launch
// in its sequence (odd launches run reversed when the tiling flips).
int plan_launch(tl_plan* p, const tl_plan::Tiling& t, hipStream_t s, const char* in, char* out, int g, int k) {
  tl_ctx* c = p->ctx;
  int base = 0, n = t.n_tiles;
  if (g >= 0) {
    base = t.host[g].tile_begin;
    n = t.host[g].n_xy_tiles * t.host[g].n_z_tiles;
  }
  StepConfig cfg = t.cfg;
  cfg.rev = (cfg.flip && (k & 1)) ? 1 : 0;
  return launch(c, "smearing step", [&] {
    return tl::launch_step(p->prec, eff_width(p, cfg), cfg, t.dev, (int)t.host.size(), base, n, in, out, p->alpha, p->beta,
                           t.lds, s);
  });
}

int plan_step(tl_plan* p, hipStream_t s, int parity, int g, int k) {
  return plan_launch(p, p->tile, s, p->buf[parity], p->buf[parity ^ 1], g, k);
}

// Launches of one run of the n steps (each flips the resident buffer).
int plan_launches(const tl_plan* p) {
  return p->tile.cfg.variant == 8 ? p->n_steps / 2 + (p->n_steps & 1) : p->n_steps;
}

// Queue the n steps starting from buffer `parity` on stream s.
int plan_enqueue(tl_plan* p, hipStream_t s, int parity) {
  if (p->flags & TL_PLAIN) {
    for (int g = 0; g < (int)p->tile.host.size(); g++) {
      int q = parity;
      for (int k = 0; k < p->n_steps; k++) {
        TL_TRY(plan_step(p, s, q, g, k));
        q ^= 1;
      }
    }
  } else if (p->tile.cfg.variant == 8) {
    int q = parity;
    for (int k = 0; k < p->n_steps / 2; k++) {
      TL_TRY(plan_step(p, s, q, -1, k));
      q ^= 1;
    }
    if (p->n_steps & 1) TL_TRY(plan_launch(p, p->single, s, p->buf[q], p->buf[q ^ 1], -1, 0));
  } else {
    int q = parity;
    for (int k = 0; k < p->n_steps; k++) {
      TL_TRY(plan_step(p, s, q, -1, k));
      q ^= 1;
    }
  }
  return TL_OK;
}

std::string tune_key(const tl_plan* p) {
  std::string k = p->ctx->arch + "|p" + std::to_string(p->prec) + "|w" + std::to_string(p->width) +
                  ((p->flags & TL_PLAIN) ? "|plain" : "|batch") + ((p->flags & TL_ONE_STEP) ? "|one" : "");
  for (const auto& g : p->groups) {
    const tl_geom& ge = p->jobs[g.job].job.g;
    k += "|" + std::to_string(ge.L[0]) + "x" + std::to_string(ge.L[1]) + "x" + std::to_string(ge.L[2]) + ":" +
         std::to_string(g.nr);
  }
  return k;
}

// Time every candidate tiling on the plan's own data (buffer cur -> cur^1,
// which leaves the input untouched), require each candidate's output to be
// bit-identical to the first candidate's, keep the fastest.  Then, for batched
// plans of two or more steps, time the two-step tilings against two launches
// of that winner (output bit-identical to them, time per step compared).
int plan_autotune(tl_plan* p) {
  tl_ctx* c = p->ctx;
  const std::string key = tune_key(p);
  auto hit = c->tune.find(key);
  if (hit != c->tune.end()) {
    // a cached tiling that does not apply to this plan (a cache file written by another
    // version of the library, or edited) is dropped and the plan tuned again
    const char* why = nullptr;
    const Tuned& tu = hit->second;
    if (tiling_applies(p, tu.cfg, &why) && (tu.cfg.variant != 8 || tiling_applies(p, tu.single, &why))) {
      c->stats.tune_hits++;
      return upload_tuned(p, tu);
    }
    if (c->log) fprintf(stderr, "[twolink] tune %s: cached tiling %s does not apply (%s), tuning again\n", key.c_str(),
                        cfg_text(tu.cfg).c_str(), why);
    c->tune.erase(hit);
  }
  c->stats.tune_sweeps++;
  std::vector<StepConfig> cands, cands2;
  const int cu = std::max(c->n_cu, 1);
  // the plan's RHS groups, and (batched plans with wider groups) every RHS on its own tiles:
  // more parallel work for small lattices at the price of loading each two-link once per RHS
  std::vector<int> widths{0};
  if (!(p->flags & TL_PLAIN) && p->width > 1) widths.push_back(1);
  for (int wd : widths)
    for (int variant : {0, 2, 3, 4, 5, 6, 7}) {
      const bool lds_variant = variant >= 5;
      const int ew = wd > 0 ? wd : p->width;
      if (tl::is_one(p->prec) && variant != 0 && variant != 4 && variant != 7) continue;   // one-link: hops of one site
      if ((variant == 2 || variant == 3 || lds_variant) && tl::vprec(p->prec) == tl::F64 && ew > 1) continue;   // would run variant 0
      if (lds_variant && !c->big_lds) continue;
      const std::vector<int> tzs = (variant == 0 || variant == 4) ? std::vector<int>{1, 2, 4}
                                   : (variant >= 6 ? std::vector<int>{4, 8, 16} : std::vector<int>{8, 16, 32});
      const std::vector<int> blocks = lds_variant ? std::vector<int>{512, 256} : std::vector<int>{256, 128, 64};
      for (int block : blocks)
        for (int tz : tzs)
          for (int grid : {0, cu, 8 * cu})   // one workgroup per tile, or persistent: 1 or 8 per CU
            for (int nt : {0, 1})
              for (int flip : {0, 1}) {
                StepConfig g{variant, block, tz, grid, nt, flip, 0};
                g.width = wd;
                cands.push_back(g);
              }
    }
  if (!(p->flags & (TL_PLAIN | TL_ONE_STEP)) && p->n_steps >= 2 && c->big_lds &&
      !(tl::vprec(p->prec) == tl::F64 && p->width > 1))
    for (int block : {512, 448, 384, 320, 256})
      for (int tz : {4, 8, 16, 32})
        for (int grid : {0, cu})
          for (int nt : {0, 1})
            for (int flip : {0, 1}) cands2.push_back({8, block, tz, grid, nt, flip, 0});
  void* ref = nullptr;
  void* flag_mem = nullptr;
  TL_TRY(dev_alloc(c, &ref, p->buf_bytes));
  int rc = dev_alloc(c, &flag_mem, 256);
  if (rc != TL_OK) {
    (void)hipFree(ref);
    return rc;
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    rc = fail(c, TL_ERR_HIP, "hipEventCreate failed");
  const int reps = 10;
  // Batched plans time their one launch per step.  Plain plans (one launch per group) time one
  // group of each distinct lattice shape and weigh it by the number of groups of that shape,
  // so that the tiling suits every shape of the batch, not only the first.
  std::vector<std::pair<int, int>> timed{{-1, 1}};   // (group, weight); -1: every group at once
  if (p->flags & TL_PLAIN) {
    timed.clear();
    for (int g = 0; g < (int)p->groups.size(); g++) {
      const tl_geom& ge = p->jobs[p->groups[g].job].job.g;
      bool seen = false;
      for (auto& tw : timed) {
        const tl_geom& gt = p->jobs[p->groups[tw.first].job].job.g;
        if (gt.L[0] == ge.L[0] && gt.L[1] == ge.L[1] && gt.L[2] == ge.L[2] && p->groups[tw.first].nr == p->groups[g].nr) {
          tw.second++;
          seen = true;
          break;
        }
      }
      if (!seen) timed.push_back({g, 1});
    }
  }
  // time reps launches of p->tile (after two untimed) for each timed group, then compare the
  // output with ref (have_ref false: keep it as ref instead); ms: per step
  auto trial = [&](bool have_ref, float* ms, bool* same) -> int {
    *ms = 0.0f;
    for (const auto& tw : timed) {
      for (int w = 0; w < 2; w++) TL_TRY(plan_step(p, c->stream, p->cur, tw.first, w));
      (void)hipEventRecord(e0, c->stream);
      for (int k = 0; k < reps; k++) TL_TRY(plan_step(p, c->stream, p->cur, tw.first, k));
      (void)hipEventRecord(e1, c->stream);
      if (hipEventSynchronize(e1) != hipSuccess) return fail(c, TL_ERR_HIP, "autotune timing failed");
      float t = 0.0f;
      (void)hipEventElapsedTime(&t, e0, e1);
      *ms += t / reps * tw.second;
    }
    *same = true;
    if (!have_ref) {
      if (hipMemcpyAsync(ref, p->buf[p->cur ^ 1], p->buf_bytes, hipMemcpyDeviceToDevice, c->stream) != hipSuccess)
        return fail(c, TL_ERR_HIP, "autotune reference copy failed");
    } else {
      int one = 0;
      (void)hipMemsetAsync(flag_mem, 0, sizeof(int), c->stream);
      (void)tl::launch_compare(static_cast<const char*>(ref), p->buf[p->cur ^ 1], (int64_t)p->buf_bytes,
                               static_cast<int*>(flag_mem), c->stream);
      (void)hipMemcpyAsync(&one, flag_mem, sizeof(int), hipMemcpyDeviceToHost, c->stream);
      (void)hipStreamSynchronize(c->stream);
      *same = one == 0;
    }
    return TL_OK;
  };
  auto log = [&](const StepConfig& g, float ms_step, bool same) {
    if (c->log)
      fprintf(stderr, "[twolink] tune %s variant=%d block=%d tz=%d grid=%d nt=%d flip=%d width=%d: %.4f ms/step%s\n",
              key.c_str(), g.variant, g.block, g.tz, g.grid, g.nt, g.flip, eff_width(p, g), ms_step,
              same ? "" : "  OUTPUT DIFFERS - rejected");
  };
  float best = 1e30f;
  StepConfig best_cfg = cands[0];
  bool have_ref = false;
  for (size_t ci = 0; ci < cands.size() && rc == TL_OK; ci++) {
    const char* why = nullptr;
    if (!tiling_applies(p, cands[ci], &why)) continue;
    rc = upload_tiling(p, cands[ci], &p->tile);
    if (rc != TL_OK) break;
    float ms = 0.0f;
    bool same = true;
    rc = trial(have_ref, &ms, &same);
    if (rc != TL_OK) break;
    have_ref = true;
    log(p->tile.cfg, ms, same);
    if (same && ms < best) {
      best = ms;
      best_cfg = p->tile.cfg;
    }
  }
  Tuned tu;
  tu.cfg = best_cfg;
  if (rc == TL_OK && !cands2.empty()) {
    // reference: two launches of the one-step winner, buffer cur -> cur^1 -> ref
    rc = upload_tiling(p, best_cfg, &p->single);
    if (rc == TL_OK) rc = plan_launch(p, p->single, c->stream, p->buf[p->cur], p->buf[p->cur ^ 1], -1, 0);
    if (rc == TL_OK) rc = plan_launch(p, p->single, c->stream, p->buf[p->cur ^ 1], static_cast<char*>(ref), -1, 1);
    float best2 = 1e30f;
    StepConfig best2_cfg{};
    for (size_t ci = 0; ci < cands2.size() && rc == TL_OK; ci++) {
      const char* why = nullptr;
      if (!tiling_applies(p, cands2[ci], &why)) continue;
      rc = upload_tiling(p, cands2[ci], &p->tile);
      if (rc != TL_OK) break;
      float ms = 0.0f;
      bool same = true;
      rc = trial(true, &ms, &same);
      if (rc != TL_OK) break;
      log(p->tile.cfg, ms / 2, same);
      if (same && ms / 2 < best2) {
        best2 = ms / 2;
        best2_cfg = p->tile.cfg;
      }
    }
    if (rc == TL_OK && best2 < best) {
      tu.cfg = best2_cfg;
      tu.single = best_cfg;
    }
  }
  (void)hipStreamSynchronize(c->stream);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipFree(ref);
  (void)hipFree(flag_mem);
  if (rc != TL_OK) return rc;
  c->tune[key] = tu;
  if (!c->tune_file.empty()) tune_file_save(c);
  return upload_tuned(p, tu);
}

// TL_TILE="variant,block,tz,grid[,nt[,flip]]" fixes the step tiling of every plan (no tuning):
// used to profile or sweep one tiling at a time.  A two-step tiling (variant 8) may name its
// one-step companion after a ";" (default: variant 0, 256 threads, tz 4).
bool tile_override(Tuned* tu) {
  const char* e = getenv("TL_TILE");
  return e && parse_tuned(e, 4, tu);
}

int plan_prepare(tl_plan* p) {
  if (p->ready) return TL_OK;
  Tuned forced;
  if (tile_override(&forced)) {
    TL_TRY(upload_tuned(p, forced));
  } else if ((p->flags & TL_AUTOTUNE) && p->n_steps > 0) {
    TL_TRY(plan_autotune(p));
  }
  p->ready = true;
  return TL_OK;
}

int plan_capture(tl_plan* p, int parity) {
  tl_ctx* c = p->ctx;
  if (p->graph[parity]) return TL_OK;
  hipStream_t cs = nullptr;
  HIP_TRY(c, hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
  hipGraph_t graph = nullptr;
  int rc = TL_OK;
  if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    rc = fail(c, TL_ERR_HIP, "hipStreamBeginCapture failed");
  } else {
    rc = plan_enqueue(p, cs, parity);
    hipError_t e = hipStreamEndCapture(cs, &graph);
    if (rc == TL_OK && e != hipSuccess) rc = fail(c, TL_ERR_HIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
  }
  if (rc == TL_OK) {
    hipError_t e = hipGraphInstantiate(&p->graph[parity], graph, nullptr, nullptr, 0);
    if (e != hipSuccess) rc = fail(c, TL_ERR_HIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
    else c->stats.graphs_captured++;
  }
  if (graph) (void)hipGraphDestroy(graph);
  (void)hipStreamDestroy(cs);
  return rc;
}

void plan_free(tl_plan* p) {
  if (!p) return;
  if (p->ctx && p->ctx->device >= 0) {
    DeviceGuard dg(p->ctx->device);
    (void)hipStreamSynchronize(p->ctx->stream);
    for (auto& g : p->graph)
      if (g) (void)hipGraphExecDestroy(g);
    for (auto& b : p->buf)
      if (b) (void)hipFree(b);
    if (p->tables) (void)hipFree(p->tables);
  }
  delete p;
}

}  // namespace

// ====================================================================== C ABI

extern "C" {

int tl_version(void) { return 10100; }

int tl_create(tl_ctx** out, int device, void* stream) {
  tl_ctx* c = nullptr;
  try {
    if (!out) return fail(nullptr, TL_ERR_ARG, "out is NULL");
    *out = nullptr;
    c = new (std::nothrow) tl_ctx();
    if (!c) return fail(nullptr, TL_ERR_NOMEM, "host allocation failed");
    const char* lg = getenv("TL_LOG");
    c->log = lg && lg[0] == '1';
    const char* tf = getenv("TL_TUNE_CACHE");
    if (tf && tf[0]) {
      c->tune_file = tf;
      tune_file_load(c);
    }
    const char* fl = getenv("TL_FAULT");
    if (fl) {
      c->fault_alloc = strcmp(fl, "alloc") == 0;
      c->fault_launch = strcmp(fl, "launch") == 0;
    }
    if (device == -1) {
      c->device = -1;
      *out = c;
      return TL_OK;
    }
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess || device < 0 || device >= n) {
      delete c;
      c = nullptr;
      return fail(nullptr, TL_ERR_DEVICE, "device %d not available (%d devices%s%s)", device, e == hipSuccess ? n : 0,
                  e == hipSuccess ? "" : ": ", e == hipSuccess ? "" : hipGetErrorString(e));
    }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) {
      delete c;
      c = nullptr;
      return fail(nullptr, TL_ERR_DEVICE, "hipGetDeviceProperties(%d) failed", device);
    }
    {
      // the LDS-staged step kernels need more than the default dynamic-LDS limit;
      // without it their tilings are simply not offered
      DeviceGuard dg(device);
      if (!dg.ok) {
        delete c;
        c = nullptr;
        return fail(nullptr, TL_ERR_DEVICE, "hipSetDevice(%d) failed", device);
      }
      c->big_lds = tl::init_kernel_attributes() == hipSuccess;
      (void)hipGetLastError();
      // the fixed device area of tl_reduce_noalloc: its address on this device, looked up
      // once per device; a failure here only disables that entry point
      const hipError_t ne = tl::noalloc_scratch_init(device);
      c->noalloc = tl::noalloc_scratch(device);
      if (ne != hipSuccess || !c->noalloc) {
        c->noalloc = nullptr;
        c->noalloc_err = std::string("hipGetSymbolAddress: ") + hipGetErrorString(ne);
        (void)hipGetLastError();
      }
    }
    c->device = device;
    c->stream = static_cast<hipStream_t>(stream);
    c->n_cu = prop.multiProcessorCount;
    c->arch = prop.gcnArchName;
    *out = c;
    return TL_OK;
  } catch (...) {   // a half-built context is released; *out stays NULL
    if (out) *out = nullptr;
    delete c;
    return host_failure(nullptr);
  }
}

int tl_destroy(tl_ctx* c) {
  try {
    if (!c) return TL_ERR_ARG;
    for (auto& sp : c->smear_plans) plan_free(sp.second);
    c->smear_plans.clear();
    if (c->device >= 0) {
      DeviceGuard dg(c->device);   // teardown goes on even if the switch fails
      (void)hipStreamSynchronize(c->stream);
      if (c->scratch) (void)hipFree(c->scratch);
    }
    delete c;
    return TL_OK;
  } catch (...) {
    return host_failure(nullptr);
  }
}

int tl_set_stream(tl_ctx* c, void* stream) {
  try {
    if (!c) return TL_ERR_ARG;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (c->device >= 0 && s != c->stream) {
      // Context scratch and plan buffers are reused in stream order.  Work already queued on
      // the old stream may still read them, so the new stream waits for it (an event, no host
      // wait) before anything queued through this context runs there.
      TL_ON_DEVICE(c);
      hipEvent_t ev = nullptr;
      HIP_TRY(c, hipEventCreateWithFlags(&ev, hipEventDisableTiming));
      hipError_t e = hipEventRecord(ev, c->stream);
      if (e == hipSuccess) e = hipStreamWaitEvent(s, ev, 0);
      (void)hipEventDestroy(ev);
      if (e != hipSuccess) return fail(c, TL_ERR_HIP, "ordering the new stream after the old: %s", hipGetErrorString(e));
    }
    c->stream = s;
    return TL_OK;
  } catch (...) {
    return host_failure(c);
  }
}

int tl_sync(tl_ctx* c) {
  try {
    if (!c) return TL_ERR_ARG;
    TL_TRY(need_device(c));
    TL_ON_DEVICE(c);
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    HIP_TRY(c, hipGetLastError());
    return TL_OK;
  } catch (...) {
    return host_failure(c);
  }
}

const char* tl_last_error(const tl_ctx* c) { return c ? c->err.c_str() : g_create_err.c_str(); }

int tl_check_geom(const tl_geom* g) {
  try {
    tl_ctx tmp;
    return check_geom(&tmp, g);
  } catch (...) {
    return host_failure(nullptr);
  }
}

size_t tl_twolinks_bytes(const tl_geom* g, int prec, int n_slices) {
  if (tl_check_geom(g) != TL_OK || !valid_prec(prec) || n_slices < 0 || n_slices > g->L[3]) return 0;
  return (size_t)n_slices * 3 * (size_t)tl::padded_sites(vol3(*g)) * tl::kWBytes[fmt_code(prec)];
}

namespace {

// Shared by tl_build_twolinks (two-links, no TL_ONELINK bit) and tl_pack_links (one-links,
// TL_ONELINK bit required).
int build_links(tl_ctx* c, const tl_geom* g, const void* U, const int32_t* slices, int n_slices, int prec,
                void* W, bool one) {
  if (!c) return TL_ERR_ARG;
  TL_TRY(check_geom(c, g));
  if (!valid_prec(prec)) return fail(c, TL_ERR_PRECISION, "unknown precision %d", prec);
  if (tl::is_one(fmt_code(prec)) != one)
    return fail(c, TL_ERR_PRECISION, one ? "tl_pack_links needs TL_ONELINK in prec"
                                         : "TL_ONELINK fields are built by tl_pack_links");
  if (!U || !W) return fail(c, TL_ERR_ARG, "U and W must be non-NULL device pointers");
  if (!slices) {
    if (n_slices != 0 && n_slices != g->L[3])
      return fail(c, TL_ERR_ARG, "slices is NULL but n_slices = %d (expected 0 or Lt = %d)", n_slices, g->L[3]);
    n_slices = g->L[3];
  } else {
    if (n_slices < 1 || n_slices > g->L[3])
      return fail(c, TL_ERR_ARG, "n_slices = %d outside [1, Lt=%d]", n_slices, g->L[3]);
    std::vector<char> seen(g->L[3], 0);
    for (int j = 0; j < n_slices; j++) {
      if (slices[j] < 0 || slices[j] >= g->L[3])
        return fail(c, TL_ERR_SHAPE, "slices[%d] = %d outside [0, %d)", j, slices[j], g->L[3]);
      if (seen[slices[j]]++) return fail(c, TL_ERR_ARG, "slice %d listed twice", slices[j]);
    }
  }
  TL_TRY(need_device(c));
  TL_ON_DEVICE(c);
  const int code = fmt_code(prec);
  if (!slices) return launch(c, "two-link build", [&] { return tl::launch_build(code, U, g->L, 0, 0, n_slices, W, c->stream); });
  // runs of consecutive slices share a launch
  int j = 0;
  while (j < n_slices) {
    int k = j + 1;
    while (k < n_slices && slices[k] == slices[k - 1] + 1) k++;
    TL_TRY(launch(c, "two-link build", [&] { return tl::launch_build(code, U, g->L, slices[j], j, k - j, W, c->stream); }));
    j = k;
  }
  return TL_OK;
}

}  // namespace

int tl_build_twolinks(tl_ctx* c, const tl_geom* g, const void* U, const int32_t* slices, int n_slices, int prec,
                      void* W) {
  try {
    return build_links(c, g, U, slices, n_slices, prec, W, false);
  } catch (...) {
    return host_failure(c);
  }
}

int tl_pack_links(tl_ctx* c, const tl_geom* g, const void* U, const int32_t* slices, int n_slices, int prec,
                  void* W) {
  try {
    return build_links(c, g, U, slices, n_slices, prec, W, true);
  } catch (...) {
    return host_failure(c);
  }
}

int tl_laplacian(tl_ctx* c, const tl_geom* g, const void* W, const int32_t* w_slices, int n_w_slices, int prec,
                 int t, const void* in, void* out) {
  try {
    if (!c) return TL_ERR_ARG;
    TL_TRY(check_geom(c, g));
    if (!valid_prec(prec)) return fail(c, TL_ERR_PRECISION, "unknown precision %d", prec);
    if (!W || !in || !out) return fail(c, TL_ERR_ARG, "W, in and out must be non-NULL device pointers");
    TL_TRY(check_wslices(c, *g, w_slices, n_w_slices));
    const int slot = slot_of(*g, w_slices, n_w_slices, t);
    if (slot < 0) return fail(c, TL_ERR_SHAPE, "slice t = %d is not in the two-link field", t);
    const int64_t V3 = vol3(*g), Vp = tl::padded_sites(V3);
    const size_t nat_bytes = (size_t)V3 * 48;
    const char* a = static_cast<const char*>(in);
    const char* b = static_cast<const char*>(out);
    if (a < b + nat_bytes && b < a + nat_bytes) return fail(c, TL_ERR_ARG, "in and out overlap");
    TL_TRY(need_device(c));
    TL_ON_DEVICE(c);
    const int code = fmt_code(prec), vp = tl::vprec(code);
    const size_t fb = align256((size_t)Vp * tl::kVBytes[vp]);
    char* s = nullptr;
    TL_TRY(ctx_scratch(c, 1024 + 2 * fb, &s));
    StepGroup sg{};
    StepConfig cfg{0, 256, 4, 0, 0};
    sg.W = static_cast<const char*>(W) + (int64_t)slot * 3 * Vp * tl::kWBytes[code];
    sg.w_mu_stride = Vp * tl::kWBytes[code];
    sg.psi_off = 0;
    sg.rhs_stride = 0;
    sg.Lx = g->L[0];
    sg.Ly = g->L[1];
    sg.Lz = g->L[2];
    sg.Vp = (int32_t)Vp;
    sg.nr = 1;
    sg.n_xy_tiles = (int32_t)(((int64_t)g->L[0] * g->L[1] + cfg.block - 1) / cfg.block);
    sg.n_z_tiles = (g->L[2] + cfg.tz - 1) / cfg.tz;
    sg.tile_begin = 0;
    struct {
      StepGroup g;
      int64_t off0;
    } tab{sg, 0};
    TL_TRY(upload(c, s, &tab, sizeof tab));
    const StepGroup* gdev = reinterpret_cast<const StepGroup*>(s);
    const int64_t* offdev = reinterpret_cast<const int64_t*>(s + offsetof(decltype(tab), off0));
    char* A = s + 1024;
    char* B = A + fb;
    TL_TRY(launch(c, "pack", [&] { return tl::launch_pack(vp, in, A, offdev, 1, V3, Vp, c->stream); }));
    // Lap = alpha in + beta sum_hops: two-link -3/2, 1/4 (eq. tlLapl1); one-link -6, 1 (H - 6)
    const double la = tl::is_one(code) ? -6.0 : -1.5, lb = tl::is_one(code) ? 1.0 : 0.25;
    TL_TRY(launch(c, "laplacian", [&] { return tl::launch_step(code, 1, cfg, gdev, 1, 0, sg.n_xy_tiles * sg.n_z_tiles, A, B, la, lb,
                                        0, c->stream); }));
    return launch(c, "unpack", [&] { return tl::launch_unpack(vp, B, out, offdev, 1, V3, Vp, c->stream); });
  } catch (...) {
    return host_failure(c);
  }
}

int tl_plan_create(tl_ctx* c, const tl_job* jobs, int n_jobs, int n_steps, double sigma, int prec, unsigned flags,
                   tl_plan** out) {
  try {
    if (!c) return TL_ERR_ARG;
    if (!out) return fail(c, TL_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (!jobs || n_jobs < 1) return fail(c, TL_ERR_ARG, "need at least one job");
    if (!valid_prec(prec)) return fail(c, TL_ERR_PRECISION, "unknown precision %d", prec);
    if (flags & ~(unsigned)(TL_PLAIN | TL_GRAPH | TL_AUTOTUNE | TL_ONE_STEP))
      return fail(c, TL_ERR_ARG, "unknown flag bits 0x%x", flags);
    if ((flags & TL_PLAIN) && (flags & TL_GRAPH)) return fail(c, TL_ERR_ARG, "TL_PLAIN runs eager launches; it excludes TL_GRAPH");
    if (n_steps < 0) return fail(c, TL_ERR_ARG, "n_steps = %d is negative", n_steps);
    if (!std::isfinite(sigma)) return fail(c, TL_ERR_ARG, "sigma is not finite");
    const bool one = tl::is_one(fmt_code(prec));
    if (n_steps > 0) {
      const double s = sigma / n_steps;
      if (s < 0.0 || s > max_step(one))
        return fail(c, TL_ERR_ARG, "sigma/n = %g outside [0, %s]", s, one ? "1/6" : "2/3");
    }
    for (int j = 0; j < n_jobs; j++) {
      const tl_job& jb = jobs[j];
      TL_TRY(check_geom(c, &jb.g));
      if (!jb.W || !jb.psi) return fail(c, TL_ERR_ARG, "job %d: W and psi must be non-NULL", j);
      if (jb.n_rhs < 1 || !jb.t_of_rhs) return fail(c, TL_ERR_ARG, "job %d: needs n_rhs >= 1 and t_of_rhs", j);
      TL_TRY(check_wslices(c, jb.g, jb.w_slices, jb.n_w_slices));
      for (int r = 0; r < jb.n_rhs; r++)
        if (slot_of(jb.g, jb.w_slices, jb.n_w_slices, jb.t_of_rhs[r]) < 0)
          return fail(c, TL_ERR_SHAPE, "job %d RHS %d: slice %d not in the two-link field", j, r, jb.t_of_rhs[r]);
    }
    TL_TRY(need_device(c));
    TL_ON_DEVICE(c);
  
    tl_plan* p = new (std::nothrow) tl_plan();
    if (!p) return fail(c, TL_ERR_NOMEM, "host allocation failed");
    struct Release {   // frees the plan on every exit but the successful one
      tl_plan* p;
      ~Release() { plan_free(p); }
    } release{p};
    p->ctx = c;
    p->prec = fmt_code(prec);
    p->n_steps = n_steps;
    p->sigma = sigma;
    p->flags = flags;
    if (n_steps > 0) step_coeffs(one, n_steps, sigma, &p->alpha, &p->beta);
    const int max_width = (flags & TL_PLAIN) ? 1 : 4;
  
    // resident order: per job, per slot (in slice order), RHS in job order;
    // groups of up to max_width RHS, balanced within a slot.
    size_t off = 0;
    for (int j = 0; j < n_jobs; j++) {
      tl_plan::JobCopy jc;
      jc.job = jobs[j];
      jc.t_of_rhs.assign(jobs[j].t_of_rhs, jobs[j].t_of_rhs + jobs[j].n_rhs);
      if (jobs[j].w_slices) jc.w_slices.assign(jobs[j].w_slices, jobs[j].w_slices + jobs[j].n_w_slices);
      jc.job.t_of_rhs = jc.t_of_rhs.data();
      jc.job.w_slices = jobs[j].w_slices ? jc.w_slices.data() : nullptr;
      jc.V3 = vol3(jc.job.g);
      jc.Vp = tl::padded_sites(jc.V3);
      jc.res_index.assign(jc.job.n_rhs, -1);
      p->max_v3 = std::max(p->max_v3, jc.V3);
      std::map<int, std::vector<int>> by_slot;
      for (int r = 0; r < jc.job.n_rhs; r++)
        by_slot[slot_of(jc.job.g, jc.job.w_slices, jc.job.n_w_slices, jc.t_of_rhs[r])].push_back(r);
      const size_t rb = align256((size_t)jc.Vp * tl::kVBytes[p->prec]);
      for (auto& kv : by_slot) {
        const int k = (int)kv.second.size();
        const int ng = (k + max_width - 1) / max_width;
        int done = 0;
        for (int q = 0; q < ng; q++) {
          const int nr = (k - done + (ng - q) - 1) / (ng - q);
          tl_plan::Group gr{j, kv.first, (int)p->res.size(), nr};
          for (int i = 0; i < nr; i++) {
            const int r = kv.second[done + i];
            jc.res_index[r] = (int)p->res.size();
            p->res.push_back({j, r, kv.first, (int64_t)off});
            off += rb;
          }
          done += nr;
          p->width = std::max(p->width, nr);
          p->groups.push_back(gr);
        }
      }
      p->jobs.push_back(std::move(jc));
    }
    p->buf_bytes = std::max<size_t>(off, 256);
  
    // device memory: two resident buffers and the tables
    int rc = TL_OK;
    for (int k = 0; k < 2 && rc == TL_OK; k++) {
      void* b = nullptr;
      rc = dev_alloc(c, &b, p->buf_bytes);
      p->buf[k] = static_cast<char*>(b);
    }
    const size_t n_res = p->res.size();
    // two tilings' step groups: a tiling may split the plan's groups down to one RHS each
    p->group_cap = n_res;
    const size_t gbytes = 2 * align256(n_res * sizeof(StepGroup));
    const size_t obytes = align256(n_res * sizeof(int64_t));
    const size_t rbytes = align256(n_res * sizeof(tl::RedField));
    const size_t pbytes = align256((size_t)tl::red_partials_doubles((int)n_res, p->max_v3) * sizeof(double));
    if (rc == TL_OK) {
      void* t = nullptr;
      rc = dev_alloc(c, &t, gbytes + obytes + rbytes + pbytes);
      p->tables = static_cast<char*>(t);
    }
    if (rc == TL_OK) {
      p->tile.dev = reinterpret_cast<StepGroup*>(p->tables);
      p->single.dev = reinterpret_cast<StepGroup*>(p->tables + gbytes / 2);
      p->packoff_dev = reinterpret_cast<int64_t*>(p->tables + gbytes);
      p->red_dev = reinterpret_cast<tl::RedField*>(p->tables + gbytes + obytes);
      p->partials = reinterpret_cast<double*>(p->tables + gbytes + obytes + rbytes);
      std::vector<int64_t> po;
      std::vector<tl::RedField> rf;
      for (auto& jc : p->jobs) {
        p->packoff_first.push_back((int64_t)po.size());
        for (int r = 0; r < jc.job.n_rhs; r++) po.push_back(p->res[jc.res_index[r]].off);
      }
      for (auto& jc : p->jobs)
        for (int r = 0; r < jc.job.n_rhs; r++) {
          const int64_t o = p->res[jc.res_index[r]].off;
          rf.push_back({o, o, jc.V3, jc.Vp, 0});
        }
      int64_t oo = 0;
      for (auto& f : rf) {
        f.out_off = oo;
        oo += f.V3;
      }
      rc = upload(c, p->packoff_dev, po.data(), po.size() * sizeof(int64_t));
      if (rc == TL_OK) rc = upload(c, p->red_dev, rf.data(), rf.size() * sizeof(tl::RedField));
    }
    if (rc == TL_OK) {
      // zero the resident buffers so tuning runs never see stale bit patterns
      for (int k = 0; k < 2 && rc == TL_OK; k++)
        if (hipMemsetAsync(p->buf[k], 0, p->buf_bytes, c->stream) != hipSuccess)
          rc = fail(c, TL_ERR_HIP, "hipMemsetAsync failed");
    }
    if (rc == TL_OK) rc = upload_tiling(p, p->tile.cfg, &p->tile);
    if (rc != TL_OK) return rc;
    // info
    tl_plan_info& in = p->info;
    in.n_groups = (int32_t)p->groups.size();
    in.group_width = p->width;
    in.launches_per_step = (flags & TL_PLAIN) ? in.n_groups : 1;
    double bytes = 0.0, flops = 0.0;
    int64_t rs = 0;
    for (auto& gr : p->groups) {
      const double v3 = (double)p->jobs[gr.job].V3;
      bytes += v3 * (3.0 * tl::kWBytes[p->prec] + 2.0 * gr.nr * tl::kVBytes[p->prec]);
      flops += v3 * (444.0 * gr.nr + (tl::is_w12(p->prec) ? 3 * 42.0 : 0.0));
      rs += (int64_t)p->jobs[gr.job].V3 * gr.nr;
    }
    in.rhs_sites = rs;
    in.bytes_per_step = bytes;
    in.flops_per_step = flops;
    in.resident_bytes = (int64_t)(2 * p->buf_bytes + gbytes + obytes + rbytes + pbytes);
    release.p = nullptr;
    *out = p;
    return TL_OK;
  } catch (...) {
    return host_failure(c);
  }
}

int tl_plan_load(tl_plan* p) {
  try {
    if (!p) return TL_ERR_ARG;
    tl_ctx* c = p->ctx;
    TL_ON_DEVICE(c);
    for (size_t j = 0; j < p->jobs.size(); j++) {
      const auto& jc = p->jobs[j];
      TL_TRY(launch(c, "pack", [&] { return tl::launch_pack(tl::vprec(p->prec), jc.job.psi, p->buf[p->cur], p->packoff_dev + p->packoff_first[j],
                                          jc.job.n_rhs, jc.V3, jc.Vp, c->stream); }));
    }
    return TL_OK;
  } catch (...) {
    return host_failure(p ? p->ctx : nullptr);
  }
}

int tl_plan_run(tl_plan* p) {
  try {
    if (!p) return TL_ERR_ARG;
    tl_ctx* c = p->ctx;
    if (p->n_steps == 0) return TL_OK;
    TL_ON_DEVICE(c);
    TL_TRY(plan_prepare(p));
    if (p->flags & TL_GRAPH) {
      TL_TRY(plan_capture(p, p->cur));
      if (c->fault_launch) return fail(c, TL_ERR_HIP, "graph launch failed (TL_FAULT=launch)");
      HIP_TRY(c, hipGraphLaunch(p->graph[p->cur], c->stream));
    } else {
      TL_TRY(plan_enqueue(p, c->stream, p->cur));
    }
    p->cur ^= (plan_launches(p) & 1);
    return TL_OK;
  } catch (...) {
    return host_failure(p ? p->ctx : nullptr);
  }
}

int tl_plan_store(tl_plan* p) {
  try {
    if (!p) return TL_ERR_ARG;
    tl_ctx* c = p->ctx;
    TL_ON_DEVICE(c);
    for (size_t j = 0; j < p->jobs.size(); j++) {
      const auto& jc = p->jobs[j];
      TL_TRY(launch(c, "unpack", [&] { return tl::launch_unpack(tl::vprec(p->prec), p->buf[p->cur], jc.job.psi, p->packoff_dev + p->packoff_first[j],
                                            jc.job.n_rhs, jc.V3, jc.Vp, c->stream); }));
    }
    return TL_OK;
  } catch (...) {
    return host_failure(p ? p->ctx : nullptr);
  }
}

int tl_plan_reduce(tl_plan* p, int kind, const tl_plan* other, double* out) {
  try {
    if (!p) return TL_ERR_ARG;
    tl_ctx* c = p->ctx;
    if (kind < TL_NORM2 || kind > TL_SITE_NORM) return fail(c, TL_ERR_ARG, "unknown reduction kind %d", kind);
    if (!out) return fail(c, TL_ERR_ARG, "out is NULL");
    const char* b = nullptr;
    if (kind == TL_DOT) {
      if (!other) return fail(c, TL_ERR_ARG, "TL_DOT needs a second plan");
      if (other->ctx != c || tl::vprec(other->prec) != tl::vprec(p->prec) || other->buf_bytes != p->buf_bytes || other->res.size() != p->res.size())
        return fail(c, TL_ERR_ARG, "TL_DOT: plans differ in context, precision or shape");
      for (size_t i = 0; i < p->res.size(); i++)
        if (other->res[i].off != p->res[i].off) return fail(c, TL_ERR_ARG, "TL_DOT: plans differ in layout");
      b = other->buf[other->cur];
    }
    TL_ON_DEVICE(c);
    // a (this) is the second argument of <other, this>
    return launch(c, "reduction", [&] { return tl::launch_reduce(kind, tl::vprec(p->prec), p->buf[p->cur], b, p->red_dev, (int)p->res.size(), p->max_v3,
                                          p->partials, out, c->stream); });
  } catch (...) {
    return host_failure(p ? p->ctx : nullptr);
  }
}

int tl_plan_time(tl_plan* p, int reps, double* ms_per_step) {
  try {
    if (!p) return TL_ERR_ARG;
    tl_ctx* c = p->ctx;
    if (reps < 1 || !ms_per_step) return fail(c, TL_ERR_ARG, "need reps >= 1 and an output pointer");
    if (p->n_steps == 0) return fail(c, TL_ERR_ARG, "plan has no steps");
    TL_ON_DEVICE(c);
    TL_TRY(tl_plan_run(p));   // tuning and graph capture happen outside the timed region
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = TL_OK;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
      if (e0) (void)hipEventDestroy(e0);
      return fail(c, TL_ERR_HIP, "hipEventCreate failed");
    }
    (void)hipEventRecord(e0, c->stream);
    for (int k = 0; k < reps && rc == TL_OK; k++) rc = tl_plan_run(p);
    (void)hipEventRecord(e1, c->stream);
    float ms = 0.0f;
    if (rc == TL_OK) {
      if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
        rc = fail(c, TL_ERR_HIP, "event timing failed");
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc == TL_OK) *ms_per_step = ms / ((double)reps * p->n_steps * p->info.launches_per_step);
    return rc;
  } catch (...) {
    return host_failure(p ? p->ctx : nullptr);
  }
}

int tl_stream_time(tl_ctx* c, void* buf, int64_t bytes, int n_in, int kinds, int grid, int reps, double* ms) {
  try {
    if (!c) return TL_ERR_ARG;
    if (!buf || !ms || reps < 1) return fail(c, TL_ERR_ARG, "need a buffer, an output pointer and reps >= 1");
    if (n_in < 1 || n_in > 16) return fail(c, TL_ERR_ARG, "n_in = %d outside [1, 16]", n_in);
    if (kinds < 0 || kinds > 3 || grid < 0) return fail(c, TL_ERR_ARG, "bad kinds %d or grid %d", kinds, grid);
    if (reinterpret_cast<uintptr_t>(buf) % 256) return fail(c, TL_ERR_ARG, "buffer not 256-byte aligned");
    const int64_t n_words = bytes / 16 / (n_in + 1);
    if (n_words < 1) return fail(c, TL_ERR_ARG, "buffer of %lld bytes too small", (long long)bytes);
    TL_TRY(need_device(c));
    TL_ON_DEVICE(c);
    const int g = grid > 0 ? grid : 16 * std::max(c->n_cu, 1);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
      if (e0) (void)hipEventDestroy(e0);
      return fail(c, TL_ERR_HIP, "hipEventCreate failed");
    }
    int rc = launch(c, "stream", [&] { return tl::launch_stream(buf, n_words, n_in, kinds, g, c->stream); });
    if (rc == TL_OK) (void)hipEventRecord(e0, c->stream);
    for (int k = 0; k < reps && rc == TL_OK; k++)
      rc = launch(c, "stream", [&] { return tl::launch_stream(buf, n_words, n_in, kinds, g, c->stream); });
    float t = 0.0f;
    if (rc == TL_OK) {
      (void)hipEventRecord(e1, c->stream);
      if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&t, e0, e1) != hipSuccess)
        rc = fail(c, TL_ERR_HIP, "event timing failed");
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc == TL_OK) *ms = t / reps;
    return rc;
  } catch (...) {
    return host_failure(c);
  }
}

int tl_plan_get_info(const tl_plan* p, tl_plan_info* info) {
  try {
    if (!p || !info) return TL_ERR_ARG;
    *info = p->info;
    const tl_plan::Tiling& t = p->tile;
    info->n_tiles = t.n_tiles;
    info->variant = t.cfg.variant;
    info->block = t.cfg.block;
    info->tz = t.cfg.tz;
    info->grid = t.cfg.grid > 0 ? std::min(t.cfg.grid, t.n_tiles) : t.n_tiles;
    info->nt = t.cfg.nt;
    info->flip = t.cfg.flip;
    info->steps_per_launch = t.cfg.variant == 8 ? 2 : 1;
    info->tile_width = eff_width(p, t.cfg);
    return TL_OK;
  } catch (...) {
    return host_failure(p ? p->ctx : nullptr);
  }
}

int tl_plan_destroy(tl_plan* p) {
  try {
    if (!p) return TL_ERR_ARG;
    plan_free(p);
    return TL_OK;
  } catch (...) {
    return host_failure(nullptr);
  }
}

}  // extern "C"

namespace {

constexpr size_t kSmearPlans = 4;   // tl_smear(TL_GRAPH) plans a context keeps

// Everything a tl_smear plan depends on: the job list (geometries, device pointers, slice lists,
// RHS slices), n, sigma (its bits), the precision code and the flags.
std::string smear_signature(const tl_job* jobs, int n_jobs, int n_steps, double sigma, int prec, unsigned flags) {
  std::string k;
  char buf[128];
  uint64_t sb;
  std::memcpy(&sb, &sigma, sizeof sb);
  snprintf(buf, sizeof buf, "n%d|s%llx|p%d|f%u|j%d", n_steps, (unsigned long long)sb, prec, flags, n_jobs);
  k += buf;
  for (int j = 0; j < n_jobs; j++) {
    const tl_job& b = jobs[j];
    snprintf(buf, sizeof buf, "|%d,%d,%d,%d:%p:%p:%d:", b.g.L[0], b.g.L[1], b.g.L[2], b.g.L[3], b.W, b.psi, b.n_rhs);
    k += buf;
    for (int r = 0; r < b.n_rhs; r++) k += std::to_string(b.t_of_rhs[r]) + ",";
    if (b.w_slices) {
      k += "w";
      for (int i = 0; i < b.n_w_slices; i++) k += std::to_string(b.w_slices[i]) + ",";
    }
  }
  return k;
}

}  // namespace

extern "C" {

int tl_smear(tl_ctx* c, const tl_job* jobs, int n_jobs, int n_steps, double sigma, int prec, unsigned flags) {
  try {
    if (!c) return TL_ERR_ARG;
    // the signature reads the jobs' host arrays: malformed jobs are not kept (tl_plan_create refuses them)
    bool keep = (flags & TL_GRAPH) && jobs && n_jobs >= 1;
    for (int j = 0; keep && j < n_jobs; j++)
      if (jobs[j].n_rhs < 1 || !jobs[j].t_of_rhs || (jobs[j].w_slices && jobs[j].n_w_slices < 1)) keep = false;
    std::string sig;
    if (keep) {
      sig = smear_signature(jobs, n_jobs, n_steps, sigma, prec, flags);
      for (auto it = c->smear_plans.begin(); it != c->smear_plans.end(); ++it) {
        if (it->first != sig) continue;
        c->smear_plans.splice(c->smear_plans.begin(), c->smear_plans, it);   // most recent first
        tl_plan* p = c->smear_plans.front().second;
        c->stats.smear_plan_hits++;
        p->cur = 0;   // the sources are packed afresh, into the buffer whose graph was captured first
        int rc = tl_plan_load(p);
        if (rc == TL_OK) rc = tl_plan_run(p);
        if (rc == TL_OK) rc = tl_plan_store(p);
        return rc;
      }
    }
    tl_plan* p = nullptr;
    TL_TRY(tl_plan_create(c, jobs, n_jobs, n_steps, sigma, prec, flags, &p));
    int rc = tl_plan_load(p);
    if (rc == TL_OK) rc = tl_plan_run(p);
    if (rc == TL_OK) rc = tl_plan_store(p);
    if (!keep || rc != TL_OK) {
      plan_free(p);   // waits for the queued work before releasing the resident buffers
      return rc;
    }
    c->smear_plans.emplace_front(std::move(sig), p);
    if (c->smear_plans.size() > kSmearPlans) {
      plan_free(c->smear_plans.back().second);
      c->smear_plans.pop_back();
    }
    return rc;
  } catch (...) {
    return host_failure(c);
  }
}

int tl_get_stats(const tl_ctx* c, tl_ctx_stats* out) {
  if (!c || !out) return TL_ERR_ARG;
  *out = c->stats;
  return TL_OK;
}

namespace {

int check_reduce_args(tl_ctx* c, int kind, int64_t n_sites, int n_rhs, const void* psi, const void* phi,
                      const double* out) {
  if (kind < TL_NORM2 || kind > TL_SITE_NORM) return fail(c, TL_ERR_ARG, "unknown reduction kind %d", kind);
  if (n_sites < 1 || n_rhs < 1) return fail(c, TL_ERR_ARG, "need n_sites >= 1 and n_rhs >= 1");
  if (!psi || !out || (kind == TL_DOT && !phi)) return fail(c, TL_ERR_ARG, "NULL field or output");
  if (n_sites > (int64_t(1) << 40)) return fail(c, TL_ERR_SHAPE, "n_sites too large");
  return TL_OK;
}

}  // namespace

int tl_reduce_noalloc(tl_ctx* c, int kind, int64_t n_sites, int n_rhs, const void* psi, const void* phi,
                      double* out) {
  try {
    if (!c) return TL_ERR_ARG;
    TL_TRY(check_reduce_args(c, kind, n_sites, n_rhs, psi, phi, out));
    if (kind != TL_SITE_NORM) {
      const int64_t need = tl::red_partials_doubles(n_rhs, n_sites);
      if (need > tl::kNoallocPartials)
        return fail(c, TL_ERR_SHAPE,
                    "tl_reduce_noalloc: %lld partial sums needed, the fixed area holds %lld "
                    "(n_rhs * ceil(n_sites / 4096) must not exceed %lld)",
                    (long long)need, (long long)tl::kNoallocPartials, (long long)(tl::kNoallocPartials / 2));
    }
    TL_TRY(need_device(c));
    TL_ON_DEVICE(c);
    if (!c->noalloc) return fail(c, TL_ERR_HIP, "no fixed reduction area on device %d (%s)", c->device, c->noalloc_err.c_str());
    return launch(c, "reduction", [&] { return tl::launch_reduce_flat(kind, psi, phi, n_sites, n_rhs, c->noalloc, out, c->stream); });
  } catch (...) {
    return host_failure(c);
  }
}

int tl_reduce(tl_ctx* c, int kind, int64_t n_sites, int n_rhs, const void* psi, const void* phi, double* out) {
  try {
    if (!c) return TL_ERR_ARG;
    TL_TRY(check_reduce_args(c, kind, n_sites, n_rhs, psi, phi, out));
    TL_TRY(need_device(c));
    TL_ON_DEVICE(c);
    std::vector<tl::RedField> rf(n_rhs);
    for (int r = 0; r < n_rhs; r++) rf[r] = {(int64_t)r * n_sites * 3, (int64_t)r * n_sites * 3, n_sites, 0, (int64_t)r * n_sites};
    const size_t fbytes = align256(rf.size() * sizeof(tl::RedField));
    const size_t pbytes = (size_t)tl::red_partials_doubles(n_rhs, n_sites) * sizeof(double);
    char* s = nullptr;
    TL_TRY(ctx_scratch(c, fbytes + pbytes, &s));
    TL_TRY(upload(c, s, rf.data(), rf.size() * sizeof(tl::RedField)));
    // a = psi, b = phi: <phi, psi>
    return launch(c, "reduction", [&] { return tl::launch_reduce(kind, -1, static_cast<const char*>(psi), static_cast<const char*>(phi),
                                          reinterpret_cast<const tl::RedField*>(s), n_rhs, n_sites,
                                          reinterpret_cast<double*>(s + fbytes), out, c->stream); });
  } catch (...) {
    return host_failure(c);
  }
}

}  // extern "C"
