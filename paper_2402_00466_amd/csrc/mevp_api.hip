// mevp_api.hip -- host runtime behind the C ABI of include/mevp.h.
//
// Holds no numerics: validates arguments on the host, carves the caller's
// device workspace into the context's arrays, builds the block -> (domain,
// first element/node) maps for batched launches, and enqueues the kernels of
// mevp_kernels.hip on the context's stream.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "mevp.h"
#include "mevp_index.hpp"
#include "mevp_internal.hpp"

using namespace mevp;

struct mevp_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  mevp_precision prec = MEVP_FP64;
  mevp_params params{};
  KParams kp{};
  int nd = 0, ns = 0, na = 0;
  std::vector<mevp_domain_desc> desc;
  std::vector<DomDev> dom_h;
  std::vector<Blk> eblk_h, nblk_h;
  int n_nblk = 0;                     // node blocks (nblk_h.size(); kept apart for mevp_step_static)
  std::vector<Tile> tiles_h;
  Launch eblk_split{};                // element blocks grouped by geometry kind (GeoKind order)
  Launch tile_split{};                // tiles likewise
  Tile *tiles_d = nullptr;
  int cur = 0;                        // which of the two v / S buffers holds the state
  mevp_strategy strategy = MEVP_STRATEGY_FUSED;
  int shape = 0;                      // fused-kernel tile shape (index into kTileShapes)
  DevArrays d{};
  DomDev *doms_d = nullptr;
  Blk *eblk_d = nullptr, *nblk_d = nullptr;
  size_t tot_e = 0, tot_n = 0, tot_v = 0;
  std::vector<unsigned char> geo_set, fld_set, frc_set;
  // optional kernel timing: event pairs per phase
  struct Timer {
    std::vector<hipEvent_t> ev;  // 2 per launch
    int used = 0;
  } timer[3];
  int timer_cap = 0;
  // one captured time step per state-buffer parity (hipGraph replay)
  struct StepGraph {
    int n = -1;
    int cur_after = 0;
    hipGraph_t g = nullptr;
    hipGraphExec_t x = nullptr;
  } graphs[2];
  hipStream_t cap = nullptr;  // private stream for the captures
  bool use_graph = true;
};

namespace {

constexpr size_t kAlign = 256;
constexpr long long kIndexMax = 0x7fffffffLL;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

bool finite(double x) { return isfinite(x) != 0; }

// Host-side log on stderr, enabled by the environment variable MEVP_LOG (read
// once per process): 1 = context creation, autotuning trials and choice,
// step-graph capture failures and failing calls; 2 = also every launch
// configuration set and every step graph captured. Logging never changes a
// result or a status.
int log_level() {
  static const int level = [] {
    const char *e = getenv("MEVP_LOG");
    return e ? atoi(e) : 0;
  }();
  return level;
}

__attribute__((format(printf, 2, 3))) void mlog(int level, const char *fmt, ...) {
  if (log_level() < level) return;
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  fprintf(stderr, "[mevp] %s\n", buf);
}

const char *strategy_name(int s) {
  switch (s) {
    case MEVP_STRATEGY_FUSED: return "fused";
    case MEVP_STRATEGY_TWO_PHASE: return "two_phase";
    case MEVP_STRATEGY_PERSISTENT: return "persistent";
    case MEVP_STRATEGY_FUSED_PAIR: return "fused_pair";
    case MEVP_STRATEGY_FUSED_TRIPLE: return "fused_triple";
  }
  return "?";
}

const char *precision_name(int p) {
  return p == MEVP_FP64 ? "fp64" : p == MEVP_MIXED ? "mixed" : p == MEVP_MIXED_BF16 ? "mixed_bf16" : "?";
}

// A call's status, logged when it is not MEVP_OK.
mevp_status logged(const char *call, mevp_status st) {
  if (st != MEVP_OK) mlog(1, "%s: %s (status %d)", call, mevp_status_string(st), (int)st);
  return st;
}

mevp_status validate_params(const mevp_params *p) {
  if (!p) return MEVP_EINVAL;
  const double v[] = {p->Pstar, p->C, p->DeltaMin, p->alpha, p->beta, p->rho_i, p->rho_a,
                      p->C_a, p->rho_o, p->C_o, p->f_cor, p->dt};
  for (double x : v)
    if (!finite(x)) return MEVP_EINVAL;
  if (p->Pstar < 0 || p->DeltaMin < 1e-100 || p->alpha <= 0 || p->beta < 0 || p->dt <= 0 ||
      p->rho_i <= 0 || p->rho_a < 0 || p->C_a < 0 || p->rho_o < 0 || p->C_o < 0)
    return MEVP_EINVAL;
  if (p->relax_form != 0 && p->relax_form != 1) return MEVP_EINVAL;
  return MEVP_OK;
}

KParams derive(const mevp_params &p) {
  KParams k{};
  k.Pstar = p.Pstar;
  k.C = p.C;
  k.dmin2 = p.DeltaMin * p.DeltaMin;
  k.dmin2_16 = k.dmin2 / 16.0;
  if (p.relax_form == 1) {
    k.fac = p.alpha / (1.0 + p.alpha);
    k.ainv = 1.0 / (1.0 + p.alpha);
  } else {
    k.ainv = 1.0 / p.alpha;
    k.fac = 1.0 - k.ainv;
  }
  k.beta = p.beta;
  k.inv_dt = 1.0 / p.dt;
  k.rho_i = p.rho_i;
  k.rhoCa = p.rho_a * p.C_a;
  k.rhoCo = p.rho_o * p.C_o;
  k.f_dt = p.f_cor * p.dt;
  return k;
}

// Layout of the workspace: offsets in bytes of every array.
struct Layout {
  size_t doms, eblk, nblk, tiles, flag, vert, xnode, H, A, adv, wind, ocean, v, nc, S, fe, total;
  size_t tot_e, tot_n, tot_v;
  int n_eblk, n_nblk;
  int ns, na;
};

mevp_status plan(const mevp_domain_desc *dd, int nd, mevp_precision prec, Layout *L) {
  if (!dd || nd < 1) return MEVP_EINVAL;
  if (prec != MEVP_FP64 && prec != MEVP_MIXED && prec != MEVP_MIXED_BF16) return MEVP_EINVAL;
  const int ns = dd[0].n_s, na = dd[0].n_a;
  if (!(ns == 3 || ns == 6 || ns == 8) || !(na == 1 || na == 3 || na == 6)) return MEVP_EINVAL;
  if (prec == MEVP_MIXED_BF16 && (ns != 6 || na != 1)) return MEVP_EINVAL;  // the trial's kernels
  long long te = 0, tn = 0, tv = 0, neb = 0, nnb = 0, ntl = 0;
  for (int i = 0; i < nd; ++i) {
    const mevp_domain_desc &d = dd[i];
    if (d.n_s != ns || d.n_a != na) return MEVP_EINVAL;
    if (d.nx < 1 || d.ny < 1 || d.nx > 1000000 || d.ny > 1000000) return MEVP_EINVAL;
    const long long e = (long long)d.nx * d.ny;
    const long long n = (2LL * d.nx + 1) * (2LL * d.ny + 1);
    const long long v = ((long long)d.nx + 1) * (d.ny + 1);
    te += e;
    tn += n;
    tv += v;
    neb += (e + kElemBlock - 1) / kElemBlock;
    nnb += (n + kNodeBlock - 1) / kNodeBlock;
    long long most = 0;  // tile table sized for the shape with the most tiles
    for (int sh = 0; sh < kNumTileShapes; ++sh) {
      const int tx = kTileShapes[sh][0] - 1, ty = kTileShapes[sh][1] - 1;
      const long long nt = (long long)((d.nx + tx - 1) / tx) * ((d.ny + ty - 1) / ty);
      if (nt > most) most = nt;
    }
    ntl += most;
    if (te > kIndexMax || tn > kIndexMax || 2 * tn > kIndexMax || 18 * te > (1LL << 40))
      return MEVP_EINVAL;
  }
  const size_t ws = (prec == MEVP_FP64) ? sizeof(double) : sizeof(float);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = align_up(off + bytes);
    return o;
  };
  L->doms = take(sizeof(DomDev) * nd);
  L->eblk = take(sizeof(Blk) * neb);
  L->nblk = take(sizeof(Blk) * nnb);
  L->tiles = take(sizeof(Tile) * ntl);
  L->flag = take(sizeof(int) * 4);
  L->vert = take(sizeof(double) * 2 * tv);
  L->xnode = take(sizeof(double) * 2 * tn);
  L->H = take(sizeof(double) * na * te);
  L->A = take(sizeof(double) * na * te);
  L->adv = take(sizeof(double) * 4 * na * te);
  L->wind = take(sizeof(double) * 2 * tn);
  L->ocean = take(sizeof(double) * 2 * tn);
  L->v = take(sizeof(double) * 4 * tn);
  L->nc = take(sizeof(double) * 6 * tn);
  L->S = take(ws * 6 * ns * te);
  L->fe = take(ws * 18 * te);
  L->total = off;
  L->tot_e = (size_t)te;
  L->tot_n = (size_t)tn;
  L->tot_v = (size_t)tv;
  L->n_eblk = (int)neb;
  L->n_nblk = (int)nnb;
  L->ns = ns;
  L->na = na;
  return MEVP_OK;
}

mevp_status hip_status(hipError_t e) { return e == hipSuccess ? MEVP_OK : MEVP_EDEVICE; }

bool bad_dom(const mevp_ctx *c, int dom) { return !c || dom < 0 || dom >= c->nd; }

// copy with either host or device source/destination, stream-ordered
mevp_status copy(void *dst, const void *src, size_t bytes, hipStream_t s) {
  if (bytes == 0) return MEVP_OK;
  return hip_status(hipMemcpyAsync(dst, src, bytes, hipMemcpyDefault, s));
}

void timer_free(mevp_ctx *c) {
  for (auto &t : c->timer) {
    for (hipEvent_t e : t.ev)
      if (e) (void)hipEventDestroy(e);
    t.ev.clear();
    t.used = 0;
  }
  c->timer_cap = 0;
}

// Record the start event of phase `ph` if timing is on and slots remain;
// returns the slot or -1.
int timer_start(mevp_ctx *c, int ph) {
  auto &t = c->timer[ph];
  if (c->timer_cap == 0 || t.used >= c->timer_cap) return -1;
  if (hipEventRecord(t.ev[2 * t.used], c->stream) != hipSuccess) return -1;
  return t.used;
}
void timer_stop(mevp_ctx *c, int ph, int slot) {
  if (slot < 0) return;
  auto &t = c->timer[ph];
  if (hipEventRecord(t.ev[2 * slot + 1], c->stream) == hipSuccess) t.used = slot + 1;
}

void graphs_clear(mevp_ctx *c) {
  for (auto &g : c->graphs) {
    if (g.x) (void)hipGraphExecDestroy(g.x);
    if (g.g) (void)hipGraphDestroy(g.g);
    g = mevp_ctx::StepGraph{};
  }
}

// Element blocks and fused-kernel tiles grouped by the geometry kind of their
// domain (GeoKind order: parallelogram, bilinear, isoparametric), one launch of
// the matching element kernel per non-empty group.
void order_blocks(mevp_ctx *c) {
  c->eblk_h.clear();
  c->tiles_h.clear();
  const int TX = kTileShapes[c->shape][0] - 1, TY = kTileShapes[c->shape][1] - 1;
  for (int kind = 0; kind < kNumGeo; ++kind) {
    const size_t e0 = c->eblk_h.size(), t0 = c->tiles_h.size();
    for (int i = 0; i < c->nd; ++i) {
      if (c->dom_h[i].kind != kind) continue;
      const DomDev &D = c->dom_h[i];
      for (int f = 0; f < D.ne; f += kElemBlock) c->eblk_h.push_back(Blk{i, f});
      const int ntx = (D.nx + TX - 1) / TX, nty = (D.ny + TY - 1) / TY;
      for (int k = 0; k < ntx * nty; ++k) {
        int col, row;
        strip_tile(k, ntx, nty, strip_width(TX, kStripElems), col, row);
        c->tiles_h.push_back(Tile{i, col * TX, row * TY, 0});
      }
    }
    c->eblk_split.n[kind] = (int)(c->eblk_h.size() - e0);
    c->tile_split.n[kind] = (int)(c->tiles_h.size() - t0);
  }
  // Workgroup i of a launch runs on XCD i % 8. Permute each launch's tiles so
  // that every XCD gets one contiguous band of the strip-ordered list:
  // neighbouring tiles share halo elements and cache lines, which then meet in
  // the same L2.
  auto xcd_order = [](Tile *t, int n) {
    std::vector<Tile> src(t, t + n);
    int start = 0;
    for (int x = 0; x < kNumXcd; ++x) {
      const int cnt = (n - x + kNumXcd - 1) / kNumXcd;  // workgroups x, x+8, ...
      for (int s = 0; s < cnt; ++s) t[x + s * kNumXcd] = src[start + s];
      start += cnt;
    }
  };
  int t0 = 0;
  for (int kind = 0; kind < kNumGeo; ++kind) {
    xcd_order(c->tiles_h.data() + t0, c->tile_split.n[kind]);
    t0 += c->tile_split.n[kind];
  }
}

// Host allocations (the context, its block tables, the tuner's state copies)
// may fail; no exception crosses the C ABI: an exhausted host heap becomes
// MEVP_EHOSTMEM and anything else thrown MEVP_EINTERNAL.
template <class F>
mevp_status host_guard(F &&f) noexcept {
  try {
    return f();
  } catch (const std::bad_alloc &) {
    return MEVP_EHOSTMEM;
  } catch (...) {
    return MEVP_EINTERNAL;
  }
}

size_t s_words(const mevp_ctx *c) { return (size_t)3 * c->ns * c->tot_e; }
size_t s_bytes(const mevp_ctx *c) {
  return (c->prec == MEVP_FP64 ? sizeof(double) : sizeof(float));
}
// current / other state buffers
double *v_buf(mevp_ctx *c, int which) { return c->d.v + (size_t)which * 2 * c->tot_n; }
void *S_buf(mevp_ctx *c, int which) {
  return static_cast<char *>(c->d.S) + (size_t)which * s_words(c) * s_bytes(c);
}

}  // namespace

extern "C" {

const char *mevp_version(void) { return "mevp-gfx950 0.1.0"; }

const char *mevp_status_string(mevp_status s) {
  switch (s) {
    case MEVP_OK: return "ok";
    case MEVP_EINVAL: return "invalid argument";
    case MEVP_ENOMEM: return "workspace too small";
    case MEVP_EDEVICE: return "device error";
    case MEVP_ESTATE: return "call out of order";
    case MEVP_ENONFINITE: return "non-finite or invalid values";
    case MEVP_EUNSUPPORTED: return "unsupported device";
    case MEVP_EINTERNAL: return "internal self-check failed";
    case MEVP_EHOSTMEM: return "host memory allocation failed";
  }
  return "unknown status";
}

mevp_status mevp_default_params(mevp_params *out) {
  if (!out) return MEVP_EINVAL;
  out->Pstar = 27500.0;
  out->C = 20.0;
  out->DeltaMin = 2e-9;
  out->alpha = 300.0;
  out->beta = 300.0;
  out->rho_i = 900.0;
  out->rho_a = 1.3;
  out->C_a = 1.2e-3;
  out->rho_o = 1026.0;
  out->C_o = 5.5e-3;
  out->f_cor = 1.46e-4;
  out->dt = 120.0;
  out->relax_form = 0;
  return MEVP_OK;
}

mevp_status mevp_workspace_size(const mevp_domain_desc *domains, int n_domains,
                                mevp_precision precision, size_t *bytes) {
  if (!bytes) return MEVP_EINVAL;
  Layout L;
  mevp_status st = plan(domains, n_domains, precision, &L);
  if (st != MEVP_OK) return st;
  *bytes = L.total;
  return MEVP_OK;
}

static mevp_status create_impl(const mevp_params *params, mevp_precision precision,
                               const mevp_domain_desc *domains, int n_domains, void *workspace,
                               size_t ws_bytes, void *hip_stream, mevp_ctx **out) {
  if (!out) return MEVP_EINVAL;
  *out = nullptr;
  mevp_status st = validate_params(params);
  if (st != MEVP_OK) return st;
  Layout L;
  st = plan(domains, n_domains, precision, &L);
  if (st != MEVP_OK) return st;
  if (!workspace || (reinterpret_cast<uintptr_t>(workspace) % kAlign) != 0) return MEVP_EINVAL;
  if (ws_bytes < L.total) return MEVP_ENOMEM;

  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return MEVP_EDEVICE;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return MEVP_EDEVICE;
  if (strncmp(prop.gcnArchName, "gfx950", 6) != 0) return MEVP_EUNSUPPORTED;

  std::unique_ptr<mevp_ctx> owner(new mevp_ctx());
  mevp_ctx *c = owner.get();
  c->device = dev;
  c->stream = static_cast<hipStream_t>(hip_stream);
  c->prec = precision;
  c->params = *params;
  c->kp = derive(*params);
  c->nd = n_domains;
  c->ns = L.ns;
  c->na = L.na;
  c->desc.assign(domains, domains + n_domains);
  c->tot_e = L.tot_e;
  c->tot_n = L.tot_n;
  c->tot_v = L.tot_v;
  c->geo_set.assign(n_domains, 0);
  c->fld_set.assign(n_domains, 0);
  c->frc_set.assign(n_domains, 0);

  int eo = 0, no = 0, vo = 0;
  for (int i = 0; i < n_domains; ++i) {
    const mevp_domain_desc &dd = domains[i];
    DomDev D;
    D.nx = dd.nx;
    D.ny = dd.ny;
    D.ne = dd.nx * dd.ny;
    D.nn = (2 * dd.nx + 1) * (2 * dd.ny + 1);
    D.nv = (dd.nx + 1) * (dd.ny + 1);
    D.elem_off = eo;
    D.node_off = no;
    D.vert_off = vo;
    D.kind = kGeoBilinear;  // until set_geometry classifies the cells
    eo += D.ne;
    no += D.nn;
    vo += D.nv;
    c->dom_h.push_back(D);
    for (int f = 0; f < D.nn; f += kNodeBlock) c->nblk_h.push_back(Blk{i, f});
  }
  c->n_nblk = (int)c->nblk_h.size();
  order_blocks(c);

  char *base = static_cast<char *>(workspace);
  c->doms_d = reinterpret_cast<DomDev *>(base + L.doms);
  c->eblk_d = reinterpret_cast<Blk *>(base + L.eblk);
  c->nblk_d = reinterpret_cast<Blk *>(base + L.nblk);
  c->tiles_d = reinterpret_cast<Tile *>(base + L.tiles);
  DevArrays &d = c->d;
  d.doms = c->doms_d;
  d.eblk = c->eblk_d;
  d.nblk = c->nblk_d;
  d.tiles = c->tiles_d;
  d.flag = reinterpret_cast<int *>(base + L.flag);
  d.vert = reinterpret_cast<double *>(base + L.vert);
  d.xnode = reinterpret_cast<double *>(base + L.xnode);
  d.H = reinterpret_cast<double *>(base + L.H);
  d.A = reinterpret_cast<double *>(base + L.A);
  d.adv = reinterpret_cast<double *>(base + L.adv);
  d.wind = reinterpret_cast<double *>(base + L.wind);
  d.ocean = reinterpret_cast<double *>(base + L.ocean);
  d.v = reinterpret_cast<double *>(base + L.v);
  d.nc = reinterpret_cast<double *>(base + L.nc);
  d.S = base + L.S;
  d.fe = base + L.fe;

  hipStream_t s = c->stream;
  mevp_status rc = copy(c->doms_d, c->dom_h.data(), sizeof(DomDev) * n_domains, s);
  if (rc == MEVP_OK) rc = copy(c->eblk_d, c->eblk_h.data(), sizeof(Blk) * c->eblk_h.size(), s);
  if (rc == MEVP_OK) rc = copy(c->nblk_d, c->nblk_h.data(), sizeof(Blk) * c->nblk_h.size(), s);
  if (rc == MEVP_OK) rc = copy(c->tiles_d, c->tiles_h.data(), sizeof(Tile) * c->tiles_h.size(), s);
  // zero everything after the tables: fields, state, scratch
  if (rc == MEVP_OK)
    rc = hip_status(launch_fill(base + L.flag, (L.total - L.flag) / 4, 0u, s));
  // the host vectors above must outlive the asynchronous copies
  if (rc == MEVP_OK) rc = hip_status(hipStreamSynchronize(s));
  if (rc != MEVP_OK) return rc;
  *out = owner.release();
  return MEVP_OK;
}

mevp_status mevp_create(const mevp_params *params, mevp_precision precision,
                        const mevp_domain_desc *domains, int n_domains, void *workspace,
                        size_t ws_bytes, void *hip_stream, mevp_ctx **out) {
  if (out) *out = nullptr;
  const mevp_status st = host_guard([&] {
    return create_impl(params, precision, domains, n_domains, workspace, ws_bytes, hip_stream,
                       out);
  });
  if (st == MEVP_OK)
    mlog(1, "create: %d domain(s), %zu elements, %zu nodes, %s, n_s %d, n_a %d, workspace %zu bytes, device %d",
         n_domains, (*out)->tot_e, (*out)->tot_n, precision_name(precision), (*out)->ns,
         (*out)->na, ws_bytes, (*out)->device);
  return logged("mevp_create", st);
}

mevp_status mevp_set_params(mevp_ctx *ctx, const mevp_params *params) {
  if (!ctx) return MEVP_EINVAL;
  mevp_status st = validate_params(params);
  if (st != MEVP_OK) return st;
  ctx->params = *params;
  ctx->kp = derive(*params);
  graphs_clear(ctx);  // kernel arguments changed
  return MEVP_OK;
}

// Record the geometry kind of a domain; when it changes, the domain table,
// the launch grouping and the captured graphs are rebuilt.
static mevp_status set_kind(mevp_ctx *ctx, int dom, int kind) {
  if (ctx->dom_h[dom].kind == kind) return MEVP_OK;
  hipStream_t s = ctx->stream;
  graphs_clear(ctx);
  const int old = ctx->dom_h[dom].kind;
  ctx->dom_h[dom].kind = kind;
  mevp_status ht = host_guard([&] {
    order_blocks(ctx);
    return MEVP_OK;
  });
  if (ht != MEVP_OK) {
    ctx->dom_h[dom].kind = old;
    (void)host_guard([&] {
      order_blocks(ctx);  // the previous tables, same sizes as before
      return MEVP_OK;
    });
    return ht;
  }
  mevp_status st = copy(ctx->doms_d, ctx->dom_h.data(), sizeof(DomDev) * ctx->nd, s);
  if (st == MEVP_OK) st = copy(ctx->eblk_d, ctx->eblk_h.data(), sizeof(Blk) * ctx->eblk_h.size(), s);
  if (st == MEVP_OK) st = copy(ctx->tiles_d, ctx->tiles_h.data(), sizeof(Tile) * ctx->tiles_h.size(), s);
  // the host tables must outlive the asynchronous copies
  if (st == MEVP_OK) st = hip_status(hipStreamSynchronize(s));
  return st;
}

mevp_status mevp_set_geometry(mevp_ctx *ctx, int dom, const double *vertex_xy) {
  if (bad_dom(ctx, dom) || !vertex_xy) return MEVP_EINVAL;
  const DomDev &D = ctx->dom_h[dom];
  hipStream_t s = ctx->stream;
  mevp_status st = copy(const_cast<double *>(ctx->d.vert) + 2 * (size_t)D.vert_off, vertex_xy,
                        sizeof(double) * 2 * D.nv, s);
  // classify the cells: all parallelograms -> the constant-Jacobian kernel
  int *flag = ctx->d.flag + 1;
  if (st == MEVP_OK) st = hip_status(launch_fill(flag, 1, 1u, s));
  if (st == MEVP_OK) st = hip_status(launch_cell_shape(ctx->d, dom, D.ne, flag, s));
  int aff = 0;
  if (st == MEVP_OK) st = hip_status(hipMemcpyAsync(&aff, flag, sizeof(int), hipMemcpyDeviceToHost, s));
  if (st == MEVP_OK) st = hip_status(hipStreamSynchronize(s));
  if (st == MEVP_OK) st = set_kind(ctx, dom, aff ? kGeoAffine : kGeoBilinear);
  if (st == MEVP_OK) ctx->geo_set[dom] = 1;
  return st;
}

mevp_status mevp_set_geometry_cg2(mevp_ctx *ctx, int dom, const double *node_xy) {
  if (bad_dom(ctx, dom) || !node_xy) return MEVP_EINVAL;
  if (ctx->prec == MEVP_MIXED_BF16) return MEVP_EINVAL;  // vertex geometry only
  const DomDev &D = ctx->dom_h[dom];
  hipStream_t s = ctx->stream;
  mevp_status st = copy(const_cast<double *>(ctx->d.xnode) + 2 * (size_t)D.node_off, node_xy,
                        sizeof(double) * 2 * D.nn, s);
  // the vertices (corner nodes) are kept for the input checks
  if (st == MEVP_OK) st = hip_status(launch_corner_vertices(ctx->d, dom, D.nv, s));
  if (st == MEVP_OK) st = hip_status(hipStreamSynchronize(s));
  if (st == MEVP_OK) st = set_kind(ctx, dom, kGeoIso);
  if (st == MEVP_OK) ctx->geo_set[dom] = 1;
  return st;
}

mevp_status mevp_set_fields(mevp_ctx *ctx, int dom, const double *H, const double *A) {
  if (bad_dom(ctx, dom) || !H || !A) return MEVP_EINVAL;
  const DomDev &D = ctx->dom_h[dom];
  const size_t n = (size_t)ctx->na * D.ne;
  mevp_status st = copy(const_cast<double *>(ctx->d.H) + (size_t)ctx->na * D.elem_off, H,
                        sizeof(double) * n, ctx->stream);
  if (st == MEVP_OK)
    st = copy(const_cast<double *>(ctx->d.A) + (size_t)ctx->na * D.elem_off, A,
              sizeof(double) * n, ctx->stream);
  if (st == MEVP_OK) ctx->fld_set[dom] = 1;
  return st;
}

mevp_status mevp_set_forcing(mevp_ctx *ctx, int dom, const double *wind_xy,
                             const double *ocean_xy) {
  if (bad_dom(ctx, dom) || !wind_xy || !ocean_xy) return MEVP_EINVAL;
  const DomDev &D = ctx->dom_h[dom];
  const size_t o = 2 * (size_t)D.node_off, n = 2 * (size_t)D.nn;
  mevp_status st = copy(const_cast<double *>(ctx->d.wind) + o, wind_xy, sizeof(double) * n,
                        ctx->stream);
  if (st == MEVP_OK)
    st = copy(const_cast<double *>(ctx->d.ocean) + o, ocean_xy, sizeof(double) * n, ctx->stream);
  if (st == MEVP_OK) ctx->frc_set[dom] = 1;
  return st;
}

mevp_status mevp_set_state(mevp_ctx *ctx, int dom, const double *v_xy, const double *S) {
  if (bad_dom(ctx, dom) || !v_xy || !S) return MEVP_EINVAL;
  const DomDev &D = ctx->dom_h[dom];
  const size_t n = (size_t)3 * ctx->ns * D.ne, o = (size_t)3 * ctx->ns * D.elem_off;
  if (ctx->prec != MEVP_FP64) {
    hipPointerAttribute_t attr;
    if (hipPointerGetAttributes(&attr, S) != hipSuccess || attr.type != hipMemoryTypeDevice) {
      (void)hipGetLastError();
      return MEVP_EINVAL;  // the rounding to float runs on the device: S must be device memory
    }
  }
  // v_xy (host or device, [2][nn]) to the other state buffer, then interleaved
  // per node ([nn][2]) into the current one: the other buffer is free until
  // the next subcycle writes it
  const size_t vo = 2 * (size_t)D.node_off;
  mevp_status st = copy(v_buf(ctx, ctx->cur ^ 1) + vo, v_xy, sizeof(double) * 2 * D.nn, ctx->stream);
  if (st == MEVP_OK)
    st = hip_status(launch_interleave2(v_buf(ctx, ctx->cur ^ 1) + vo, v_buf(ctx, ctx->cur) + vo,
                                       (size_t)D.nn, ctx->stream));
  if (st != MEVP_OK) return st;
  // S to the kernels' [3][ne][n_s]: in FP64 through the other state buffer (S
  // may be host memory), in the mixed forms straight from S (device memory)
  const size_t ne = (size_t)D.ne;
  if (ctx->prec == MEVP_FP64) {
    double *stage = static_cast<double *>(S_buf(ctx, ctx->cur ^ 1)) + o;
    st = copy(stage, S, sizeof(double) * n, ctx->stream);
    if (st == MEVP_OK)
      st = hip_status(launch_stress_in(stage, static_cast<double *>(S_buf(ctx, ctx->cur)) + o,
                                       false, ne, ctx->ns, ctx->stream));
    return st;
  }
  return hip_status(launch_stress_in(S, static_cast<float *>(S_buf(ctx, ctx->cur)) + o, true, ne,
                                     ctx->ns, ctx->stream));
}

mevp_status mevp_get_state(mevp_ctx *ctx, int dom, double *v_xy, double *S) {
  if (bad_dom(ctx, dom)) return MEVP_EINVAL;
  const DomDev &D = ctx->dom_h[dom];
  if (S && ctx->prec != MEVP_FP64) {
    hipPointerAttribute_t attr;
    if (hipPointerGetAttributes(&attr, S) != hipSuccess || attr.type != hipMemoryTypeDevice) {
      (void)hipGetLastError();
      return MEVP_EINVAL;
    }
  }
  if (v_xy) {
    // back to [2][nn] through the other state buffer (free until the next
    // subcycle), then to v_xy (host or device)
    const size_t vo = 2 * (size_t)D.node_off;
    mevp_status st = hip_status(launch_deinterleave2(v_buf(ctx, ctx->cur) + vo,
                                                     v_buf(ctx, ctx->cur ^ 1) + vo, (size_t)D.nn,
                                                     ctx->stream));
    if (st == MEVP_OK)
      st = copy(v_xy, v_buf(ctx, ctx->cur ^ 1) + vo, sizeof(double) * 2 * D.nn, ctx->stream);
    if (st != MEVP_OK) return st;
  }
  if (S) {
    // back to [3][n_s][ne]: in FP64 through the other state buffer, then to S
    // (host or device); in the mixed forms straight into S (device memory)
    const size_t n = (size_t)3 * ctx->ns * D.ne, o = (size_t)3 * ctx->ns * D.elem_off;
    const size_t ne = (size_t)D.ne;
    if (ctx->prec == MEVP_FP64) {
      double *stage = static_cast<double *>(S_buf(ctx, ctx->cur ^ 1)) + o;
      mevp_status st = hip_status(launch_stress_out(static_cast<const double *>(S_buf(ctx, ctx->cur)) + o,
                                                    false, stage, ne, ctx->ns, ctx->stream));
      if (st == MEVP_OK) st = copy(S, stage, sizeof(double) * n, ctx->stream);
      return st;
    }
    return hip_status(launch_stress_out(static_cast<const float *>(S_buf(ctx, ctx->cur)) + o, true,
                                        S, ne, ctx->ns, ctx->stream));
  }
  return MEVP_OK;
}

static bool inputs_set(const mevp_ctx *ctx) {
  for (int i = 0; i < ctx->nd; ++i)
    if (!ctx->geo_set[i] || !ctx->fld_set[i] || !ctx->frc_set[i]) return false;
  return true;
}

static mevp_status begin_step_on(mevp_ctx *ctx, hipStream_t stream) {
  const int slot = timer_start(ctx, 2);
  int ntiles = 0;
  for (int k = 0; k < kNumGeo; ++k) ntiles += ctx->tile_split.n[k];
  mevp_status st = hip_status(launch_begin_step(ctx->d, ctx->kp, ctx->na, ctx->ns,
                                                v_buf(ctx, ctx->cur), ctx->shape, ntiles,
                                                stream));
  timer_stop(ctx, 2, slot);
  return st;
}

mevp_status mevp_begin_step(mevp_ctx *ctx) {
  if (!ctx) return MEVP_EINVAL;
  if (!inputs_set(ctx)) return logged("mevp_begin_step", MEVP_ESTATE);
  return logged("mevp_begin_step", begin_step_on(ctx, ctx->stream));
}

// Subcycles per launch of the fused strategies: FUSED_PAIR / FUSED_TRIPLE run
// 2 / 3, but three per launch exist for parallelogram cells only (with a
// bilinear domain FUSED_TRIPLE runs two per launch) and with an isoparametric
// domain both run one per launch.
static int fused_depth(const mevp_ctx *ctx) {
  const Launch &ts = ctx->tile_split;
  int most = ctx->strategy == MEVP_STRATEGY_FUSED_TRIPLE ? 3
             : ctx->strategy == MEVP_STRATEGY_FUSED_PAIR ? 2 : 1;
  if (most == 3 && ts.n[kGeoBilinear] > 0) most = 2;
  if (ts.n[kGeoIso] > 0) most = 1;
  return most;
}

// The persistent strategy runs all subcycles of a call in one cooperative
// launch when every tile takes the same kernel (one geometry kind).
static bool persistent_whole(const mevp_ctx *ctx) {
  int kinds = 0;
  for (int k = 0; k < kNumGeo; ++k) kinds += ctx->tile_split.n[k] > 0;
  return ctx->strategy == MEVP_STRATEGY_PERSISTENT && kinds == 1;
}

mevp_status mevp_get_launch_depth(mevp_ctx *ctx, int *depth) {
  if (!ctx || !depth) return MEVP_EINVAL;
  if (persistent_whole(ctx))
    *depth = 0;
  else if (ctx->strategy == MEVP_STRATEGY_TWO_PHASE || ctx->strategy == MEVP_STRATEGY_PERSISTENT)
    *depth = 1;
  else
    *depth = fused_depth(ctx);
  return MEVP_OK;
}

static mevp_status subcycles_on(mevp_ctx *ctx, int n, hipStream_t stream) {
  const int prec = ctx->prec;
  if (n == 0) return MEVP_OK;
  if (persistent_whole(ctx)) {
    const int nxt = ctx->cur ^ 1;
    FusedArgs f;
    f.b0 = Bufs{v_buf(ctx, ctx->cur), v_buf(ctx, nxt), S_buf(ctx, ctx->cur), S_buf(ctx, nxt)};
    f.b1 = Bufs{v_buf(ctx, nxt), v_buf(ctx, ctx->cur), S_buf(ctx, nxt), S_buf(ctx, ctx->cur)};
    f.shape = ctx->shape;
    f.persist = 1;
    f.n_sub = n;
    f.depth = 1;
    const int slot = timer_start(ctx, 0);
    hipError_t e = launch_fused_subcycle(ctx->d, ctx->kp, ctx->ns, ctx->na, prec, ctx->tile_split,
                                         f, stream);
    timer_stop(ctx, 0, slot);
    if (e == hipSuccess) {
      if (n & 1) ctx->cur = nxt;
      return MEVP_OK;
    }
    if (e != hipErrorCooperativeLaunchTooLarge) return MEVP_EDEVICE;
    (void)hipGetLastError();  // too many tiles resident per CU: one launch per subcycle
  }
  for (int it = 0; it < n; ++it) {
    hipError_t e;
    if (ctx->strategy != MEVP_STRATEGY_TWO_PHASE) {
      // FUSED_PAIR / FUSED_TRIPLE: fused_depth subcycles per launch while that
      // many remain, then the rest in one launch
      const int most = fused_depth(ctx);
      const int depth = most < n - it ? most : n - it;
      const int nxt = ctx->cur ^ 1;
      FusedArgs f;
      f.b0 = Bufs{v_buf(ctx, ctx->cur), v_buf(ctx, nxt), S_buf(ctx, ctx->cur), S_buf(ctx, nxt)};
      f.b1 = f.b0;
      f.shape = ctx->shape;
      f.persist = 0;
      f.n_sub = depth;
      f.depth = depth;
      const int slot = timer_start(ctx, 0);
      e = launch_fused_subcycle(ctx->d, ctx->kp, ctx->ns, ctx->na, prec, ctx->tile_split, f,
                                stream);
      timer_stop(ctx, 0, slot);
      if (e == hipSuccess) ctx->cur = nxt;
      it += depth - 1;
    } else {
      const Bufs b{v_buf(ctx, ctx->cur), v_buf(ctx, ctx->cur), S_buf(ctx, ctx->cur),
                   S_buf(ctx, ctx->cur)};
      int slot = timer_start(ctx, 0);
      e = launch_element_phase(ctx->d, ctx->kp, ctx->ns, ctx->na, prec, ctx->eblk_split, b,
                               stream);
      timer_stop(ctx, 0, slot);
      if (e == hipSuccess) {
        slot = timer_start(ctx, 1);
        e = launch_node_phase(ctx->d, ctx->kp, prec != MEVP_FP64, ctx->n_nblk, b, stream);
        timer_stop(ctx, 1, slot);
      }
    }
    if (e != hipSuccess) return MEVP_EDEVICE;
  }
  return MEVP_OK;
}

mevp_status mevp_subcycles(mevp_ctx *ctx, int n) {
  if (!ctx || n < 0) return MEVP_EINVAL;
  if (!inputs_set(ctx)) return logged("mevp_subcycles", MEVP_ESTATE);
  return logged("mevp_subcycles", subcycles_on(ctx, n, ctx->stream));
}

mevp_status mevp_advect(mevp_ctx *ctx) {
  if (!ctx) return MEVP_EINVAL;
  if (!inputs_set(ctx)) return logged("mevp_advect", MEVP_ESTATE);
  // the element blocks (grouped by geometry kind) cover every element of every domain
  const size_t n = (size_t)ctx->na * ctx->tot_e;
  double *H = const_cast<double *>(ctx->d.H), *A = const_cast<double *>(ctx->d.A);
  double *H1 = ctx->d.adv, *A1 = H1 + n, *H2 = A1 + n, *A2 = H2 + n;
  const double *v = v_buf(ctx, ctx->cur), dt = ctx->params.dt;
  hipStream_t s = ctx->stream;
  const Launch &L = ctx->eblk_split;
  hipError_t e = launch_advect_stage(ctx->d, ctx->na, L, v, H, A, H, A, H1, A1, dt, 0.0, 1.0, s);
  if (e == hipSuccess)
    e = launch_advect_stage(ctx->d, ctx->na, L, v, H, A, H1, A1, H2, A2, dt, 0.75, 0.25, s);
  if (e == hipSuccess)
    e = launch_advect_stage(ctx->d, ctx->na, L, v, H, A, H2, A2, H, A, dt, 1.0 / 3.0, 2.0 / 3.0, s);
  return logged("mevp_advect", hip_status(e));
}

mevp_status mevp_get_fields(mevp_ctx *ctx, int dom, double *H, double *A) {
  if (bad_dom(ctx, dom)) return MEVP_EINVAL;
  const DomDev &D = ctx->dom_h[dom];
  const size_t n = (size_t)ctx->na * D.ne, o = (size_t)ctx->na * D.elem_off;
  mevp_status st = MEVP_OK;
  if (H) st = copy(H, ctx->d.H + o, sizeof(double) * n, ctx->stream);
  if (st == MEVP_OK && A) st = copy(A, ctx->d.A + o, sizeof(double) * n, ctx->stream);
  return st;
}

mevp_status mevp_set_strategy(mevp_ctx *ctx, mevp_strategy strategy) {
  if (!ctx) return MEVP_EINVAL;
  mevp_config c;
  mevp_get_config(ctx, &c);
  c.strategy = strategy;
  return mevp_set_config(ctx, &c);
}

mevp_status mevp_get_config(mevp_ctx *ctx, mevp_config *out) {
  if (!ctx || !out) return MEVP_EINVAL;
  out->strategy = ctx->strategy;
  out->tile_nx = kTileShapes[ctx->shape][0] - 1;
  out->tile_ny = kTileShapes[ctx->shape][1] - 1;
  return MEVP_OK;
}

static mevp_status set_config_impl(mevp_ctx *ctx, const mevp_config *cfg);

mevp_status mevp_set_config(mevp_ctx *ctx, const mevp_config *cfg) {
  const mevp_status st = set_config_impl(ctx, cfg);
  if (st == MEVP_OK)
    mlog(2, "config: %s, tile %dx%d", strategy_name(cfg->strategy), cfg->tile_nx, cfg->tile_ny);
  return logged("mevp_set_config", st);
}

static mevp_status set_config_impl(mevp_ctx *ctx, const mevp_config *cfg) {
  if (!ctx || !cfg) return MEVP_EINVAL;
  if (cfg->strategy != MEVP_STRATEGY_FUSED && cfg->strategy != MEVP_STRATEGY_TWO_PHASE &&
      cfg->strategy != MEVP_STRATEGY_PERSISTENT && cfg->strategy != MEVP_STRATEGY_FUSED_PAIR &&
      cfg->strategy != MEVP_STRATEGY_FUSED_TRIPLE)
    return MEVP_EINVAL;
  int shape = -1;
  for (int sh = 0; sh < kNumTileShapes; ++sh)
    if (kTileShapes[sh][0] - 1 == cfg->tile_nx && kTileShapes[sh][1] - 1 == cfg->tile_ny) shape = sh;
  if (shape < 0 || (shape != 0 && ctx->na != 1)) return MEVP_EINVAL;  // see kTileShapes
  if (cfg->strategy == MEVP_STRATEGY_FUSED_TRIPLE && ctx->na != 1) return MEVP_EINVAL;
  // the bfloat16 trial has the fused kernels only
  if (ctx->prec == MEVP_MIXED_BF16 && (cfg->strategy == MEVP_STRATEGY_TWO_PHASE ||
                                       cfg->strategy == MEVP_STRATEGY_PERSISTENT))
    return MEVP_EINVAL;
  ctx->strategy = static_cast<mevp_strategy>(cfg->strategy);
  graphs_clear(ctx);
  if (shape != ctx->shape) {
    const int old = ctx->shape;
    ctx->shape = shape;
    mevp_status ht = host_guard([&] {
      order_blocks(ctx);
      return MEVP_OK;
    });
    if (ht != MEVP_OK) {
      ctx->shape = old;
      (void)host_guard([&] {
        order_blocks(ctx);
        return MEVP_OK;
      });
      return ht;
    }
    mevp_status st = copy(ctx->tiles_d, ctx->tiles_h.data(), sizeof(Tile) * ctx->tiles_h.size(), ctx->stream);
    if (st == MEVP_OK) st = copy(ctx->eblk_d, ctx->eblk_h.data(), sizeof(Blk) * ctx->eblk_h.size(), ctx->stream);
    // the host tables must outlive the asynchronous copies
    if (st == MEVP_OK) st = hip_status(hipStreamSynchronize(ctx->stream));
    return st;
  }
  return MEVP_OK;
}

// Capture begin-step + n subcycles on the private stream into g (nothing runs).
static mevp_status capture_step(mevp_ctx *ctx, int n, mevp_ctx::StepGraph &g) {
  if (!ctx->cap && hipStreamCreateWithFlags(&ctx->cap, hipStreamNonBlocking) != hipSuccess) {
    ctx->cap = nullptr;
    return MEVP_EDEVICE;
  }
  const int cur0 = ctx->cur;
  if (hipStreamBeginCapture(ctx->cap, hipStreamCaptureModeThreadLocal) != hipSuccess)
    return MEVP_EDEVICE;
  mevp_status st = begin_step_on(ctx, ctx->cap);
  if (st == MEVP_OK) st = subcycles_on(ctx, n, ctx->cap);
  hipGraph_t graph = nullptr;
  const hipError_t e = hipStreamEndCapture(ctx->cap, &graph);
  g.cur_after = ctx->cur;
  ctx->cur = cur0;  // the capture ran nothing
  if (st != MEVP_OK || e != hipSuccess || !graph) {
    if (graph) (void)hipGraphDestroy(graph);
    (void)hipGetLastError();
    return MEVP_EDEVICE;
  }
  hipGraphExec_t exec = nullptr;
  if (hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess) {
    (void)hipGraphDestroy(graph);
    (void)hipGetLastError();
    return MEVP_EDEVICE;
  }
  g.g = graph;
  g.x = exec;
  g.n = n;
  mlog(2, "step: graph captured (start of step + %d subcycles, %s, tile %dx%d)", n,
       strategy_name(ctx->strategy), kTileShapes[ctx->shape][0] - 1, kTileShapes[ctx->shape][1] - 1);
  return MEVP_OK;
}

static mevp_status step_impl(mevp_ctx *ctx, int n_subcycles);

mevp_status mevp_step(mevp_ctx *ctx, int n_subcycles) {
  return logged("mevp_step", step_impl(ctx, n_subcycles));
}

static mevp_status step_impl(mevp_ctx *ctx, int n_subcycles) {
  if (!ctx || n_subcycles < 0) return MEVP_EINVAL;
  if (!inputs_set(ctx)) return MEVP_ESTATE;
  // replay a captured step when nothing needs per-launch events; cooperative
  // launches are not captured
  if (ctx->use_graph && ctx->timer_cap == 0 && ctx->strategy != MEVP_STRATEGY_PERSISTENT) {
    mevp_ctx::StepGraph &g = ctx->graphs[ctx->cur];
    if (g.x && g.n != n_subcycles) {
      (void)hipGraphExecDestroy(g.x);
      (void)hipGraphDestroy(g.g);
      g = mevp_ctx::StepGraph{};
    }
    if (!g.x && capture_step(ctx, n_subcycles, g) != MEVP_OK) {
      ctx->use_graph = false;  // capture unsupported here: launch eagerly from now on
      mlog(1, "step: graph capture failed, launching the kernels directly from now on");
    } else if (g.x) {
      if (hipGraphLaunch(g.x, ctx->stream) != hipSuccess) return MEVP_EDEVICE;
      ctx->cur = g.cur_after;
      return MEVP_OK;
    }
  }
  mevp_status st = begin_step_on(ctx, ctx->stream);
  if (st != MEVP_OK) return st;
  return subcycles_on(ctx, n_subcycles, ctx->stream);
}

mevp_status mevp_set_graph(mevp_ctx *ctx, int enable) {
  if (!ctx) return MEVP_EINVAL;
  graphs_clear(ctx);
  ctx->use_graph = enable != 0;
  return MEVP_OK;
}

mevp_status mevp_sync(mevp_ctx *ctx) {
  if (!ctx) return MEVP_EINVAL;
  return hip_status(hipStreamSynchronize(ctx->stream));
}

static mevp_status read_flag(mevp_ctx *ctx, int *flag) {
  mevp_status st = hip_status(hipMemcpyAsync(flag, ctx->d.flag, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
  if (st == MEVP_OK) st = hip_status(hipStreamSynchronize(ctx->stream));
  return st;
}

mevp_status mevp_check_inputs(mevp_ctx *ctx) {
  if (!ctx) return MEVP_EINVAL;
  hipStream_t s = ctx->stream;
  mevp_status st = hip_status(launch_fill(ctx->d.flag, 1, 0u, s));
  const size_t te = ctx->tot_e, tn = ctx->tot_n;
  if (st == MEVP_OK) st = hip_status(launch_check_finite(ctx->d.vert, 2 * ctx->tot_v, ctx->d.flag, 1, s));
  if (st == MEVP_OK) st = hip_status(launch_check_finite(ctx->d.xnode, 2 * tn, ctx->d.flag, 1, s));
  if (st == MEVP_OK) st = hip_status(launch_check_finite(ctx->d.H, ctx->na * te, ctx->d.flag, 1, s));
  if (st == MEVP_OK) st = hip_status(launch_check_finite(ctx->d.A, ctx->na * te, ctx->d.flag, 1, s));
  if (st == MEVP_OK) st = hip_status(launch_check_finite(ctx->d.wind, 2 * tn, ctx->d.flag, 1, s));
  if (st == MEVP_OK) st = hip_status(launch_check_finite(ctx->d.ocean, 2 * tn, ctx->d.flag, 1, s));
  if (st == MEVP_OK)
    st = hip_status(launch_check_jacobian(ctx->d, ctx->ns, (int)ctx->eblk_h.size(), 2, s));
  int flag = 0;
  if (st == MEVP_OK) st = read_flag(ctx, &flag);
  if (st != MEVP_OK) return logged("mevp_check_inputs", st);
  return logged("mevp_check_inputs", flag ? MEVP_ENONFINITE : MEVP_OK);
}

mevp_status mevp_check_state(mevp_ctx *ctx) {
  if (!ctx) return MEVP_EINVAL;
  hipStream_t s = ctx->stream;
  mevp_status st = hip_status(launch_fill(ctx->d.flag, 1, 0u, s));
  const size_t nS = (size_t)3 * ctx->ns * ctx->tot_e;
  if (st == MEVP_OK) st = hip_status(launch_check_finite(v_buf(ctx, ctx->cur), 2 * ctx->tot_n, ctx->d.flag, 1, s));
  if (st == MEVP_OK) {
    if (ctx->prec == MEVP_FP64)
      st = hip_status(launch_check_finite(static_cast<const double *>(S_buf(ctx, ctx->cur)), nS, ctx->d.flag, 1, s));
    else
      st = hip_status(launch_check_finite_f(static_cast<const float *>(S_buf(ctx, ctx->cur)), nS, ctx->d.flag, 1, s));
  }
  int flag = 0;
  if (st == MEVP_OK) st = read_flag(ctx, &flag);
  if (st != MEVP_OK) return logged("mevp_check_state", st);
  return logged("mevp_check_state", flag ? MEVP_ENONFINITE : MEVP_OK);
}

mevp_status mevp_timing_enable(mevp_ctx *ctx, int max_launches) {
  if (!ctx || max_launches < 0 || max_launches > (1 << 20)) return MEVP_EINVAL;
  mevp_status st = hip_status(hipStreamSynchronize(ctx->stream));
  timer_free(ctx);
  if (st != MEVP_OK || max_launches == 0) return st;
  for (auto &t : ctx->timer) {
    mevp_status ht = host_guard([&] {
      t.ev.assign(2 * (size_t)max_launches, nullptr);
      return MEVP_OK;
    });
    if (ht != MEVP_OK) {
      timer_free(ctx);
      return ht;
    }
    for (auto &e : t.ev)
      if (hipEventCreate(&e) != hipSuccess) {
        timer_free(ctx);
        return MEVP_EDEVICE;
      }
  }
  ctx->timer_cap = max_launches;
  return MEVP_OK;
}

mevp_status mevp_timing_read(mevp_ctx *ctx, int *count, double *total_ms) {
  if (!ctx) return MEVP_EINVAL;
  mevp_status st = hip_status(hipStreamSynchronize(ctx->stream));
  if (st != MEVP_OK) return st;
  for (int ph = 0; ph < 3; ++ph) {
    auto &t = ctx->timer[ph];
    double sum = 0.0;
    for (int i = 0; i < t.used; ++i) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, t.ev[2 * i], t.ev[2 * i + 1]) != hipSuccess) return MEVP_EDEVICE;
      sum += ms;
    }
    if (count) count[ph] = t.used;
    if (total_ms) total_ms[ph] = sum;
    t.used = 0;
  }
  return MEVP_OK;
}

// ---------------------------------------------------------------------------
// Autotuner
// ---------------------------------------------------------------------------
static std::string tune_key(const mevp_ctx *c) {
  long long ne = 0, mx = 0, my = 0;
  for (const auto &d : c->desc) {
    ne += (long long)d.nx * d.ny;
    if (d.nx > mx) mx = d.nx;
    if (d.ny > my) my = d.ny;
  }
  // elements per geometry kind (parallelogram, bilinear, isoparametric)
  long long ek[kNumGeo] = {0, 0, 0};
  for (const auto &D : c->dom_h) ek[D.kind] += D.ne;
  char buf[200];
  snprintf(buf, sizeof buf, "gfx950/%s/ns%d/na%d/dom%d/el%lld/max%lldx%lld/geo%lld.%lld.%lld",
           c->prec == MEVP_MIXED ? "mixed" : c->prec == MEVP_MIXED_BF16 ? "mixed_bf16" : "fp64", c->ns, c->na, c->nd, ne, mx, my, ek[0], ek[1],
           ek[2]);
  return buf;
}

static bool cache_lookup(const char *path, const std::string &key, mevp_config *cfg) {
  FILE *f = path ? fopen(path, "r") : nullptr;
  if (!f) return false;
  char line[512], k[256];
  bool hit = false;
  while (fgets(line, sizeof line, f)) {
    mevp_config c;
    if (sscanf(line, "%255s %d %d %d", k, &c.strategy, &c.tile_nx, &c.tile_ny) == 4 && key == k) {
      *cfg = c;  // the last matching line wins
      hit = true;
    }
  }
  fclose(f);
  return hit;
}

static mevp_status save_state(mevp_ctx *c, std::vector<char> &buf) {
  const size_t vb = sizeof(double) * 2 * c->tot_n, sb = s_words(c) * s_bytes(c);
  buf.resize(vb + sb);
  mevp_status st = hip_status(hipMemcpyAsync(buf.data(), v_buf(c, c->cur), vb, hipMemcpyDeviceToHost, c->stream));
  if (st == MEVP_OK)
    st = hip_status(hipMemcpyAsync(buf.data() + vb, S_buf(c, c->cur), sb, hipMemcpyDeviceToHost, c->stream));
  if (st == MEVP_OK) st = hip_status(hipStreamSynchronize(c->stream));
  return st;
}

static mevp_status restore_state(mevp_ctx *c, const std::vector<char> &buf) {
  const size_t vb = sizeof(double) * 2 * c->tot_n, sb = s_words(c) * s_bytes(c);
  mevp_status st = hip_status(hipMemcpyAsync(v_buf(c, c->cur), buf.data(), vb, hipMemcpyHostToDevice, c->stream));
  if (st == MEVP_OK)
    st = hip_status(hipMemcpyAsync(S_buf(c, c->cur), buf.data() + vb, sb, hipMemcpyHostToDevice, c->stream));
  if (st == MEVP_OK) st = hip_status(hipStreamSynchronize(c->stream));
  return st;
}

static mevp_status tune_impl(mevp_ctx *ctx, int n_trial, const char *cache_path,
                             mevp_config *chosen) {
  if (!ctx || n_trial < 1 || n_trial > 100000) return MEVP_EINVAL;
  if (!inputs_set(ctx)) return MEVP_ESTATE;
  const std::string key = tune_key(ctx);
  mevp_config cfg;
  if (cache_lookup(cache_path, key, &cfg) && mevp_set_config(ctx, &cfg) == MEVP_OK) {
    mlog(1, "tune: %s from the cache: %s, tile %dx%d", key.c_str(), strategy_name(cfg.strategy),
         cfg.tile_nx, cfg.tile_ny);
    if (chosen) *chosen = cfg;
    return MEVP_OK;
  }
  std::vector<mevp_config> cand;
  for (int sh = 0; sh < kNumTileShapes; ++sh) {
    if (sh != 0 && ctx->na != 1) continue;
    cand.push_back(mevp_config{MEVP_STRATEGY_FUSED, kTileShapes[sh][0] - 1, kTileShapes[sh][1] - 1});
    cand.push_back(
        mevp_config{MEVP_STRATEGY_FUSED_PAIR, kTileShapes[sh][0] - 1, kTileShapes[sh][1] - 1});
    if (ctx->na == 1)
      cand.push_back(
          mevp_config{MEVP_STRATEGY_FUSED_TRIPLE, kTileShapes[sh][0] - 1, kTileShapes[sh][1] - 1});
  }
  if (ctx->prec != MEVP_MIXED_BF16)
    cand.push_back(mevp_config{MEVP_STRATEGY_TWO_PHASE, kTileShapes[0][0] - 1, kTileShapes[0][1] - 1});
  // PERSISTENT is not a candidate: on MI355X its grid-wide barrier and static
  // tile assignment cost about 30 us per subcycle over graph-replayed launches
  // of the same tiles, which start a fraction of a microsecond apart, so it
  // never wins (it stays available through mevp_set_config).

  mevp_config before;
  mevp_get_config(ctx, &before);
  const int timer_cap = ctx->timer_cap;
  ctx->timer_cap = 0;  // no per-launch events inside the trials
  mevp_status st = begin_step_on(ctx, ctx->stream);
  std::vector<char> saved, ref, got;
  if (st == MEVP_OK) st = save_state(ctx, saved);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (st == MEVP_OK && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess))
    st = MEVP_EDEVICE;
  float best = 0.f;
  int best_i = -1;
  const int cur0 = ctx->cur;
  for (size_t i = 0; i < cand.size() && st == MEVP_OK; ++i) {
    st = mevp_set_config(ctx, &cand[i]);
    if (st != MEVP_OK) break;
    // warm-up trial (first-use costs), then the timed one, both from the saved state
    for (int rep = 0; rep < 2 && st == MEVP_OK; ++rep) {
      ctx->cur = cur0;
      st = restore_state(ctx, saved);
      if (st != MEVP_OK) break;
      if (rep == 1) st = hip_status(hipEventRecord(e0, ctx->stream));
      if (st == MEVP_OK) st = subcycles_on(ctx, n_trial, ctx->stream);
      if (st == MEVP_OK && rep == 1) st = hip_status(hipEventRecord(e1, ctx->stream));
      if (st == MEVP_OK) st = hip_status(hipStreamSynchronize(ctx->stream));
    }
    float ms = 0.f;
    if (st == MEVP_OK) st = hip_status(hipEventElapsedTime(&ms, e0, e1));
    // every configuration must reproduce the first one bit for bit
    if (st == MEVP_OK) st = save_state(ctx, i == 0 ? ref : got);
    if (st == MEVP_OK && i > 0 && (got.size() != ref.size() || memcmp(got.data(), ref.data(), ref.size()) != 0)) {
      st = MEVP_EINTERNAL;
      mlog(1, "tune: %s, tile %dx%d differs from %s, tile %dx%d after %d subcycles",
           strategy_name(cand[i].strategy), cand[i].tile_nx, cand[i].tile_ny,
           strategy_name(cand[0].strategy), cand[0].tile_nx, cand[0].tile_ny, n_trial);
    }
    if (st == MEVP_OK)
      mlog(1, "tune: %s, tile %dx%d: %.3f ms for %d subcycles", strategy_name(cand[i].strategy),
           cand[i].tile_nx, cand[i].tile_ny, ms, n_trial);
    if (st == MEVP_OK && (best_i < 0 || ms < best)) {
      best = ms;
      best_i = (int)i;
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  // leave the state as it was, with the winner (or the previous config on error)
  ctx->cur = cur0;
  mevp_status rs = saved.empty() ? MEVP_OK : restore_state(ctx, saved);
  ctx->timer_cap = timer_cap;
  mevp_status cs = mevp_set_config(ctx, st == MEVP_OK ? &cand[best_i] : &before);
  if (st != MEVP_OK) return st;
  if (rs != MEVP_OK) return rs;
  if (cs != MEVP_OK) return cs;
  if (chosen) *chosen = cand[best_i];
  mlog(1, "tune: %s: chose %s, tile %dx%d", key.c_str(), strategy_name(cand[best_i].strategy),
       cand[best_i].tile_nx, cand[best_i].tile_ny);
  if (cache_path) {
    FILE *f = fopen(cache_path, "a");
    if (f) {
      fprintf(f, "%s %d %d %d\n", key.c_str(), cand[best_i].strategy, cand[best_i].tile_nx,
              cand[best_i].tile_ny);
      fclose(f);
    }
  }
  return MEVP_OK;
}

mevp_status mevp_tune(mevp_ctx *ctx, int n_trial, const char *cache_path, mevp_config *chosen) {
  return logged("mevp_tune", host_guard([&] { return tune_impl(ctx, n_trial, cache_path, chosen); }));
}

// ---------------------------------------------------------------------------
// mevp_step_static: one time step of one domain with no allocation
// ---------------------------------------------------------------------------
}  // extern "C"

namespace {

// The working memory of mevp_step_static: a file-scope device array, one copy
// per GPU (each device that runs the library holds its own until the process
// ends). Host code never passes the name `scratch` to a kernel or a copy: in
// host code it is a stand-in, not a device address. The array's address on a
// device is asked of HIP once, with that device current (scratch_base), and
// only that address is used.
__device__ __align__(256) unsigned char scratch[MEVP_STATIC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::once_flag g_scratch_once[kMaxDevices];
void *g_scratch_ptr[kMaxDevices];
mevp_status g_scratch_status[kMaxDevices];

// Device address of `scratch` on the current device `dev` (first call per
// device: checks the architecture and looks the address up).
mevp_status scratch_base(int dev, char **out) {
  if (dev < 0 || dev >= kMaxDevices) return MEVP_EDEVICE;
  std::call_once(g_scratch_once[dev], [dev] {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) {
      g_scratch_status[dev] = MEVP_EDEVICE;
      return;
    }
    if (strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
      g_scratch_status[dev] = MEVP_EUNSUPPORTED;
      return;
    }
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      (void)hipGetLastError();
      g_scratch_status[dev] = MEVP_EDEVICE;
      return;
    }
    g_scratch_ptr[dev] = ptr;
    g_scratch_status[dev] = MEVP_OK;
    mlog(1, "step_static: %zu bytes of file-scope scratch on device %d", (size_t)MEVP_STATIC_SCRATCH_BYTES, dev);
  });
  *out = static_cast<char *>(g_scratch_ptr[dev]);
  return g_scratch_status[dev];
}

// Layout of the scratch for one domain: the tables, the check flag, both v
// buffers, the node constants and both S buffers (the inputs are read where
// the caller keeps them).
struct StaticLayout {
  size_t doms, eblk, nblk, tiles, flag, v, nc, S, total;
  int n_eblk, n_nblk, n_tiles;
};

mevp_status plan_static(const mevp_domain_desc *dd, mevp_precision prec, int shape,
                        StaticLayout *L) {
  Layout full;
  mevp_status st = plan(dd, 1, prec, &full);  // validates the descriptor and precision
  if (st != MEVP_OK) return st;
  const size_t ws = (prec == MEVP_FP64) ? sizeof(double) : sizeof(float);
  const int tx = kTileShapes[shape][0] - 1, ty = kTileShapes[shape][1] - 1;
  L->n_eblk = full.n_eblk;
  L->n_nblk = full.n_nblk;
  L->n_tiles = ((dd->nx + tx - 1) / tx) * ((dd->ny + ty - 1) / ty);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = align_up(off + bytes);
    return o;
  };
  L->doms = take(sizeof(DomDev));
  L->eblk = take(sizeof(Blk) * L->n_eblk);
  L->nblk = take(sizeof(Blk) * L->n_nblk);
  L->tiles = take(sizeof(Tile) * L->n_tiles);
  L->flag = take(sizeof(int) * 4);
  L->v = take(sizeof(double) * 4 * full.tot_n);
  L->nc = take(sizeof(double) * 6 * full.tot_n);
  L->S = take(ws * 6 * full.ns * full.tot_e);
  L->total = off;
  return MEVP_OK;
}

bool device_pointer(const void *p) {
  hipPointerAttribute_t attr;
  if (hipPointerGetAttributes(&attr, p) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return attr.type == hipMemoryTypeDevice;
}

mevp_status step_static_impl(const mevp_params *params, mevp_precision precision,
                             const mevp_domain_desc *domain, const double *vertex_xy,
                             const double *H, const double *A, const double *wind_xy,
                             const double *ocean_xy, double *v_xy, double *S, int n_subcycles,
                             void *hip_stream) {
  mevp_status st = validate_params(params);
  if (st != MEVP_OK) return st;
  if (!domain || !vertex_xy || !H || !A || !wind_xy || !ocean_xy || !v_xy || !S ||
      n_subcycles < 0)
    return MEVP_EINVAL;
  // three subcycles per launch on 16 x 16 tiles (two on general cells); with
  // n_a != 1 two per launch on 16 x 14 tiles (the kernels that exist there)
  const int shape = domain->n_a == 1 ? 1 : 0;
  StaticLayout L;
  st = plan_static(domain, precision, shape, &L);
  if (st != MEVP_OK) return st;
  if (L.total > MEVP_STATIC_SCRATCH_BYTES) return MEVP_ENOMEM;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return MEVP_EDEVICE;
  char *base = nullptr;
  st = scratch_base(dev, &base);
  if (st != MEVP_OK) return st;
  // the kernels read the inputs where they are: they must be device memory
  const void *ptrs[] = {vertex_xy, H, A, wind_xy, ocean_xy, v_xy, S};
  for (const void *p : ptrs)
    if (!device_pointer(p) || reinterpret_cast<uintptr_t>(p) % sizeof(double) != 0)
      return MEVP_EINVAL;

  const mevp_domain_desc &dd = *domain;
  DomDev D;
  D.nx = dd.nx;
  D.ny = dd.ny;
  D.ne = dd.nx * dd.ny;
  D.nn = (2 * dd.nx + 1) * (2 * dd.ny + 1);
  D.nv = (dd.nx + 1) * (dd.ny + 1);
  D.elem_off = D.node_off = D.vert_off = 0;
  D.kind = kGeoBilinear;  // until the cells are classified

  // a context on the stack, with no host tables: its vectors stay empty and
  // nothing in it owns memory
  mevp_ctx c;
  c.device = dev;
  c.stream = static_cast<hipStream_t>(hip_stream);
  c.prec = precision;
  c.params = *params;
  c.kp = derive(*params);
  c.nd = 1;
  c.ns = dd.n_s;
  c.na = dd.n_a;
  c.tot_e = (size_t)D.ne;
  c.tot_n = (size_t)D.nn;
  c.tot_v = (size_t)D.nv;
  c.n_nblk = L.n_nblk;
  c.strategy = dd.n_a == 1 ? MEVP_STRATEGY_FUSED_TRIPLE : MEVP_STRATEGY_FUSED_PAIR;
  c.shape = shape;
  c.use_graph = false;
  DevArrays &d = c.d;
  DomDev *doms = reinterpret_cast<DomDev *>(base + L.doms);
  Blk *eblk = reinterpret_cast<Blk *>(base + L.eblk);
  Blk *nblk = reinterpret_cast<Blk *>(base + L.nblk);
  Tile *tiles = reinterpret_cast<Tile *>(base + L.tiles);
  d.doms = doms;
  d.eblk = eblk;
  d.nblk = nblk;
  d.tiles = tiles;
  d.flag = reinterpret_cast<int *>(base + L.flag);
  d.vert = vertex_xy;
  d.xnode = nullptr;  // vertex geometry only
  d.H = H;
  d.A = A;
  d.adv = nullptr;    // no advection
  d.wind = wind_xy;
  d.ocean = ocean_xy;
  d.v = reinterpret_cast<double *>(base + L.v);
  d.nc = reinterpret_cast<double *>(base + L.nc);
  d.S = base + L.S;
  d.fe = nullptr;     // the fused strategies keep element forces in LDS

  hipStream_t s = c.stream;
  const int tx = kTileShapes[shape][0] - 1, ty = kTileShapes[shape][1] - 1;
  // the array keeps the previous call's contents: clear this call's part
  st = hip_status(launch_fill(base + L.flag, (L.total - L.flag) / 4, 0u, s));
  if (st == MEVP_OK)
    st = hip_status(launch_single_tables(D, tx, ty, doms, eblk, L.n_eblk, nblk, L.n_nblk, tiles,
                                         L.n_tiles, s));
  // classify the cells as mevp_set_geometry does (all parallelograms -> the
  // constant-Jacobian kernels), waiting for the one flag
  int *flag = d.flag + 1;
  if (st == MEVP_OK) st = hip_status(launch_fill(flag, 1, 1u, s));
  if (st == MEVP_OK) st = hip_status(launch_cell_shape(d, 0, D.ne, flag, s));
  int aff = 0;
  if (st == MEVP_OK)
    st = hip_status(hipMemcpyAsync(&aff, flag, sizeof(int), hipMemcpyDeviceToHost, s));
  if (st == MEVP_OK) st = hip_status(hipStreamSynchronize(s));
  if (st != MEVP_OK) return st;
  D.kind = aff ? kGeoAffine : kGeoBilinear;
  c.tile_split.n[D.kind] = L.n_tiles;
  c.eblk_split.n[D.kind] = L.n_eblk;
  st = hip_status(launch_single_tables(D, tx, ty, doms, eblk, L.n_eblk, nblk, L.n_nblk, tiles,
                                       L.n_tiles, s));
  // state in, the step, state out
  if (st == MEVP_OK) st = hip_status(launch_interleave2(v_xy, v_buf(&c, 0), (size_t)D.nn, s));
  if (st == MEVP_OK)
    st = hip_status(launch_stress_in(S, S_buf(&c, 0), precision != MEVP_FP64, (size_t)D.ne, c.ns, s));
  if (st == MEVP_OK) st = begin_step_on(&c, s);
  if (st == MEVP_OK) st = subcycles_on(&c, n_subcycles, s);
  if (st == MEVP_OK) st = hip_status(launch_deinterleave2(v_buf(&c, c.cur), v_xy, (size_t)D.nn, s));
  if (st == MEVP_OK)
    st = hip_status(launch_stress_out(S_buf(&c, c.cur), precision != MEVP_FP64, S, (size_t)D.ne, c.ns, s));
  return st;
}

}  // namespace

extern "C" {

mevp_status mevp_step_static(const mevp_params *params, mevp_precision precision,
                             const mevp_domain_desc *domain, const double *vertex_xy,
                             const double *H, const double *A, const double *wind_xy,
                             const double *ocean_xy, double *v_xy, double *S, int n_subcycles,
                             void *hip_stream) {
  return logged("mevp_step_static", host_guard([&] {
    return step_static_impl(params, precision, domain, vertex_xy, H, A, wind_xy, ocean_xy, v_xy,
                            S, n_subcycles, hip_stream);
  }));
}

void mevp_destroy(mevp_ctx *ctx) {
  if (!ctx) return;
  graphs_clear(ctx);
  if (ctx->cap) (void)hipStreamDestroy(ctx->cap);
  timer_free(ctx);
  delete ctx;
}

}  // extern "C"
