// ss_batch.hip -- many independent quenches advanced together.
//
// The paper's production runs are many independent quenches from Poisson
// starts ("Simulations").  One configuration of a few thousand particles fills
// a small part of the device, and its L-BFGS step is a chain of short launches,
// so run one at a time the quenches are bound by launch latency.  Here every
// kernel of a minimiser step is one launch over the blocks of all
// configurations still running: block b of a batched launch executes block
// units[b].idx of configuration units[b].slot's own grid (see BUnit), with the
// same device code as the single-configuration kernels.  Each configuration's
// launch shape comes from the tile table by (d, N, M) alone, so its results are
// the same whatever else is in the batch.
//
// The host enqueues steps a few ahead, reads a per-configuration running word
// gathered into pinned memory, and rebuilds the work lists without the
// configurations it has seen stop (they exit at once until then).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <numeric>
#include <string>
#include <vector>

#include "ss.h"
#include "ss_internal.h"
#include "ss_min.h"
#include "ss_engine.h"

namespace ss {
namespace eng {

size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

int dot_blocks_of(int64_t nv) { return (int)std::max<int64_t>(1, std::min<int64_t>(kDotBlocks, (nv + 1023) / 1024)); }

// minimiser memory of one configuration: g, xt, gt, p, (m + 1) S and Y vectors,
// the state and the dot partials
size_t min_bytes(int64_t nv, int m, int G) {
  const size_t vec = al256(sizeof(double) * 2 * (size_t)nv);
  return vec * (4 + 2 * (size_t)(m + 1)) + al256(sizeof(MinState)) + al256(sizeof(double) * 2 * (2 * m + 2) * G);
}

int setup_slot(ss_ctx* ctx, const ss_problem* p, const ss_min_opts* op, HostSlot* h) {
  int rc = prepare_tiled(ctx, p, &h->pl, &h->c, &h->sc, &h->cb, &h->s2);
  if (rc) return rc;
  if (!min_opts_valid(op)) {
    ctx->last_error = "invalid minimiser options";
    return SS_EINVAL;
  }
  h->prob = *p;
  h->opts = *op;
  h->nv = (int64_t)p->d * p->N;
  // FIRE keeps no (s, y) history: the smallest history layout holds its
  // velocity products (3 of the 2 m + 2 product slots)
  h->m = op->method == 1 ? 1 : op->history;
  h->G = dot_blocks_of(h->nv);
  h->bytes = al256(h->c.total) + min_bytes(h->nv, h->m, h->G);
  const int groups = (h->c.R1 + kTabRun - 1) / kTabRun;
  h->n_table = ((int64_t)p->d * groups * p->N + kThreads - 1) / kThreads;
  h->n_nk = h->sc->nunits;
  h->n_nk2 = h->s2 ? h->pl->t2_ntiles * h->s2->nrows : 0;
  h->n_comb = h->c.combine_blocks;
  h->n_grad = ((p->N + 63) / 64) * h->c.Q;
  h->n_gcomb = (h->nv + kThreads - 1) / kThreads;
  h->n_dots = (int64_t)h->G * (2 * h->m + 2);
  h->n_vec = (h->nv + kThreads - 1) / kThreads;
  h->work = (double)p->M * (double)p->N;
  h->phase = op->precision == 0 ? 1 : 0;
  return SS_OK;
}

int64_t max_units(const HostSlot& h) {
  const int64_t nk = h.s2 ? h.n_nk2 : h.n_nk;
  return h.n_table + nk + h.n_comb + h.n_grad + h.n_gcomb + h.n_dots + h.n_vec;
}

MinParams stage_params(const HostSlot& h, int64_t iters_done) {
  MinParams P = min_params(&h.opts, &h.prob);
  if (h.phase == 0 && h.opts.precision == 2) {
    // the FP64 stage of a staged quench ends at its own floor or its first
    // line-search failure (as in ss_minimize)
    P.s_floor = std::max(h.opts.s_floor, h.opts.fp64_floor);
    P.max_ls_fail = 1;
  }
  P.max_iter = std::max<int64_t>(0, h.opts.max_iter - iters_done);
  return P;
}

// work lists of the configurations in `active` (largest first within every launch)
void build_lists(const std::vector<HostSlot>& hs, std::vector<int> active, std::vector<BUnit>& U,
                 std::vector<int32_t>& list, Lists& L) {
  std::stable_sort(active.begin(), active.end(), [&](int a, int b) { return hs[a].work > hs[b].work; });
  U.clear();
  list.assign(active.begin(), active.end());
  L = Lists();
  L.nlist = (int64_t)list.size();
  auto add = [&](int64_t n_of_slot, int s) {
    for (int64_t i = 0; i < n_of_slot; ++i) U.push_back(BUnit{(int32_t)s, (int32_t)i});
  };
  L.table_off = (int64_t)U.size();
  for (int s : active) {
    add(hs[s].n_table, s);
    L.table_work += (double)hs[s].prob.d * hs[s].c.R1 * hs[s].prob.N;
  }
  L.table_n = (int64_t)U.size() - L.table_off;
  // the pair passes, separately for the configurations in double-double (phase 1)
  // and in FP64 (phase 0)
  for (int ph = 1; ph >= 0; --ph) {
    auto& nkg = ph ? L.nk : L.nk64;
    auto& grg = ph ? L.grad : L.grad64;
    // n(k) pass grouped by (d, LDS tile); d = 2 configurations with a tiled
    // schedule form a group of their own (pt = 0)
    auto tiled = [&](int s) { return hs[s].s2 != nullptr; };
    {
      Lists::Group g{2, 0, 0, (int64_t)U.size(), 0, 0.0};
      for (int s : active)
        if (hs[s].phase == ph && tiled(s)) {
          add(hs[s].n_nk2, s);
          g.pairs += hs[s].work;
        }
      g.n = (int64_t)U.size() - g.off;
      if (g.n > 0) nkg.push_back(g);
    }
    for (int d = 1; d <= 4; ++d)
      for (int pt : {16, 4, 1}) {
        Lists::Group g{d, pt, 0, (int64_t)U.size(), 0, 0.0};
        for (int s : active)
          if (hs[s].phase == ph && !tiled(s) && hs[s].prob.d == d && hs[s].c.pt == pt) {
            add(hs[s].n_nk, s);
            g.R1max = std::max(g.R1max, hs[s].c.R1);
            g.pairs += hs[s].work;
          }
        g.n = (int64_t)U.size() - g.off;
        if (g.n > 0) nkg.push_back(g);
      }
    int64_t& co = ph ? L.comb_off : L.comb64_off;
    int64_t& cn = ph ? L.comb_n : L.comb64_n;
    co = (int64_t)U.size();
    for (int s : active)
      if (hs[s].phase == ph) add(hs[s].n_comb, s);
    cn = (int64_t)U.size() - co;
    for (int d = 1; d <= 4; ++d) {
      Lists::Group g{d, 0, 0, (int64_t)U.size(), 0, 0.0};
      for (int s : active)
        if (hs[s].phase == ph && hs[s].prob.d == d) {
          add(hs[s].n_grad, s);
          g.pairs += hs[s].work;
        }
      g.n = (int64_t)U.size() - g.off;
      if (g.n > 0) grg.push_back(g);
    }
    int64_t& go = ph ? L.gcomb_off : L.gcomb64_off;
    int64_t& gn = ph ? L.gcomb_n : L.gcomb64_n;
    go = (int64_t)U.size();
    for (int s : active)
      if (hs[s].phase == ph) add(hs[s].n_gcomb, s);
    gn = (int64_t)U.size() - go;
  }
  L.dots_off = (int64_t)U.size();
  for (int s : active) add(hs[s].n_dots, s);
  L.dots_n = (int64_t)U.size() - L.dots_off;
  L.vec_off = (int64_t)U.size();
  for (int s : active) add(hs[s].n_vec, s);
  L.vec_n = (int64_t)U.size() - L.vec_off;
}


// device-side header of the batch workspace
struct Header {
  EvalSlot* es;
  MinSlot* ms;
  BUnit* units;
  int32_t* list;
  SlotFlags* flags;
  size_t bytes;
};

// byte offsets of the header parts: es, ms, units, list, flags, end
void header_offsets(int count, int64_t ucap, size_t off[6]) {
  off[0] = 0;
  off[1] = off[0] + al256(sizeof(EvalSlot) * count);
  off[2] = off[1] + al256(sizeof(MinSlot) * count);
  off[3] = off[2] + al256(sizeof(BUnit) * (size_t)std::max<int64_t>(ucap, 1));
  off[4] = off[3] + al256(sizeof(int32_t) * count);
  off[5] = off[4] + al256(sizeof(SlotFlags) * count);
}

Header carve_header(char* base, int count, int64_t ucap) {
  size_t off[6];
  header_offsets(count, ucap, off);
  Header h;
  h.es = (EvalSlot*)(base + off[0]);
  h.ms = (MinSlot*)(base + off[1]);
  h.units = (BUnit*)(base + off[2]);
  h.list = (int32_t*)(base + off[3]);
  h.flags = (SlotFlags*)(base + off[4]);
  h.bytes = off[5];
  return h;
}

void fill_slot(const HostSlot& h, char* mem, double* x, const double* v, EvalSlot* E, MinSlot* C) {
  const LaunchCfg& c = h.c;
  memset(E, 0, sizeof(*E));
  memset(C, 0, sizeof(*C));
  E->d = h.prob.d;
  E->R1 = c.R1;
  E->Q = c.Q;
  E->pt = c.pt;
  E->N = h.prob.N;
  E->M = h.prob.M;
  E->nsegs = h.pl->nsegs;
  E->combine_blocks = c.combine_blocks;
  E->pblocks = (h.prob.N + 63) / 64;
  E->L = h.prob.L;
  E->segs = h.pl->segs;
  E->units = h.sc->units;
  E->rows_of = h.sc->rows_of;
  E->k_of_slot = h.pl->k_of_slot;
  E->runs = h.pl->runs;
  E->chunk_begin = h.cb;
  E->canon_of_lex = h.pl->canon_of_lex;
  E->v = h.prob.vkind == 0 ? nullptr : v;
  E->so = h.pl->slot_off;
  if (h.s2) {
    E->nk2 = 1;
    E->R = h.pl->R;
    E->t2_nrows = h.s2->nrows;
    E->t2_chunk = h.s2->chunk;
    E->t2_tiles = h.pl->t2_tiles;
    E->t2_lexinfo = h.pl->t2_lexinfo;
    E->t2_rows_of = h.s2->rows_of;
    E->t2_ident = h.pl->t2_ident;
  }
  E->tab = (double*)(mem + c.off_tab);
  E->part = (double*)(mem + c.off_part);
  E->csw = (double*)(mem + c.off_csw);
  E->gpart = (double*)(mem + c.off_gpart);
  E->blk = (double*)(mem + c.off_blk);
  // minimiser memory
  const size_t vec = al256(sizeof(double) * 2 * (size_t)h.nv);
  char* p = mem + al256(c.total);
  auto take = [&](size_t n) {
    char* r = p;
    p += n;
    return r;
  };
  VecSet& V = C->V;
  V.x = x;
  V.g = (double*)take(vec);
  V.xt = (double*)take(vec);
  V.gt = (double*)take(vec);
  V.p = (double*)take(vec);
  for (int i = 0; i <= h.m; ++i) V.S[i] = (double*)take(vec);
  for (int i = 0; i <= h.m; ++i) V.Y[i] = (double*)take(vec);
  C->S = (MinState*)take(al256(sizeof(MinState)));
  C->partial = (double*)take(al256(sizeof(double) * 2 * (2 * h.m + 2) * h.G));
  C->P = stage_params(h, 0);
  C->keep = 0;
  C->eblk = E->blk;
  C->neblk = c.combine_blocks;
  C->nv = h.nv;
  C->dot_blocks = h.G;
  E->pos[0] = V.x;
  E->pos[1] = V.xt;
  E->grad[0] = V.g;
  E->grad[1] = V.gt;
  E->phi = C->S->f;
  E->smax = C->S->smax;
  E->running = &C->S->running;
}

hipError_t launch_eval(ss_ctx* ctx, const DevArrays& D, const Lists& L, int which, int gate, hipStream_t st) {
  hipError_t e = timed(ctx, 2, st, L.table_work,
                       [&] { return launch_batch_table(D.es, D.units + L.table_off, L.table_n, which, gate, st); });
  if (e != hipSuccess) return e;
  for (const auto& g : L.nk) {
    e = timed(ctx, 0, st, g.pairs, [&] {
      return g.pt == 0 ? launch_batch_nk2(D.es, D.units + g.off, g.n, gate, st)
                       : launch_batch_nk(g.d, g.pt, g.R1max, D.es, D.units + g.off, g.n, gate, st);
    });
    if (e != hipSuccess) return e;
  }
  e = launch_batch_combine(D.es, D.units + L.comb_off, L.comb_n, gate, st);
  if (e != hipSuccess) return e;
  for (const auto& g : L.grad) {
    e = timed(ctx, 1, st, g.pairs, [&] { return launch_batch_grad(g.d, D.es, D.units + g.off, g.n, gate, st); });
    if (e != hipSuccess) return e;
  }
  e = launch_batch_gcomb(D.es, D.units + L.gcomb_off, L.gcomb_n, which, gate, st);
  if (e != hipSuccess) return e;
  // configurations in their FP64 stage
  for (const auto& g : L.nk64) {
    e = g.pt == 0 ? launch_batch_nk2_64(D.es, D.units + g.off, g.n, gate, st)
                  : launch_batch_nk64(g.d, g.pt, g.R1max, D.es, D.units + g.off, g.n, gate, st);
    if (e != hipSuccess) return e;
  }
  e = launch_batch_combine64(D.es, D.units + L.comb64_off, L.comb64_n, gate, st);
  if (e != hipSuccess) return e;
  for (const auto& g : L.grad64) {
    e = launch_batch_grad64(g.d, D.es, D.units + g.off, g.n, gate, st);
    if (e != hipSuccess) return e;
  }
  return launch_batch_gcomb64(D.es, D.units + L.gcomb64_off, L.gcomb64_n, which, gate, st);
}

hipError_t launch_start(ss_ctx* ctx, const DevArrays& D, const Lists& L, hipStream_t st) {
  hipError_t e = launch_eval(ctx, D, L, 0, 0, st);
  if (e == hipSuccess) e = launch_batch_final(D.es, D.list, L.nlist, st);
  if (e == hipSuccess) e = launch_batch_init(D.ms, D.list, L.nlist, st);
  return e;
}

hipError_t launch_tick(ss_ctx* ctx, const DevArrays& D, const Lists& L, hipStream_t st) {
  hipError_t e = launch_batch_dots(D.ms, D.units + L.dots_off, L.dots_n, 0, st);
  if (e == hipSuccess) e = launch_batch_dots_final(D.ms, D.list, L.nlist, 0, st);
  if (e == hipSuccess) e = launch_batch_step(D.ms, D.units + L.vec_off, L.vec_n, st);
  if (e == hipSuccess) e = launch_eval(ctx, D, L, 1, 1, st);
  if (e == hipSuccess) e = launch_batch_dots(D.ms, D.units + L.dots_off, L.dots_n, 1, st);
  if (e == hipSuccess) e = launch_batch_dots_final(D.ms, D.list, L.nlist, 1, st);
  if (e == hipSuccess) e = launch_batch_accept(D.ms, D.units + L.vec_off, L.vec_n, st);
  if (e == hipSuccess) e = launch_batch_flags(D.ms, D.list, L.nlist, D.flags, st);
  return e;
}

struct Pinned {
  void* p = nullptr;
  ~Pinned() {
    if (p) hipHostFree(p);
  }
};

int setup_all(ss_ctx* ctx, int count, const ss_problem* probs, const ss_min_opts* opts, std::vector<HostSlot>& hs,
              int64_t* ucap, size_t* total) {
  if (!ctx) return SS_EINVAL;
  if (count < 1 || !probs || !opts) {
    ctx->last_error = "count < 1 or NULL problem/option arrays";
    return SS_EINVAL;
  }
  hs.assign(count, HostSlot());
  for (int i = 0; i < count; ++i) {
    int rc = setup_slot(ctx, &probs[i], &opts[i], &hs[i]);
    if (rc) {
      ctx->last_error = "configuration " + std::to_string(i) + ": " + ctx->last_error;
      return rc;
    }
  }
  std::vector<int> all(count);
  std::iota(all.begin(), all.end(), 0);
  std::vector<BUnit> U;
  std::vector<int32_t> list;
  Lists L;
  build_lists(hs, all, U, list, L);
  if ((int64_t)U.size() >= ((int64_t)1 << 31)) {
    ctx->last_error = "batch too large for one launch";
    return SS_EINVAL;
  }
  // a configuration's units depend on its evaluation precision (the tiled and
  // the piece n(k) pass differ): room for the most any of them can take
  int64_t cap = 0;
  for (const HostSlot& h : hs) cap += max_units(h);
  *ucap = std::max<int64_t>(cap, (int64_t)U.size());
  size_t hoff[6];
  header_offsets(count, *ucap, hoff);
  size_t t = hoff[5];
  for (const HostSlot& h : hs) t += h.bytes;
  *total = t;
  return SS_OK;
}

}  // namespace eng
}  // namespace ss

using namespace ss;
using namespace ss::eng;

extern "C" int ss_set_tiles(ss_ctx* ctx, const ss_tile* tiles, int count) {
  if (!ctx || count < 0 || (count > 0 && !tiles)) return SS_EINVAL;
  std::vector<ss_tile_entry> t;
  for (int i = 0; i < count; ++i) {
    const ss_tile& e = tiles[i];
    if (e.d < 0 || e.d > 4 || e.nk_chunk < 1 || e.grad_k < 1 || e.max_N < 1 || e.max_M < 1) {
      ctx->last_error = "invalid tile entry " + std::to_string(i);
      return SS_EINVAL;
    }
    t.push_back(ss_tile_entry{e.d, e.max_N, e.max_M, TileSpec{e.nk_chunk, e.grad_k}});
  }
  std::lock_guard<std::mutex> g(ctx->mu);
  ctx->tiles = t;
  return SS_OK;
}

extern "C" int ss_get_tile(ss_ctx* ctx, const ss_problem* prob, ss_tile* out) {
  if (!ctx || !prob || !out) return SS_EINVAL;
  std::lock_guard<std::mutex> g(ctx->mu);
  const TileSpec t = tile_for(ctx, prob->d, prob->N, prob->M);
  out->d = prob->d;
  out->max_N = prob->N;
  out->max_M = prob->M;
  out->nk_chunk = t.nk_chunk;
  out->grad_k = t.grad_k;
  return SS_OK;
}

extern "C" int ss_batch_workspace_size(ss_ctx* ctx, int count, const ss_problem* probs, const ss_min_opts* opts,
                                       size_t* bytes) {
  if (!ctx || !bytes) return SS_EINVAL;
  std::vector<HostSlot> hs;
  int64_t ucap = 0;
  return setup_all(ctx, count, probs, opts, hs, &ucap, bytes);
}

extern "C" int ss_minimize_batch(ss_ctx* ctx, int count, const ss_problem* probs, const double* const* v_dev,
                                 double* const* pos_dev, const ss_min_opts* opts, ss_min_result* out, void* ws,
                                 size_t ws_bytes, void* stream) {
  if (!ctx) return SS_EINVAL;
  const auto t0 = std::chrono::steady_clock::now();
  std::vector<HostSlot> hs;
  int64_t ucap = 0;
  size_t need = 0;
  int rc = setup_all(ctx, count, probs, opts, hs, &ucap, &need);
  if (rc) return rc;
  if (!pos_dev || !out || !ws) {
    ctx->last_error = "NULL required pointer";
    return SS_EINVAL;
  }
  for (int i = 0; i < count; ++i) {
    if (!pos_dev[i]) {
      ctx->last_error = "pos_dev[" + std::to_string(i) + "] is NULL";
      return SS_EINVAL;
    }
    if (probs[i].vkind != 0 && (!v_dev || !v_dev[i])) {
      ctx->last_error = "configuration " + std::to_string(i) + ": vkind != 0 needs v_dev";
      return SS_EINVAL;
    }
  }
  if (ws_bytes < need) {
    ctx->last_error = "workspace too small";
    return SS_EINVAL;
  }
  hipStream_t st = (hipStream_t)stream;
  char* base = (char*)ws;
  const Header H = carve_header(base, count, ucap);
  std::vector<EvalSlot> es(count);
  std::vector<MinSlot> ms(count);
  {
    size_t off = H.bytes;
    for (int i = 0; i < count; ++i) {
      fill_slot(hs[i], base + off, pos_dev[i], v_dev ? v_dev[i] : nullptr, &es[i], &ms[i]);
      off += hs[i].bytes;
    }
  }
  int err = SS_OK;
  auto ok = [&](hipError_t e, const char* what) {
    if (e != hipSuccess && err == SS_OK) {
      ctx->last_error = std::string(what) + ": " + hipGetErrorString(e);
      err = e == hipErrorOutOfMemory ? SS_ENOMEM : SS_EHIP;
    }
    return err == SS_OK;
  };
  constexpr int kDepth = 3;
  // pinned staging: descriptors, unit lists, flag ring, final states
  const size_t desc_bytes = sizeof(EvalSlot) * count + sizeof(MinSlot) * count;
  const size_t list_bytes = sizeof(BUnit) * (size_t)std::max<int64_t>(ucap, 1) + sizeof(int32_t) * count;
  constexpr int kStages = 4;  // list uploads in flight
  Pinned pin_desc, pin_list[kStages], pin_flags, pin_state;
  if (!ok(hipHostMalloc(&pin_desc.p, desc_bytes, hipHostMallocDefault), "hipHostMalloc")) return err;
  for (auto& pl : pin_list)
    if (!ok(hipHostMalloc(&pl.p, list_bytes, hipHostMallocDefault), "hipHostMalloc")) return err;
  if (!ok(hipHostMalloc(&pin_flags.p, sizeof(SlotFlags) * count * kDepth, hipHostMallocDefault), "hipHostMalloc"))
    return err;
  if (!ok(hipHostMalloc(&pin_state.p, sizeof(MinState) * count, hipHostMallocDefault), "hipHostMalloc")) return err;
  memcpy(pin_desc.p, es.data(), sizeof(EvalSlot) * count);
  memcpy((char*)pin_desc.p + sizeof(EvalSlot) * count, ms.data(), sizeof(MinSlot) * count);
  ok(hipMemcpyAsync(H.es, pin_desc.p, sizeof(EvalSlot) * count, hipMemcpyHostToDevice, st), "descriptor copy");
  ok(hipMemcpyAsync(H.ms, (char*)pin_desc.p + sizeof(EvalSlot) * count, sizeof(MinSlot) * count,
                    hipMemcpyHostToDevice, st),
     "descriptor copy");

  hipEvent_t ev[kDepth] = {}, ev_up[kStages] = {};
  for (int q = 0; q < kDepth && err == SS_OK; ++q) ok(hipEventCreateWithFlags(&ev[q], hipEventDisableTiming), "event");
  for (int q = 0; q < kStages && err == SS_OK; ++q)
    ok(hipEventCreateWithFlags(&ev_up[q], hipEventDisableTiming), "event");
  bool up_pending[kStages] = {};
  int up_next = 0;

  std::vector<BUnit> U;
  std::vector<int32_t> list;
  Lists L;
  const DevArrays D{H.es, H.ms, H.units, H.list, H.flags};
  // work lists go through a ring of pinned staging buffers, each reused once its
  // previous copy has completed; stream order keeps the device copy behind the
  // launches that read the previous lists
  auto upload = [&](const std::vector<int>& active) {
    build_lists(hs, active, U, list, L);
    if ((int64_t)U.size() > ucap) {
      ctx->last_error = "batched work list larger than its buffer";
      err = SS_EHIP;
      return false;
    }
    const int k = up_next;
    up_next = (up_next + 1) % kStages;
    if (up_pending[k] && !ok(hipEventSynchronize(ev_up[k]), "event sync")) return false;
    char* pl = (char*)pin_list[k].p;
    memcpy(pl, U.data(), sizeof(BUnit) * U.size());
    memcpy(pl + sizeof(BUnit) * ucap, list.data(), sizeof(int32_t) * list.size());
    if (!U.empty()) ok(hipMemcpyAsync(H.units, pl, sizeof(BUnit) * U.size(), hipMemcpyHostToDevice, st), "list copy");
    ok(hipMemcpyAsync(H.list, pl + sizeof(BUnit) * ucap, sizeof(int32_t) * list.size(), hipMemcpyHostToDevice, st),
       "list copy");
    ok(hipEventRecord(ev_up[k], st), "event record");
    up_pending[k] = true;
    return err == SS_OK;
  };
  // staged quenches whose FP64 stage has stopped continue in double-double from
  // their positions: new stage parameters (the kept pairs are carried over),
  // the double-double starting evaluation and tests, then back to the lists
  std::vector<int64_t> iters64(count, 0), evals64(count, 0);
  // flags of ticks enqueued before a configuration's switch still show its
  // stopped FP64 stage: they are read only from this tick on
  std::vector<int64_t> valid_from(count, 0);
  int64_t tick = 0;
  MinSlot* ms_pin = (MinSlot*)((char*)pin_desc.p + sizeof(EvalSlot) * count);
  auto switch_to_dd = [&](const std::vector<int>& sw, const std::vector<int>& active_now) {
    for (int s : sw) {
      hs[s].phase = 1;
      valid_from[s] = tick;
      ms_pin[s].P = stage_params(hs[s], iters64[s]);
      ms_pin[s].keep = 1;
      // the previous copy from this cell finished before the first step ran
      if (!ok(hipMemcpyAsync(H.ms + s, ms_pin + s, sizeof(MinSlot), hipMemcpyHostToDevice, st), "descriptor copy"))
        return false;
    }
    if (!upload(sw) || !ok(launch_start(ctx, D, L, st), "batched restart")) return false;
    return upload(active_now);
  };
  std::vector<int> active(count);
  std::iota(active.begin(), active.end(), 0);
  std::vector<double> t_stop(count, -1.0);
  // the starting evaluation and the first tests of every configuration
  if (upload(active)) ok(launch_start(ctx, D, L, st), "batched start");
  double last_print = 0.0;
  while (err == SS_OK) {
    if (!ok(launch_tick(ctx, D, L, st), "batched step")) break;
    const int q = (int)(tick % kDepth);
    SlotFlags* hf = (SlotFlags*)pin_flags.p + (size_t)q * count;
    if (!ok(hipMemcpyAsync(hf, H.flags, sizeof(SlotFlags) * count, hipMemcpyDeviceToHost, st), "flag copy")) break;
    if (!ok(hipEventRecord(ev[q], st), "event record")) break;
    ++tick;
    if (tick < kDepth) continue;
    const int w = (int)(tick % kDepth);  // the oldest step in flight
    if (!ok(hipEventSynchronize(ev[w]), "event sync")) break;
    const SlotFlags* f = (SlotFlags*)pin_flags.p + (size_t)w * count;
    // the flags of step tick - kDepth cover the configurations listed then,
    // which include every configuration listed now
    std::vector<int> still, sw;
    const double now = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    const int64_t seen = tick - kDepth;  // the tick these flags come from
    for (int s : active) {
      if (f[s].running || seen < valid_from[s]) {
        still.push_back(s);
      } else if (hs[s].phase == 0 && hs[s].opts.precision == 2 && f[s].status != 3) {
        iters64[s] = f[s].iter;  // the FP64 stage's totals
        evals64[s] = f[s].evals;
        sw.push_back(s);
        still.push_back(s);
      } else if (t_stop[s] < 0.0) {
        t_stop[s] = now;
      }
    }
    if (ctx->progress_interval > 0.0 && now - last_print >= ctx->progress_interval) {
      fprintf(stderr, "[ss_minimize_batch] step %lld: %zu of %d configurations running, t %.1fs\n",
              (long long)tick, still.size(), count, now);
      fflush(stderr);
      last_print = now;
    }
    if (still.empty()) break;
    if (!sw.empty()) {
      active = still;
      if (!switch_to_dd(sw, active)) break;
    } else if (still.size() < active.size()) {
      active = still;
      if (!upload(active)) break;
    }
  }
  ok(hipStreamSynchronize(st), "final sync");
  if (err == SS_OK) {
    for (int i = 0; i < count; ++i)
      ok(hipMemcpyAsync((MinState*)pin_state.p + i, ms[i].S, sizeof(MinState), hipMemcpyDeviceToHost, st),
         "state copy");
    ok(hipStreamSynchronize(st), "state sync");
  }
  for (int q = 0; q < kDepth; ++q)
    if (ev[q]) hipEventDestroy(ev[q]);
  for (int q = 0; q < kStages; ++q)
    if (ev_up[q]) hipEventDestroy(ev_up[q]);
  if (err != SS_OK) return err;
  const double end = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  for (int i = 0; i < count; ++i) {
    const MinState& hs_ = ((MinState*)pin_state.p)[i];
    out[i].status = hs_.status;
    out[i].iters = hs_.iter + iters64[i];
    out[i].evals = hs_.evals + evals64[i];
    out[i].grad_evals = out[i].evals;
    out[i].phi[0] = hs_.f[0];
    out[i].phi[1] = hs_.f[1];
    out[i].smax[0] = hs_.smax[0];
    out[i].smax[1] = hs_.smax[1];
    out[i].seconds = t_stop[i] >= 0.0 ? t_stop[i] : end;
    // FP64-only quenches never switch: all their iterations are FP64
    const bool all64 = hs[i].opts.precision == 1;
    out[i].iters_fp64 = all64 ? hs_.iter : iters64[i];
    out[i].evals_fp64 = all64 ? hs_.evals : evals64[i];
  }
  return SS_OK;
}
