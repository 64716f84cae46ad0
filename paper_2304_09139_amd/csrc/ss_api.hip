// ss_api.hip -- the C interface (include/ss.h): contexts, wavevector plans,
// launch shapes, workspace layout and the energy/gradient driver.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "ss.h"
#include "ss_internal.h"

namespace ss {
hipError_t launch_table(const double* pos, int d, int64_t N, int R1, double* tab, hipStream_t st,
                        const int* active);
hipError_t launch_nk(const LaunchCfg& c, const Span* segs, int64_t nseg, const NkUnit* units, int64_t nunits,
                     const double* tab, double* part, const SlotOffsets& so, hipStream_t st, const int* active);
hipError_t launch_nk_combine(const LaunchCfg& c, const double* part, const int32_t* rows_of,
                             const int32_t* k_of_slot, const int32_t* canon_of_lex, const double* v, double* nk_out,
                             double* csw, double* blk, hipStream_t st, const int* active);
hipError_t launch_final(const LaunchCfg& c, const double* blk, double* phi, double* smax, double* kmax, hipStream_t st,
                        const int* active);
hipError_t launch_nk64(const LaunchCfg& c, const Span* segs, int64_t nseg, const NkUnit* units, int64_t nunits,
                       const double* tab, double* part, const SlotOffsets& so, hipStream_t st, const int* active);
hipError_t launch_nk_combine64(const LaunchCfg& c, const double* part, const int32_t* rows_of,
                               const int32_t* k_of_slot, const int32_t* canon_of_lex, const double* v,
                               double* nk_out, double* csw, double* blk, hipStream_t st, const int* active);
hipError_t launch_grad64(const LaunchCfg& c, const Span* runs, const int32_t* chunk_begin, const double* tab,
                         const double* csw, double* gpart, hipStream_t st, const int* active);
hipError_t launch_grad_combine64(const LaunchCfg& c, const double* gpart, double L, bool times_L, double* grad,
                                 hipStream_t st, const int* active);
hipError_t launch_grad(const LaunchCfg& c, const Span* runs, const int32_t* chunk_begin, const double* tab,
                       const double* csw, double* gpart, hipStream_t st, const int* active);
hipError_t launch_grad_combine(const LaunchCfg& c, const double* gpart, double L, double* grad, hipStream_t st,
                               const int* active);
hipError_t launch_weights(const int32_t* n, int64_t M, int d, int64_t R2, int vkind, double* v, hipStream_t st);
hipError_t enumerate(int d, int64_t R2, int R, hipStream_t st, Plan* pl);
size_t minimize_extra_bytes(int64_t nv);
int grad_blocks_per_cu(int d);
int nk_blocks_per_cu(int d, int pt, int R1);
int nk2_blocks_per_cu();
hipError_t launch_nk2(const int32_t* tiles, int64_t ntiles, const int32_t* lexinfo, int R, const double* tab,
                      int64_t N, int R1, int64_t chunk, int nrows, double* part, int64_t M, hipStream_t st,
                      const int* active);
hipError_t launch_nk2_64(const int32_t* tiles, int64_t ntiles, const int32_t* lexinfo, int R, const double* tab,
                         int64_t N, int R1, int64_t chunk, int nrows, double* part, int64_t M, hipStream_t st,
                         const int* active);
}  // namespace ss

using namespace ss;

namespace {

// Set while the allocation-free entry point runs on this thread: the plan,
// schedule and chunk-bound builders, which allocate device memory on first use,
// refuse instead (the problem must have been prepared by ss_workspace_size).
thread_local bool tl_no_alloc = false;

struct NoAllocScope {
  NoAllocScope() { tl_no_alloc = true; }
  ~NoAllocScope() { tl_no_alloc = false; }
};

// Workspace of ss_energy_grad_static: one static device array per GPU, held
// until the process ends.  Host code never passes `scratch` itself to a kernel
// (in host code the name is a host-side stand-in, not a device address); it
// uses the device address hipGetSymbolAddress gives for each device, looked up
// once per device at ss_create.
constexpr size_t kScratchBytes = (size_t)32 << 20;
static __device__ __align__(256) char scratch[kScratchBytes];

std::mutex g_scratch_mu;
std::map<int, void*> g_scratch_addr;  // device -> address of that device's `scratch`

// the current device's `scratch` address (the device must be current)
int scratch_address(int device, void** out) {
  std::lock_guard<std::mutex> g(g_scratch_mu);
  auto it = g_scratch_addr.find(device);
  if (it == g_scratch_addr.end()) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return SS_EHIP;
    it = g_scratch_addr.emplace(device, p).first;
  }
  *out = it->second;
  return SS_OK;
}

int refuse_alloc(ss_ctx* c, const char* what) {
  c->last_error = std::string(what) + " of this problem has not been built: call ss_workspace_size for it "
                  "before ss_energy_grad_static";
  return SS_ESTATE;
}

int set_err(ss_ctx* c, int code, const std::string& msg) {
  if (c) c->last_error = msg;
  return code;
}

int hip_err(ss_ctx* c, hipError_t e, const char* where) {
  std::string m = std::string(where) + ": " + hipGetErrorString(e);
  return set_err(c, e == hipErrorOutOfMemory ? SS_ENOMEM : SS_EHIP, m);
}

#define SS_HIP(ctx, call)                                   \
  do {                                                      \
    hipError_t e_ = (call);                                 \
    if (e_ != hipSuccess) return hip_err((ctx), e_, #call); \
  } while (0)

int64_t isqrt64(int64_t x) {
  int64_t r = (int64_t)sqrt((double)x);
  while (r * r > x) --r;
  while ((r + 1) * (r + 1) <= x) ++r;
  return r;
}

// |H(R2)| by columns: for each prefix p = (n_1..n_{d-1}) with |p|^2 <= R2 the last
// component ranges over |n_d| <= r = isqrt(R2 - |p|^2); the half-set rule keeps all
// of them when the first nonzero prefix component is positive, none when it is
// negative, and n_d in 1..r when the prefix is zero.
int64_t count_half(int d, int64_t R2) {
  const int64_t R = isqrt64(R2);
  if (d == 1) return R;
  int64_t total = 0;
  int64_t p[3] = {-R, -R, -R};
  const int np = d - 1;
  for (;;) {
    int64_t s = 0;
    int first = 0;
    for (int a = 0; a < np; ++a) {
      s += p[a] * p[a];
      if (!first && p[a] != 0) first = p[a] > 0 ? 1 : -1;
    }
    if (s <= R2) {
      const int64_t r = isqrt64(R2 - s);
      if (first > 0) total += 2 * r + 1;
      else if (first == 0) total += r;
    }
    int a = np - 1;
    while (a >= 0 && p[a] == R) p[a--] = -R;
    if (a < 0) break;
    ++p[a];
  }
  return total;
}

// Release a plan's device lists and schedules (every pointer may be null).
void free_plan(Plan* pl) {
  if (!pl) return;
  (void)hipFree(pl->lex_n);
  (void)hipFree(pl->canon_n);
  (void)hipFree(pl->canon_of_lex);
  (void)hipFree(pl->runs);
  (void)hipFree(pl->segs);
  (void)hipFree(pl->k_of_slot);
  for (auto& cb : pl->chunk_begin) (void)hipFree(cb.second);
  for (auto& ns : pl->nk_fixed) {
    (void)hipFree(ns.second.units);
    (void)hipFree(ns.second.rows_of);
  }
  for (auto& ns : pl->nk_sched) {
    (void)hipFree(ns.second.units);
    (void)hipFree(ns.second.rows_of);
  }
  (void)hipFree(pl->t2_tiles);
  (void)hipFree(pl->t2_lexinfo);
  (void)hipFree(pl->t2_ident);
  for (auto& ns : pl->nk2_sched) (void)hipFree(ns.second.rows_of);
  for (auto& ns : pl->nk2_fixed) (void)hipFree(ns.second.rows_of);
  delete pl;
}

int build_plan_lists(ss_ctx* ctx, Plan* pl);

// The plan of (d, R2), built and cached on first use.  On failure nothing is
// cached and everything allocated for it is released.
int build_plan(ss_ctx* ctx, int d, int64_t R2, Plan** out) {
  auto key = std::make_pair(d, R2);
  auto it = ctx->plans.find(key);
  if (it != ctx->plans.end()) {
    *out = it->second;
    return SS_OK;
  }
  if (tl_no_alloc) return refuse_alloc(ctx, "the wavevector plan");
  Plan* pl = new (std::nothrow) Plan();
  if (!pl) return set_err(ctx, SS_ENOMEM, "plan allocation");
  pl->d = d;
  pl->R2 = R2;
  pl->R = (int)isqrt64(R2);
  const int rc = build_plan_lists(ctx, pl);
  if (rc != SS_OK) {
    free_plan(pl);
    return rc;
  }
  ctx->plans[key] = pl;
  *out = pl;
  return SS_OK;
}

int build_plan_lists(ss_ctx* ctx, Plan* pl) {
  const int d = pl->d;
  const int64_t R2 = pl->R2;
  SS_HIP(ctx, enumerate(d, R2, pl->R, ctx->build_stream, pl));
  const int64_t M = pl->M;
  std::vector<int32_t> lex((size_t)M * d);
  SS_HIP(ctx, hipMemcpy(lex.data(), pl->lex_n, sizeof(int32_t) * M * d, hipMemcpyDeviceToHost));
  // runs along the last axis (maximal lexicographic stretches with equal prefix)
  std::vector<Span> runs;
  for (int64_t k = 0; k < M; ++k) {
    bool same = !runs.empty();
    if (same)
      for (int a = 0; a < d - 1; ++a)
        if (lex[k * d + a] != lex[(k - 1) * d + a]) same = false;
    if (same && lex[k * d + d - 1] != lex[(k - 1) * d + d - 1] + 1) same = false;
    if (same) {
      runs.back().len++;
    } else {
      Span s{};
      s.k0 = (int32_t)k;
      s.len = 1;
      for (int a = 0; a < d; ++a) s.n[a] = (int16_t)lex[k * d + a];
      runs.push_back(s);
    }
  }
  // pieces of the n(k) pass (see nk_body): a run with a nonzero prefix is a
  // symmetric column, last component -h .. h, and its pieces take exponents
  // t0 .. t0 + L - 1 of 0 .. h with their negatives (2L stored wavevectors, 2L - 1
  // for t0 = 0); the prefix-zero run (0, .., 0, t), t = 1 .. R, takes t alone.
  // At most kSegLen / 2 exponents per piece, balanced within a run.  A piece's k0
  // is the walk position that last component 0 has (or would have) in its run,
  // so that the wavevector with last component x sits at k0 + x.
  constexpr int kMaxT = kSegLen / 2;
  std::vector<Span> segs;
  for (const Span& r : runs) {
    bool plus = true;
    for (int a = 0; a < d - 1; ++a) plus = plus && r.n[a] == 0;
    const int first = r.n[d - 1];
    const int t_lo = plus ? first : 0;
    const int T = plus ? r.len : -first + 1;  // exponents of the run
    if (!plus && r.len != 2 * T - 1) return set_err(ctx, SS_EHIP, "a column of the half set is not symmetric");
    const int pieces = (T + kMaxT - 1) / kMaxT;
    const int base = T / pieces, extra = T % pieces;
    int off = 0;
    for (int i = 0; i < pieces; ++i) {
      Span s = r;
      const int L = base + (i < extra ? 1 : 0);
      s.k0 = r.k0 - first;
      s.n[d - 1] = (int16_t)(t_lo + off);
      s.len = plus ? L : (t_lo + off == 0 ? 2 * L - 1 : 2 * L);
      off += L;
      segs.push_back(s);
    }
  }
  std::stable_sort(segs.begin(), segs.end(), [](const Span& a, const Span& b) { return a.len > b.len; });
  for (size_t b = 0; b < segs.size(); b += kNkPieces) pl->block_maxlen.push_back(segs[b].len);
  pl->nruns = (int64_t)runs.size();
  pl->nsegs = (int64_t)segs.size();
  pl->seg_host = segs;
  // slot order of the n(k) partials (see SlotOffsets)
  {
    int64_t cnt[kSegLen] = {};
    for (const Span& sg : segs)
      for (int t = 0; t < sg.len; ++t) ++cnt[t];
    int64_t acc = 0;
    for (int t = 0; t < kSegLen; ++t) {
      pl->slot_off.off[t] = (int32_t)acc;
      acc += cnt[t];
    }
    if (acc != M) return set_err(ctx, SS_EHIP, "piece slots do not cover the wavevectors");
    std::vector<int32_t> kos((size_t)M, -1);
    for (size_t q = 0; q < segs.size(); ++q) {
      const Span& sg = segs[q];
      bool plus = true;
      for (int a = 0; a < d - 1; ++a) plus = plus && sg.n[a] == 0;
      const int t0 = sg.n[d - 1];
      for (int t = 0; t < sg.len; ++t) {
        if ((int64_t)q >= cnt[t]) return set_err(ctx, SS_EHIP, "pieces are not sorted by length");
        // stored index t -> accumulator acc (nk_body) -> last component x
        const int acc = plus ? 2 * t : (t0 == 0 && t >= 1 ? t + 1 : t);
        const int x = acc % 2 == 0 ? t0 + acc / 2 : -(t0 + acc / 2);
        const int64_t k = (int64_t)sg.k0 + x;
        if (k < 0 || k >= M || kos[pl->slot_off.off[t] + q] != -1)
          return set_err(ctx, SS_EHIP, "piece slots do not map onto the wavevectors");
        kos[pl->slot_off.off[t] + q] = (int32_t)k;
      }
    }
    {
      std::vector<char> seen((size_t)M, 0);
      for (int32_t k : kos) {
        if (k < 0 || seen[k]) return set_err(ctx, SS_EHIP, "piece slots do not map onto the wavevectors");
        seen[k] = 1;
      }
    }
    SS_HIP(ctx, hipMalloc(&pl->k_of_slot, sizeof(int32_t) * M));
    SS_HIP(ctx, hipMemcpy(pl->k_of_slot, kos.data(), sizeof(int32_t) * M, hipMemcpyHostToDevice));
  }
  SS_HIP(ctx, hipMalloc(&pl->runs, sizeof(Span) * runs.size()));
  SS_HIP(ctx, hipMalloc(&pl->segs, sizeof(Span) * segs.size()));
  SS_HIP(ctx, hipMemcpy(pl->runs, runs.data(), sizeof(Span) * runs.size(), hipMemcpyHostToDevice));
  SS_HIP(ctx, hipMemcpy(pl->segs, segs.data(), sizeof(Span) * segs.size(), hipMemcpyHostToDevice));
  pl->run_len_prefix.assign(runs.size() + 1, 0);
  for (size_t r = 0; r < runs.size(); ++r) pl->run_len_prefix[r + 1] = pl->run_len_prefix[r] + runs[r].len;
  if (d == 2 && pl->R >= kNk2SmallR) {
    // rows n0 = 0 .. R of H: walk positions off .. off + hi - lo hold n1 = lo .. hi
    const int R = pl->R;
    std::vector<int32_t> info((size_t)3 * (R + 1), 0);
    for (int n0 = 0; n0 <= R; ++n0) {
      info[3 * n0] = 0;
      info[3 * n0 + 1] = 1;
      info[3 * n0 + 2] = 0;  // empty unless found below
    }
    for (int64_t k = 0; k < M; ++k) {
      const int n0 = lex[2 * k], n1 = lex[2 * k + 1];
      if (n0 < 0 || n0 > R) return set_err(ctx, SS_EHIP, "wavevector outside the half space");
      if (k == 0 || lex[2 * (k - 1)] != n0) {
        info[3 * n0] = (int32_t)k;
        info[3 * n0 + 1] = n1;
      } else if (n1 != lex[2 * (k - 1) + 1] + 1) {
        return set_err(ctx, SS_EHIP, "rows of H are not intervals in walk order");
      }
      info[3 * n0 + 2] = n1;
    }
    std::vector<int32_t> tiles;
    for (int a0 = 0; a0 <= R; a0 += 16)
      for (int b0 = -R; b0 <= R; b0 += 16) {
        bool meets = false;
        for (int n0 = a0; n0 < a0 + 16 && n0 <= R && !meets; ++n0)
          meets = info[3 * n0 + 1] <= info[3 * n0 + 2] && info[3 * n0 + 1] <= b0 + 15 && info[3 * n0 + 2] >= b0;
        if (meets) {
          tiles.push_back(a0);
          tiles.push_back(b0);
        }
      }
    std::vector<int32_t> ident((size_t)M);
    for (int64_t k = 0; k < M; ++k) ident[k] = (int32_t)k;
    pl->t2_ntiles = (int64_t)tiles.size() / 2;
    SS_HIP(ctx, hipMalloc(&pl->t2_tiles, sizeof(int32_t) * tiles.size()));
    SS_HIP(ctx, hipMalloc(&pl->t2_lexinfo, sizeof(int32_t) * info.size()));
    SS_HIP(ctx, hipMalloc(&pl->t2_ident, sizeof(int32_t) * M));
    SS_HIP(ctx, hipMemcpy(pl->t2_tiles, tiles.data(), sizeof(int32_t) * tiles.size(), hipMemcpyHostToDevice));
    SS_HIP(ctx, hipMemcpy(pl->t2_lexinfo, info.data(), sizeof(int32_t) * info.size(), hipMemcpyHostToDevice));
    SS_HIP(ctx, hipMemcpy(pl->t2_ident, ident.data(), sizeof(int32_t) * M, hipMemcpyHostToDevice));
  }
  return SS_OK;
}

// wavevector chunks of about equal pair count for the gradient pass
int chunk_bounds(ss_ctx* ctx, Plan* pl, int Q, int32_t** out) {
  auto it = pl->chunk_begin.find(Q);
  if (it != pl->chunk_begin.end()) {
    *out = it->second;
    return SS_OK;
  }
  if (tl_no_alloc) return refuse_alloc(ctx, "the gradient chunk bounds");
  std::vector<int32_t> b(Q + 1);
  const int64_t total = pl->run_len_prefix.back();
  size_t r = 0;
  for (int q = 0; q <= Q; ++q) {
    const int64_t target = (total * q) / Q;
    while (r < pl->run_len_prefix.size() - 1 && pl->run_len_prefix[r] < target) ++r;
    b[q] = (int32_t)r;
  }
  b[Q] = (int32_t)pl->nruns;
  int32_t* dev = nullptr;
  SS_HIP(ctx, hipMalloc(&dev, sizeof(int32_t) * (Q + 1)));
  SS_HIP(ctx, hipMemcpy(dev, b.data(), sizeof(int32_t) * (Q + 1), hipMemcpyHostToDevice));
  pl->chunk_begin[Q] = dev;
  *out = dev;
  return SS_OK;
}

// Grids are sized in whole "rounds" of resident blocks (blocks per CU x CUs) so
// that the last round is not left mostly idle.
int num_cus(ss_ctx* ctx) {
  static int cached = 0;
  if (!cached) {
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, ctx->device) != hipSuccess || n <= 0) n = 256;
    cached = n;
  }
  return cached;
}

// Work split into `per` blocks per step, at most max_steps steps: the step count
// whose block total fills its last round of `capacity` resident blocks best,
// trying 1..rounds rounds (stops at the first that is at least 90% full).
int64_t rounds_fit(int64_t capacity, int64_t per, int64_t max_steps, int rounds) {
  int64_t best = 1;
  double best_eff = -1.0;
  for (int r = 1; r <= rounds; ++r) {
    const int64_t steps = std::max<int64_t>(1, std::min<int64_t>(max_steps, (capacity * r) / per));
    const int64_t blocks = steps * per;
    const int64_t full = (blocks + capacity - 1) / capacity;
    const double eff = (double)blocks / (double)(full * capacity);
    if (eff > best_eff + 0.05 || (r == 1 && eff >= 0.9)) {
      best_eff = eff;
      best = steps;
      if (eff >= 0.9) break;
    }
  }
  return best;
}

// XCD-aware launch order of the n(k) units.  Workgroups go to the kXcds XCDs
// round-robin by linear index, and every unit stages the table rows of its
// particle range.  The units sorted by first particle are cut into kXcds runs of
// equal count; run x is dealt to grid positions x, x + kXcds, ... so XCD x
// works through particles [x N / kXcds, (x + 1) N / kXcds) in order: the units
// running together on one XCD share particle ranges, and their table rows come
// from that XCD's L2 instead of once per piece block from memory.  Only the
// launch order changes (results are the same bits).
std::vector<NkUnit> xcd_order(std::vector<NkUnit> units) {
  const size_t n = units.size();
  if (n < 2 * (size_t)kXcds) return units;
  std::stable_sort(units.begin(), units.end(), [](const NkUnit& a, const NkUnit& b) {
    return a.j0 != b.j0 ? a.j0 < b.j0 : a.block < b.block;
  });
  std::vector<NkUnit> out(n);
  const size_t per = (n + kXcds - 1) / kXcds;  // units per XCD run (the last run may be shorter)
  size_t pos = 0;
  // position k * kXcds + x takes unit k of run x while every run has one;
  // the units left after the shortest run ends fill the remaining positions in order
  std::vector<size_t> next(kXcds);
  for (int x = 0; x < kXcds; ++x) next[x] = std::min(n, x * per);
  for (size_t k = 0; pos < n; ++k)
    for (int x = 0; x < kXcds && pos < n; ++x) {
      const size_t end = std::min(n, (x + 1) * per);
      if (next[x] < end) out[pos++] = units[next[x]++];
    }
  return out;
}

// n(k) pass schedule for N particles: exactly 2 .. kNkRounds rounds of resident
// blocks in total (the most that leave at least kNkMinChunk particles per unit;
// fewer units only when N is small), apportioned over the piece blocks
// in proportion to their work per particle (longest piece + base cost), so that
// every unit costs about the same and the last round is as full as the first; the
// P_b particle ranges of block b split [0, N) as evenly as integers allow (their
// edges need not fall on the LDS tile of pt particles: a unit's last tile is
// partial).  Wavevectors of block b then have P_b partial rows.  Depends only
// on (d, R2, N) and the device.
int nk_schedule(ss_ctx* ctx, Plan* pl, int64_t N, int pt, Plan::NkSched** out) {
  auto it = pl->nk_sched.find(N);
  if (it != pl->nk_sched.end()) {
    *out = &it->second;
    return SS_OK;
  }
  if (tl_no_alloc) return refuse_alloc(ctx, "the n(k) schedule");
  const size_t nb = pl->block_maxlen.size();
  // rounds: the most (2 .. kNkRounds) that keep at least kNkMinChunk particles
  // per unit on average -- more rounds balance the units' ends better, but every
  // round adds partial rows that the combine pass reads back (d=3, N=8000: 3
  // rounds cost more in the combine than they save in the n(k) pass; N=30000:
  // 3 save 4% against 2; N=60000: 4 save 2.6% against 3)
  const int64_t cap = (int64_t)num_cus(ctx) * nk_blocks_per_cu(pl->d, pt, pl->R + 1);
  int rounds = kNkRounds;
  while (rounds > 2 && N * (int64_t)nb < kNkMinChunk * rounds * cap) --rounds;
  const int64_t target = rounds * cap;
  const int64_t maxP = std::max<int64_t>(1, (N + pt - 1) / pt);  // at least pt particles per unit
  double wsum = 0.0;
  for (int L : pl->block_maxlen) wsum += L + 1.5;
  // largest-remainder apportionment of the target over the blocks
  std::vector<int64_t> P(nb);
  std::vector<std::pair<double, size_t>> rem;
  int64_t given = 0;
  for (size_t b = 0; b < nb; ++b) {
    const double share = (double)target * (pl->block_maxlen[b] + 1.5) / wsum;
    P[b] = std::max<int64_t>(1, std::min<int64_t>(maxP, (int64_t)share));
    given += P[b];
    rem.push_back({share - (double)(int64_t)share, b});
  }
  std::stable_sort(rem.begin(), rem.end(), [](const auto& x, const auto& y) { return x.first > y.first; });
  for (size_t q = 0; given < target && q < rem.size(); ++q)
    if (P[rem[q].second] < maxP) {
      P[rem[q].second] += 1;
      ++given;
    }
  std::vector<NkUnit> units;
  std::vector<int32_t> rows_of(pl->M, 1);
  int64_t maxrows = 1;
  for (size_t b = 0; b < nb; ++b) {
    const int64_t Pb = P[b];
    for (int64_t r = 0; r < Pb; ++r) {
      NkUnit u;
      u.block = (int32_t)b;
      u.row = (int32_t)r;
      u.j0 = (int32_t)(r * N / Pb);
      u.j1 = (int32_t)((r + 1) * N / Pb);
      units.push_back(u);
    }
    maxrows = std::max(maxrows, Pb);
    const size_t s0 = b * kNkPieces, s1 = std::min(pl->seg_host.size(), s0 + kNkPieces);
    for (size_t q = s0; q < s1; ++q)
      for (int t = 0; t < pl->seg_host[q].len; ++t) rows_of[pl->slot_off.off[t] + q] = (int32_t)Pb;
  }
  units = xcd_order(std::move(units));
  Plan::NkSched sc;
  sc.nunits = (int64_t)units.size();
  sc.rows = maxrows;
  SS_HIP(ctx, hipMalloc(&sc.units, sizeof(NkUnit) * units.size()));
  SS_HIP(ctx, hipMalloc(&sc.rows_of, sizeof(int32_t) * rows_of.size()));
  SS_HIP(ctx, hipMemcpy(sc.units, units.data(), sizeof(NkUnit) * units.size(), hipMemcpyHostToDevice));
  SS_HIP(ctx, hipMemcpy(sc.rows_of, rows_of.data(), sizeof(int32_t) * rows_of.size(), hipMemcpyHostToDevice));
  pl->nk_sched[N] = sc;
  *out = &pl->nk_sched[N];
  return SS_OK;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// fixed-chunk n(k) schedule of the batched launches: every piece block gets
// ceil(N / chunk) particle ranges of `chunk` particles (the last one shorter)
int nk_schedule_fixed(ss_ctx* ctx, Plan* pl, int64_t N, int pt, int64_t chunk, Plan::NkSched** out) {
  chunk = std::max<int64_t>(pt, ((chunk + pt - 1) / pt) * pt);
  const auto key = std::make_pair(N, chunk);
  auto it = pl->nk_fixed.find(key);
  if (it != pl->nk_fixed.end()) {
    *out = &it->second;
    return SS_OK;
  }
  const int64_t Pb = (N + chunk - 1) / chunk;
  const size_t nb = pl->block_maxlen.size();
  std::vector<NkUnit> units;
  units.reserve(nb * Pb);
  for (size_t b = 0; b < nb; ++b)
    for (int64_t r = 0; r < Pb; ++r)
      units.push_back(NkUnit{(int32_t)b, (int32_t)r, (int32_t)(r * chunk), (int32_t)std::min<int64_t>(N, (r + 1) * chunk)});
  std::vector<int32_t> rows_of(pl->M, (int32_t)Pb);
  Plan::NkSched sc;
  sc.nunits = (int64_t)units.size();
  sc.rows = Pb;
  SS_HIP(ctx, hipMalloc(&sc.units, sizeof(NkUnit) * units.size()));
  SS_HIP(ctx, hipMalloc(&sc.rows_of, sizeof(int32_t) * rows_of.size()));
  SS_HIP(ctx, hipMemcpy(sc.units, units.data(), sizeof(NkUnit) * units.size(), hipMemcpyHostToDevice));
  SS_HIP(ctx, hipMemcpy(sc.rows_of, rows_of.data(), sizeof(int32_t) * rows_of.size(), hipMemcpyHostToDevice));
  pl->nk_fixed[key] = sc;
  *out = &pl->nk_fixed[key];
  return SS_OK;
}

// tiled d = 2 n(k) pass: the particles split into nrows chunks (multiples of 16)
// so that tiles x nrows is about two rounds of resident blocks
int nk2_schedule(ss_ctx* ctx, Plan* pl, int64_t N, Plan::Nk2Sched** out) {
  auto it = pl->nk2_sched.find(N);
  if (it != pl->nk2_sched.end()) {
    *out = &it->second;
    return SS_OK;
  }
  if (tl_no_alloc) return refuse_alloc(ctx, "the tiled n(k) schedule");
  const int64_t target = 2 * (int64_t)num_cus(ctx) * nk2_blocks_per_cu();
  int64_t nrows = std::max<int64_t>(1, (target + pl->t2_ntiles / 2) / std::max<int64_t>(1, pl->t2_ntiles));
  nrows = std::min<int64_t>(nrows, std::min<int64_t>(kMaxNkRows, (N + 15) / 16));
  int64_t chunk = (N + nrows - 1) / nrows;
  chunk = ((chunk + 15) / 16) * 16;
  Plan::Nk2Sched sc;
  sc.chunk = chunk;
  sc.nrows = (int)((N + chunk - 1) / chunk);
  std::vector<int32_t> rows((size_t)pl->M, sc.nrows);
  SS_HIP(ctx, hipMalloc(&sc.rows_of, sizeof(int32_t) * rows.size()));
  SS_HIP(ctx, hipMemcpy(sc.rows_of, rows.data(), sizeof(int32_t) * rows.size(), hipMemcpyHostToDevice));
  pl->nk2_sched[N] = sc;
  *out = &pl->nk2_sched[N];
  return SS_OK;
}

// fixed-chunk schedule of the tiled d = 2 pass in batches: partial rows of
// `chunk` particles (rounded up to 16), a function of (N, chunk) only
int nk2_schedule_fixed(ss_ctx* ctx, Plan* pl, int64_t N, int64_t chunk, Plan::Nk2Sched** out) {
  chunk = std::max<int64_t>(16, ((chunk + 15) / 16) * 16);
  const auto key = std::make_pair(N, chunk);
  auto it = pl->nk2_fixed.find(key);
  if (it != pl->nk2_fixed.end()) {
    *out = &it->second;
    return SS_OK;
  }
  Plan::Nk2Sched sc;
  sc.chunk = chunk;
  sc.nrows = (int)((N + chunk - 1) / chunk);
  std::vector<int32_t> rows((size_t)pl->M, sc.nrows);
  SS_HIP(ctx, hipMalloc(&sc.rows_of, sizeof(int32_t) * rows.size()));
  SS_HIP(ctx, hipMemcpy(sc.rows_of, rows.data(), sizeof(int32_t) * rows.size(), hipMemcpyHostToDevice));
  pl->nk2_fixed[key] = sc;
  *out = &pl->nk2_fixed[key];
  return SS_OK;
}

// launch shape and workspace layout; tile == nullptr: the single-launch shape
// (grids sized to the device), else the batched shape of `tile`
int make_cfg(ss_ctx* ctx, const ss_problem* p, Plan* pl, LaunchCfg* c, const TileSpec* tile = nullptr) {
  c->d = p->d;
  c->N = p->N;
  c->M = p->M;
  c->R1 = pl->R + 1;
  const size_t per_particle = (size_t)p->d * c->R1 * 4 * sizeof(double);
  const size_t lds_budget = 64 * 1024;
  // d = 2 from R = kNk2MinR on: every n(k) pass (single, batched, FP64) is the
  // tiled one, which stages 32 table rows whatever R is; the piece walk, which
  // stages whole particle tables in LDS, is not used
  const bool tiles_only = p->d == 2 && pl->R >= kNk2MinR && pl->t2_ntiles > 0;
  if (16 * per_particle <= lds_budget) c->pt = 16;
  else if (4 * per_particle <= lds_budget) c->pt = 4;
  else if (per_particle <= lds_budget || tiles_only) c->pt = 1;
  else return set_err(ctx, SS_EINVAL, "cutoff radius too large for the LDS particle tables");
  c->segblocks = (pl->nsegs + kNkPieces - 1) / kNkPieces;
  Plan::NkSched* sc = nullptr;
  {
    int rc = tile ? nk_schedule_fixed(ctx, pl, c->N, c->pt, tile->nk_chunk, &sc)
                  : nk_schedule(ctx, pl, c->N, c->pt, &sc);
    if (rc) return rc;
  }
  c->P = tiles_only ? 1 : sc->rows;
  if (pl->t2_ntiles > 0 && use_nk2(p->d, pl->R, c->N, tile != nullptr)) {  // partial rows of the tiled d = 2 pass
    Plan::Nk2Sched* s2 = nullptr;
    int rc = tile ? nk2_schedule_fixed(ctx, pl, c->N, tile->nk_chunk, &s2) : nk2_schedule(ctx, pl, c->N, &s2);
    if (rc) return rc;
    c->P = std::max<int64_t>(c->P, s2->nrows);
  }
  // gradient pass: blocks of 64 particles x Q chunks, each wave of a block on one
  // of kWaves sub-chunks of equal pair count
  const int64_t pblocks = (c->N + 63) / 64;
  const int64_t maxQ = std::min<int64_t>(std::max<int64_t>(1, pl->nruns / kWaves), 1024);
  if (tile) {
    c->Q = (int)std::max<int64_t>(1, std::min<int64_t>(maxQ, (c->M + tile->grad_k - 1) / tile->grad_k));
  } else {
    const int64_t capacity = (int64_t)num_cus(ctx) * grad_blocks_per_cu(p->d);
    c->Q = (int)rounds_fit(capacity, pblocks, maxQ, 4);
    // all Q chunks of a particle block run on one XCD and share its table rows
    // in that XCD's L2: with at least Qmin chunks, the particle blocks in flight
    // on an XCD (capacity / kXcds blocks over Q chunks each) keep their table
    // rows within kGradL2Bytes.  Among Qmin .. 2 Qmin the count that fills the
    // last round of blocks best is taken.  Not when Qmin exceeds kGradMaxQ:
    // then a particle block's rows alone nearly fill the L2 (d = 2 at large
    // cutoffs) and more chunks would only add partial rows.
    const int64_t rows_bytes = 64 * (int64_t)p->d * c->R1 * 4 * (int64_t)sizeof(double);
    const int64_t qmin = std::min<int64_t>(maxQ, (capacity / kXcds * rows_bytes + kGradL2Bytes - 1) / kGradL2Bytes);
    if (c->Q < qmin && qmin <= kGradMaxQ) {
      int64_t best = qmin;
      double best_eff = -1.0;
      for (int64_t q = qmin; q <= std::min<int64_t>(maxQ, 2 * qmin); ++q) {
        const int64_t blocks = q * pblocks;
        const double eff = (double)blocks / (double)(((blocks + capacity - 1) / capacity) * capacity);
        if (eff > best_eff + 1e-9) {
          best_eff = eff;
          best = q;
        }
      }
      c->Q = (int)best;
    }
  }
  c->combine_blocks = (c->M + kCombK - 1) / kCombK;
  size_t off = 0;
  c->off_tab = off;
  off += align256((size_t)p->d * c->R1 * 4 * c->N * sizeof(double));
  c->off_part = off;
  off += align256((size_t)c->P * 4 * c->M * sizeof(double));
  c->off_csw = off;
  off += align256((size_t)4 * c->M * sizeof(double));
  c->off_gpart = off;
  off += align256((size_t)c->Q * 2 * p->d * c->N * sizeof(double));
  c->off_blk = off;
  off += align256((size_t)c->combine_blocks * 5 * sizeof(double));
  c->off_scalar = off;
  off += align256(8 * sizeof(double));
  c->total = off;
  return SS_OK;
}

int check_problem(ss_ctx* ctx, const ss_problem* p) {
  if (!p) return set_err(ctx, SS_EINVAL, "problem is NULL");
  if (p->d < 1 || p->d > 4) return set_err(ctx, SS_EINVAL, "d must be in 1..4");
  if (p->N < 1) return set_err(ctx, SS_EINVAL, "N must be >= 1");
  if (p->R2 < 1) return set_err(ctx, SS_EINVAL, "R2 must be >= 1");
  if (!(p->L > 0.0) || !isfinite(p->L)) return set_err(ctx, SS_EINVAL, "L must be positive and finite");
  if (p->vkind < 0 || p->vkind > 2) return set_err(ctx, SS_EINVAL, "vkind must be 0, 1 or 2");
  if (isqrt64(p->R2) > 32767) return set_err(ctx, SS_EINVAL, "R2 too large");
  if (p->N > ((int64_t)1 << 31) / 4) return set_err(ctx, SS_EINVAL, "N too large");
  const int64_t M = count_half(p->d, p->R2);
  if (M != p->M) return set_err(ctx, SS_EINVAL, "M does not match |H(R2)|");
  if (M < 1 || M >= ((int64_t)1 << 31)) return set_err(ctx, SS_EINVAL, "M out of range");
  return SS_OK;
}

}  // namespace

namespace ss {
// shared with the minimiser
TileSpec tile_for(ss_ctx* ctx, int d, int64_t N, int64_t M) {
  for (const ss_tile_entry& e : ctx->tiles)
    if ((e.d == 0 || e.d == d) && N <= e.max_N && M <= e.max_M) return e.t;
  // built-in shape: at most kMaxNkRows partial rows, so the partial sums stay
  // within 32 kMaxNkRows M bytes however large N is
  return TileSpec{std::max<int64_t>(kDefaultNkChunk, (N + kMaxNkRows - 1) / kMaxNkRows), kDefaultGradK};
}

// the batched shape of a problem: plan, layout, n(k) schedule and gradient chunks
int prepare_tiled(ss_ctx* ctx, const ss_problem* p, Plan** pl, LaunchCfg* cfg, Plan::NkSched** sc,
                  int32_t** chunk_begin, Plan::Nk2Sched** s2) {
  int rc = check_problem(ctx, p);
  if (rc) return rc;
  SS_HIP(ctx, hipSetDevice(ctx->device));
  std::lock_guard<std::mutex> g(ctx->mu);
  rc = build_plan(ctx, p->d, p->R2, pl);
  if (rc) return rc;
  const TileSpec t = tile_for(ctx, p->d, p->N, p->M);
  rc = make_cfg(ctx, p, *pl, cfg, &t);
  if (rc) return rc;
  rc = nk_schedule_fixed(ctx, *pl, p->N, cfg->pt, t.nk_chunk, sc);
  if (rc) return rc;
  *s2 = nullptr;
  if ((*pl)->t2_ntiles > 0 && use_nk2(p->d, (*pl)->R, p->N, true)) {
    rc = nk2_schedule_fixed(ctx, *pl, p->N, t.nk_chunk, s2);
    if (rc) return rc;
  }
  return chunk_bounds(ctx, *pl, cfg->Q * kWaves, chunk_begin);
}

int prepare(ss_ctx* ctx, const ss_problem* p, Plan** pl, LaunchCfg* cfg) {
  int rc = check_problem(ctx, p);
  if (rc) return rc;
  SS_HIP(ctx, hipSetDevice(ctx->device));
  std::lock_guard<std::mutex> g(ctx->mu);
  rc = build_plan(ctx, p->d, p->R2, pl);
  if (rc) return rc;
  return make_cfg(ctx, p, *pl, cfg);
}

namespace {
hipEvent_t prof_event(ss_ctx* ctx) {
  hipEvent_t e = nullptr;
  if (!ctx->prof.pool.empty()) {
    e = ctx->prof.pool.back();
    ctx->prof.pool.pop_back();
  } else if (hipEventCreate(&e) != hipSuccess) {
    e = nullptr;
  }
  return e;
}
}  // namespace

hipEvent_t prof_begin(ss_ctx* ctx, int which, hipStream_t st) {
  if (!(ctx->prof.mask & (1 << which))) return nullptr;
  std::lock_guard<std::mutex> g(ctx->prof.mu);
  hipEvent_t a = prof_event(ctx);
  if (a && hipEventRecord(a, st) != hipSuccess) {
    ctx->prof.pool.push_back(a);
    return nullptr;
  }
  return a;
}

void prof_end(ss_ctx* ctx, int which, hipStream_t st, hipEvent_t a, double work) {
  std::lock_guard<std::mutex> g(ctx->prof.mu);
  hipEvent_t b = prof_event(ctx);
  if (!b || hipEventRecord(b, st) != hipSuccess) {
    ctx->prof.pool.push_back(a);
    if (b) ctx->prof.pool.push_back(b);
    return;
  }
  ctx->prof.ev[which].push_back(ProfileLog::Rec{a, b, work});
}

int energy_grad_impl(ss_ctx* ctx, const ss_problem* p, Plan* pl, const LaunchCfg& c, const double* v_dev,
                     const double* pos, double* phi, double* smax, double* grad, double* nk, char* ws,
                     hipStream_t st, double* kmax, const int* active, bool fp64) {
  double* tab = (double*)(ws + c.off_tab);
  double* part = (double*)(ws + c.off_part);
  double* csw = (double*)(ws + c.off_csw);
  double* gpart = (double*)(ws + c.off_gpart);
  double* blk = (double*)(ws + c.off_blk);
  double* scal = (double*)(ws + c.off_scalar);
  const double* v = p->vkind == 0 ? nullptr : v_dev;
  const double pairs = (double)p->M * (double)p->N;
  SS_HIP(ctx, timed(ctx, 2, st, (double)p->d * c.R1 * p->N,
                    [&] { return launch_table(pos, p->d, p->N, c.R1, tab, st, active); }));
  Plan::NkSched* sc = &pl->nk_sched.at(p->N);
  // d = 2 at large cutoffs: the tiled pass writes its partials by walk position
  const auto t2 = pl->nk2_sched.find(p->N);
  const bool tiled = pl->t2_ntiles > 0 && use_nk2(p->d, pl->R, p->N, false) && t2 != pl->nk2_sched.end() &&
                     t2->second.nrows <= c.P;
  if (tiled) {
    const Plan::Nk2Sched& s2 = t2->second;
    SS_HIP(ctx, timed(ctx, 0, st, pairs, [&] {
             return fp64 ? launch_nk2_64(pl->t2_tiles, pl->t2_ntiles, pl->t2_lexinfo, pl->R, tab, p->N, c.R1, s2.chunk,
                                         s2.nrows, part, p->M, st, active)
                         : launch_nk2(pl->t2_tiles, pl->t2_ntiles, pl->t2_lexinfo, pl->R, tab, p->N, c.R1, s2.chunk,
                                      s2.nrows, part, p->M, st, active);
           }));
    if (fp64)
      SS_HIP(ctx, launch_nk_combine64(c, part, s2.rows_of, pl->t2_ident, pl->canon_of_lex, v, nk, csw, blk, st, active));
    else
      SS_HIP(ctx, launch_nk_combine(c, part, s2.rows_of, pl->t2_ident, pl->canon_of_lex, v, nk, csw, blk, st, active));
  } else {
    if (sc->rows > c.P) return set_err(ctx, SS_EHIP, "n(k) partial rows exceed the workspace layout");
    SS_HIP(ctx, timed(ctx, 0, st, pairs, [&] {
             return fp64 ? launch_nk64(c, pl->segs, pl->nsegs, sc->units, sc->nunits, tab, part, pl->slot_off, st, active)
                         : launch_nk(c, pl->segs, pl->nsegs, sc->units, sc->nunits, tab, part, pl->slot_off, st, active);
           }));
    if (fp64)
      SS_HIP(ctx, launch_nk_combine64(c, part, sc->rows_of, pl->k_of_slot, pl->canon_of_lex, v, nk, csw, blk, st, active));
    else
      SS_HIP(ctx, launch_nk_combine(c, part, sc->rows_of, pl->k_of_slot, pl->canon_of_lex, v, nk, csw, blk, st, active));
  }
  if (phi) SS_HIP(ctx, launch_final(c, blk, phi, smax ? smax : scal + 2, kmax, st, active));
  if (grad) {
    int32_t* cb = nullptr;
    {
      std::lock_guard<std::mutex> g(ctx->mu);
      int rc = chunk_bounds(ctx, pl, c.Q * kWaves, &cb);
      if (rc) return rc;
    }
    SS_HIP(ctx, timed(ctx, 1, st, pairs, [&] {
             return fp64 ? launch_grad64(c, pl->runs, cb, tab, csw, gpart, st, active)
                         : launch_grad(c, pl->runs, cb, tab, csw, gpart, st, active);
           }));
    if (fp64) SS_HIP(ctx, launch_grad_combine64(c, gpart, p->L, false, grad, st, active));
    else SS_HIP(ctx, launch_grad_combine(c, gpart, p->L, grad, st, active));
  }
  return SS_OK;
}
}  // namespace ss

extern "C" {

int ss_create(int device, ss_ctx** out) {
  if (!out) return SS_EINVAL;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return SS_EINVAL;
  if (hipSetDevice(device) != hipSuccess) return SS_EHIP;
  ss_ctx* c = new (std::nothrow) ss_ctx();
  if (!c) return SS_ENOMEM;
  c->device = device;
  if (scratch_address(device, &c->scratch) != SS_OK) {
    delete c;
    return SS_EHIP;
  }
  if (hipStreamCreateWithFlags(&c->build_stream, hipStreamNonBlocking) != hipSuccess) {
    delete c;
    return SS_EHIP;
  }
  *out = c;
  return SS_OK;
}

int ss_destroy(ss_ctx* ctx) {
  if (!ctx) return SS_OK;
  if (ctx->server) ss_server_stop(ctx);
  hipSetDevice(ctx->device);
  for (auto& kv : ctx->plans) free_plan(kv.second);
  for (auto& v : ctx->prof.ev)
    for (auto& pr : v) {
      hipEventDestroy(pr.a);
      hipEventDestroy(pr.b);
    }
  for (hipEvent_t e : ctx->prof.pool) hipEventDestroy(e);
  if (ctx->build_stream) hipStreamDestroy(ctx->build_stream);
  delete ctx;
  return SS_OK;
}

#ifndef SS_BUILD_ID
#define SS_BUILD_ID "unknown"
#endif
const char* ss_build_id(void) { return SS_BUILD_ID; }

const char* ss_strerror(int code) {
  switch (code) {
    case SS_OK: return "ok";
    case SS_PENDING: return "pending";
    case SS_EINVAL: return "invalid argument";
    case SS_ENOMEM: return "out of device memory";
    case SS_EHIP: return "HIP runtime error";
    case SS_ENOTFOUND: return "unknown ticket";
    case SS_ESTATE: return "invalid state";
    case SS_ENUMERIC: return "non-finite value";
    default: return "unknown error code";
  }
}

const char* ss_last_error(ss_ctx* ctx) { return ctx ? ctx->last_error.c_str() : ""; }

int ss_uniform_positions(int d, int64_t N, uint64_t seed, double* out) {
  if (d < 1 || d > 4 || N < 1 || !out) return SS_EINVAL;
  // SplitMix64 (Steele, Lea, Flood 2014): output i (from 1) of the sequence
  // started at seed is the finaliser of seed + i * golden gamma
  auto output = [seed](uint64_t i) {
    uint64_t z = seed + i * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  };
  const int64_t DN = (int64_t)d * N;
  for (int64_t e = 0; e < DN; ++e) {  // e = a N + j
    const double ta = std::ldexp((double)(output((uint64_t)(2 * e + 1)) >> 11), -53);   // exact
    const double tb = std::ldexp((double)(output((uint64_t)(2 * e + 2)) >> 11), -106);  // exact
    const double hi = ta + tb;  // u rounded to nearest
    out[e] = hi;
    out[DN + e] = (ta - hi) + tb;  // u - hi, exact
  }
  return SS_OK;
}

int ss_count(int d, int64_t R2, int64_t* M) {
  if (!M || d < 1 || d > 4 || R2 < 1 || isqrt64(R2) > 32767) return SS_EINVAL;
  *M = count_half(d, R2);
  return SS_OK;
}

int ss_cutoff(int d, int64_t N, double chi, int64_t* R2, int64_t* M) {
  if (!R2 || !M || d < 1 || d > 4 || N < 2 || !(chi > 0.0) || !(chi < 0.5)) return SS_EINVAL;
  const double T = chi * (double)d * (double)(N - 1);
  if (count_half(d, 1) > T) return SS_EINVAL;
  // largest R2 with M(R2) <= T (M is nondecreasing), then down to a realised shell
  int64_t lo = 1, hi = 2;
  while (count_half(d, hi) <= T) {
    lo = hi;
    hi *= 2;
    if (hi > ((int64_t)1 << 40)) return SS_EINVAL;
  }
  while (hi - lo > 1) {
    const int64_t mid = lo + (hi - lo) / 2;
    if (count_half(d, mid) <= T) lo = mid;
    else hi = mid;
  }
  int64_t s = lo;
  const int64_t Ms = count_half(d, s);
  while (s > 1 && count_half(d, s - 1) == Ms) --s;
  *R2 = s;
  *M = Ms;
  return SS_OK;
}

int ss_wavevectors(ss_ctx* ctx, int d, int64_t R2, int32_t* n_dev, int64_t capacity, int64_t* M, void* stream) {
  if (!ctx || !M) return SS_EINVAL;
  if (d < 1 || d > 4 || R2 < 1 || isqrt64(R2) > 32767) return set_err(ctx, SS_EINVAL, "bad (d, R2)");
  SS_HIP(ctx, hipSetDevice(ctx->device));
  Plan* pl = nullptr;
  {
    std::lock_guard<std::mutex> g(ctx->mu);
    int rc = build_plan(ctx, d, R2, &pl);
    if (rc) return rc;
  }
  *M = pl->M;
  if (!n_dev) return SS_OK;
  if (capacity < pl->M) return set_err(ctx, SS_EINVAL, "capacity < M");
  hipStream_t st = (hipStream_t)stream;
  SS_HIP(ctx, hipMemcpyAsync(n_dev, pl->canon_n, sizeof(int32_t) * pl->M * d, hipMemcpyDeviceToDevice, st));
  SS_HIP(ctx, hipStreamSynchronize(st));
  return SS_OK;
}

int ss_weights(ss_ctx* ctx, const ss_problem* prob, const int32_t* n_dev, double* v_dev, void* stream) {
  if (!ctx) return SS_EINVAL;
  int rc = check_problem(ctx, prob);
  if (rc) return rc;
  if (!n_dev || !v_dev) return set_err(ctx, SS_EINVAL, "NULL n_dev or v_dev");
  if (prob->vkind != 0 && prob->vkind != 1) return set_err(ctx, SS_EINVAL, "ss_weights needs vkind 0 or 1");
  SS_HIP(ctx, hipSetDevice(ctx->device));
  SS_HIP(ctx, launch_weights(n_dev, prob->M, prob->d, prob->R2, prob->vkind, v_dev, (hipStream_t)stream));
  return SS_OK;
}

int ss_workspace_size(ss_ctx* ctx, const ss_problem* prob, int op, size_t* bytes) {
  if (!ctx || !bytes) return SS_EINVAL;
  if (op != 0 && op != 1) return set_err(ctx, SS_EINVAL, "unknown op");
  Plan* pl = nullptr;
  LaunchCfg c;
  int rc = prepare(ctx, prob, &pl, &c);
  if (rc) return rc;
  // the gradient chunk bounds too, so that everything a later
  // ss_energy_grad_static call needs exists
  {
    std::lock_guard<std::mutex> g(ctx->mu);
    int32_t* cb = nullptr;
    rc = chunk_bounds(ctx, pl, c.Q * kWaves, &cb);
    if (rc) return rc;
  }
  *bytes = c.total + (op == 1 ? minimize_extra_bytes((int64_t)prob->d * prob->N) : 0);
  return SS_OK;
}

int ss_set_progress(ss_ctx* ctx, double seconds) {
  if (!ctx || !(seconds >= 0.0) || !isfinite(seconds)) return SS_EINVAL;
  ctx->progress_interval = seconds;
  return SS_OK;
}

int ss_profile_enable(ss_ctx* ctx, int mask) {
  if (!ctx || mask < 0 || mask > 7) return SS_EINVAL;
  std::lock_guard<std::mutex> g(ctx->mu);
  ctx->prof.mask = mask;
  return SS_OK;
}

int ss_profile_read(ss_ctx* ctx, int kernel, int reset, int64_t* launches, double* total_ms, double* work) {
  if (!ctx || !launches || !total_ms || kernel < 0 || kernel > 2) return SS_EINVAL;
  std::lock_guard<std::mutex> g(ctx->prof.mu);
  auto& v = ctx->prof.ev[kernel];
  double tot = 0.0, wk = 0.0;
  for (auto& pr : v) {
    SS_HIP(ctx, hipEventSynchronize(pr.b));
    float ms = 0.0f;
    SS_HIP(ctx, hipEventElapsedTime(&ms, pr.a, pr.b));
    tot += ms;
    wk += pr.work;
  }
  *launches = (int64_t)v.size();
  *total_ms = tot;
  if (work) *work = wk;
  if (reset) {
    for (auto& pr : v) {
      ctx->prof.pool.push_back(pr.a);
      ctx->prof.pool.push_back(pr.b);
    }
    v.clear();
  }
  return SS_OK;
}

static int energy_grad_entry(ss_ctx* ctx, const ss_problem* prob, const int32_t* n_dev, const double* v_dev,
                             const double* pos_dev, double* phi_dev, double* smax_dev, double* grad_dev,
                             double* nk_dev, void* ws, size_t ws_bytes, void* stream, int precision) {
  if (!ctx) return SS_EINVAL;
  Plan* pl = nullptr;
  LaunchCfg c;
  int rc = prepare(ctx, prob, &pl, &c);
  if (rc) return rc;
  if (!n_dev || !pos_dev || !phi_dev || !ws) return set_err(ctx, SS_EINVAL, "NULL required pointer");
  if (prob->vkind != 0 && !v_dev) return set_err(ctx, SS_EINVAL, "vkind != 0 needs v_dev");
  if (ws_bytes < c.total) return set_err(ctx, SS_EINVAL, "workspace too small");
  return energy_grad_impl(ctx, prob, pl, c, v_dev, pos_dev, phi_dev, smax_dev, grad_dev, nk_dev, (char*)ws,
                          (hipStream_t)stream, nullptr, nullptr, precision == 1);
}

int ss_energy_grad(ss_ctx* ctx, const ss_problem* prob, const int32_t* n_dev, const double* v_dev,
                   const double* pos_dev, double* phi_dev, double* smax_dev, double* grad_dev, double* nk_dev,
                   void* ws, size_t ws_bytes, void* stream) {
  return energy_grad_entry(ctx, prob, n_dev, v_dev, pos_dev, phi_dev, smax_dev, grad_dev, nk_dev, ws, ws_bytes,
                           stream, 0);
}

int ss_energy_grad_static(ss_ctx* ctx, const ss_problem* prob, const int32_t* n_dev, const double* v_dev,
                          const double* pos_dev, double* phi_dev, double* smax_dev, double* grad_dev, double* nk_dev,
                          void* stream) {
  if (!ctx) return SS_EINVAL;
  NoAllocScope no_alloc;
  Plan* pl = nullptr;
  LaunchCfg c;
  int rc = prepare(ctx, prob, &pl, &c);
  if (rc) return rc;
  if (!n_dev || !pos_dev || !phi_dev) return set_err(ctx, SS_EINVAL, "NULL required pointer");
  if (prob->vkind != 0 && !v_dev) return set_err(ctx, SS_EINVAL, "vkind != 0 needs v_dev");
  if (c.total > kScratchBytes)
    return set_err(ctx, SS_ENOMEM, "the problem needs " + std::to_string(c.total) +
                                       " workspace bytes, the static scratch holds " + std::to_string(kScratchBytes));
  if (!ctx->scratch) return set_err(ctx, SS_EHIP, "no static scratch address for this device");
  return energy_grad_impl(ctx, prob, pl, c, v_dev, pos_dev, phi_dev, smax_dev, grad_dev, nk_dev, (char*)ctx->scratch,
                          (hipStream_t)stream, nullptr, nullptr, false);
}

size_t ss_static_scratch_bytes(void) { return kScratchBytes; }

int ss_energy_grad_fp64(ss_ctx* ctx, const ss_problem* prob, const int32_t* n_dev, const double* v_dev,
                        const double* pos_dev, double* phi_dev, double* smax_dev, double* grad_dev, double* nk_dev,
                        void* ws, size_t ws_bytes, void* stream) {
  return energy_grad_entry(ctx, prob, n_dev, v_dev, pos_dev, phi_dev, smax_dev, grad_dev, nk_dev, ws, ws_bytes,
                           stream, 1);
}

}  // extern "C"
