// ss_internal.h -- shared declarations of the HIP library (not part of the ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <map>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

namespace ss {

// A run of consecutive wavevectors along the last axis: n = (n_0, ..., n_{D-2}, n_{D-1} + t)
// for t in [0, len), stored at walk positions k0 .. k0+len-1 of the lexicographic list.
struct Span {
  int32_t k0;
  int32_t len;
  int16_t n[4];
};
static_assert(sizeof(Span) == 16, "Span layout");

// One block of the n(k) pass: piece block `block` over particles [j0, j1),
// writing partial row `row`.
struct NkUnit {
  int32_t block;
  int32_t row;
  int32_t j0, j1;
};

constexpr int kSegLen = 8;        // wavevectors per lane in the n(k) pass
static_assert(kSegLen % 2 == 0, "an n(k) piece stores exponents in +/- pairs");

// Slot order of the n(k) partials: pieces are sorted by length (longest first),
// so the pieces longer than t are a prefix 0 .. cnt_t - 1 of the piece list;
// wavevector t of piece s (t < len_s) is slot off[t] + s, off[t] = sum_{t' < t}
// cnt_t'.  The M slots are a permutation of the wavevectors in which the lanes
// of the n(k) pass write consecutive addresses for every t.
struct SlotOffsets {
  int32_t off[kSegLen];
};

// Everything that depends only on (d, R2): the half set in lexicographic (walk)
// order and in canonical order, the map between them, the runs along the last
// axis (gradient pass) and the run pieces of length <= kSegLen (n(k) pass).
struct Plan {
  int d = 0;
  int64_t R2 = 0, M = 0;
  int R = 0;                   // floor(sqrt(R2)); exponents are in [-R, R]
  int32_t* lex_n = nullptr;    // [M][d] walk order (device)
  int32_t* canon_n = nullptr;  // [M][d] canonical order (device)
  int32_t* canon_of_lex = nullptr;  // [M] (device)
  Span* runs = nullptr;        // [nruns] (device)
  Span* segs = nullptr;        // [nsegs] (device), sorted by length, longest first
  int64_t nruns = 0, nsegs = 0;
  std::vector<int64_t> run_len_prefix;           // host, nruns+1
  std::vector<int> block_maxlen;                 // host, longest piece of each piece block
  std::vector<Span> seg_host;                    // host copy of the pieces
  SlotOffsets slot_off{};                        // slot order of the n(k) partials
  int32_t* k_of_slot = nullptr;                  // device [M]: walk position of each slot
  std::map<int, int32_t*> chunk_begin;           // chunks -> device [chunks+1] run boundaries
  struct NkSched {
    NkUnit* units = nullptr;   // device
    int32_t* rows_of = nullptr;  // device [M]: partial rows per slot
    int64_t nunits = 0, rows = 0;
  };
  std::map<int64_t, NkSched> nk_sched;           // N -> n(k) pass schedule (single launches)
  std::map<std::pair<int64_t, int64_t>, NkSched> nk_fixed;  // (N, chunk) -> fixed-chunk schedule (batches)
  // d = 2 with R >= kNk2SmallR: the tiled n(k) pass of single launches (k_nk2)
  int32_t* t2_tiles = nullptr;    // device [t2_ntiles][2]: (a0, b0) of the 16 x 16 tiles that meet H
  int64_t t2_ntiles = 0;
  int32_t* t2_lexinfo = nullptr;  // device [R + 1][3]: walk position of (n0, lo), lo, hi
  int32_t* t2_ident = nullptr;    // device [M]: slot = walk position
  struct Nk2Sched {
    int64_t chunk = 0;            // particles per partial row
    int nrows = 0;
    int32_t* rows_of = nullptr;   // device [M], all nrows
  };
  std::map<int64_t, Nk2Sched> nk2_sched;         // N -> schedule
  std::map<std::pair<int64_t, int64_t>, Nk2Sched> nk2_fixed;  // (N, chunk) -> schedule (batches)
};

// Tile shape of the batched launches for one configuration: particles per n(k)
// unit and wavevectors per gradient block.  A function of (d, N, M) only (looked
// up in the context's tile table), so that a configuration's reduction order,
// and hence its results, are the same in every batch.
struct TileSpec {
  int64_t nk_chunk;
  int64_t grad_k;
};

struct LaunchCfg {
  int d;
  int64_t N, M;
  int R1;          // R + 1 table entries per axis
  int pt;          // particles per LDS tile in the n(k) pass
  int64_t P;       // partial rows of the n(k) pass (the most any wavevector has)
  int64_t segblocks;
  int Q;           // wavevector chunks of the gradient pass
  int64_t combine_blocks;
  // workspace layout (byte offsets)
  size_t off_tab, off_part, off_csw, off_gpart, off_blk, off_scalar, total;
};

constexpr int kThreads = 256;     // threads per block
constexpr int kWaves = 4;         // waves per block
constexpr int kNkPieces = 256;    // run pieces per n(k) block (one per lane)
constexpr int kTabRun = 16;       // phase-table exponents per thread (one sin/cos pair each)
constexpr int kCombK = 32;        // wavevectors per block of the partial combine
constexpr int kXcds = 8;          // accelerator complex dies (one L2 each); workgroups are dealt round-robin
#ifndef SS_GRAD_L2_BYTES
#define SS_GRAD_L2_BYTES (2 << 20)
#endif
// table bytes of the gradient pass's particle blocks in flight on one XCD (of its 4 MB L2)
constexpr int64_t kGradL2Bytes = SS_GRAD_L2_BYTES;
constexpr int64_t kGradMaxQ = 32;  // the largest chunk count that rule may ask for
constexpr int64_t kDefaultNkChunk = 64;   // batched tile defaults (no matching tile entry)
constexpr int64_t kDefaultGradK = 1024;
constexpr int64_t kMaxNkRows = 256;         // built-in shape: particle chunks per n(k) piece block
#ifndef SS_NK_ROUNDS
#define SS_NK_ROUNDS 4
#endif
constexpr int kNkRounds = SS_NK_ROUNDS;     // most rounds of resident blocks in a single-launch n(k) pass
constexpr int64_t kNkMinChunk = 100;        // fewest particles per n(k) unit (on average) that a round may leave
// d = 2 evaluations use the tiled n(k) pass (k_nk2) from R = kNk2MinR on; single
// launches also from R = kNk2SmallR on when N <= kNk2SmallN, where the piece
// walk's grid is small (measured: the walk is faster in between, e.g. N = 8000 at
// R = 45, and in batches below R = 48, where the grid is full anyway and the
// tiles' idle lanes outside H cost more)
constexpr int kNk2MinR = 48;
constexpr int kNk2SmallR = 16;
constexpr int64_t kNk2SmallN = 2500;
inline bool use_nk2(int d, int R, int64_t N, bool batched) {
  return d == 2 && (R >= kNk2MinR || (!batched && R >= kNk2SmallR && N <= kNk2SmallN));
}

}  // namespace ss

namespace ss {
// optional per-kernel timing: hipEvent pairs recorded on the launch stream
struct ProfileLog {
  struct Rec {
    hipEvent_t a, b;
    double work;  // pairs (n(k) and gradient passes) or table entries covered by the launch
  };
  int mask = 0;  // bit k: time kernel k
  std::mutex mu;  // event records come from the caller's thread and the server's
  std::vector<Rec> ev[3];  // 0 n(k) pass, 1 gradient pass, 2 phase table
  std::vector<hipEvent_t> pool;
};
}  // namespace ss

struct ss_ctx;
namespace ss {
// event pair around one launch of kernel `which` when its timing is enabled
hipEvent_t prof_begin(ss_ctx* ctx, int which, hipStream_t st);
void prof_end(ss_ctx* ctx, int which, hipStream_t st, hipEvent_t a, double work);
template <class F>
hipError_t timed(ss_ctx* ctx, int which, hipStream_t st, double work, F launch) {
  hipEvent_t a = prof_begin(ctx, which, st);
  hipError_t e = launch();
  if (a) prof_end(ctx, which, st, a, work);
  return e;
}
}  // namespace ss

struct ss_tile_entry {
  int d;            // 0 matches every d
  int64_t max_N, max_M;
  ss::TileSpec t;
};

struct ss_server;

struct ss_ctx {
  int device = 0;
  ss_server* server = nullptr;       // continuous-batching server, if started
  double progress_interval = 0.0;    // > 0: quenches print progress lines to stderr this often (s)
  std::vector<ss_tile_entry> tiles;  // batched tile table, first match wins
  std::string last_error;
  std::mutex mu;
  std::map<std::pair<int, int64_t>, ss::Plan*> plans;
  hipStream_t build_stream = nullptr;
  ss::ProfileLog prof;
  void* scratch = nullptr;  // this device's static scratch (ss_energy_grad_static)
};
