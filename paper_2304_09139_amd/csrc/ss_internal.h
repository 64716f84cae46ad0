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
  std::map<int, int32_t*> chunk_begin;           // Q -> device [Q+1] run boundaries
};

struct LaunchCfg {
  int d;
  int64_t N, M;
  int R1;          // R + 1 table entries per axis
  int pt;          // particles per LDS tile in the n(k) pass
  int64_t P;       // particle chunks of the n(k) pass
  int64_t chunk;   // particles per chunk
  int64_t segblocks;
  int Q;           // wavevector chunks of the gradient pass
  int64_t combine_blocks;
  // workspace layout (byte offsets)
  size_t off_tab, off_part, off_csw, off_gpart, off_blk, off_scalar, total;
};

constexpr int kSegLen = 8;        // wavevectors per lane in the n(k) pass
constexpr int kThreads = 256;

}  // namespace ss

struct ss_ctx {
  int device = 0;
  std::string last_error;
  std::mutex mu;
  std::map<std::pair<int, int64_t>, ss::Plan*> plans;
  hipStream_t build_stream = nullptr;
};
