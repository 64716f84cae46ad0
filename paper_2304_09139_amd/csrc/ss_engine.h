// ss_engine.h -- shared pieces of the batched quench engines (one-shot batches
// and the serving loop): per-configuration setup, work lists and the launch
// sequences of one minimiser step.  Not part of the ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "ss.h"
#include "ss_internal.h"
#include "ss_min.h"

namespace ss {
int prepare_tiled(ss_ctx* ctx, const ss_problem* p, Plan** pl, LaunchCfg* cfg, Plan::NkSched** sc,
                  int32_t** chunk_begin, Plan::Nk2Sched** s2);
TileSpec tile_for(ss_ctx* ctx, int d, int64_t N, int64_t M);
bool min_opts_valid(const ss_min_opts* op);
MinParams min_params(const ss_min_opts* op, const ss_problem* prob);

hipError_t launch_batch_table(const EvalSlot* es, const BUnit* units, int64_t n, int which, int gate,
                              hipStream_t st);
hipError_t launch_batch_nk(int d, int pt, int R1max, const EvalSlot* es, const BUnit* units, int64_t n, int gate,
                           hipStream_t st);
hipError_t launch_batch_nk2(const EvalSlot* es, const BUnit* units, int64_t n, int gate, hipStream_t st);
hipError_t launch_batch_combine(const EvalSlot* es, const BUnit* units, int64_t n, int gate, hipStream_t st);
hipError_t launch_batch_final(const EvalSlot* es, const int32_t* list, int64_t n, hipStream_t st);
hipError_t launch_batch_grad(int d, const EvalSlot* es, const BUnit* units, int64_t n, int gate, hipStream_t st);
hipError_t launch_batch_gcomb(const EvalSlot* es, const BUnit* units, int64_t n, int which, int gate,
                              hipStream_t st);
hipError_t launch_batch_dots(const MinSlot* ms, const BUnit* units, int64_t n, int mode, hipStream_t st);
hipError_t launch_batch_dots_final(const MinSlot* ms, const int32_t* list, int64_t n, int mode, hipStream_t st);
hipError_t launch_batch_step(const MinSlot* ms, const BUnit* units, int64_t n, hipStream_t st);
hipError_t launch_batch_accept(const MinSlot* ms, const BUnit* units, int64_t n, hipStream_t st);
hipError_t launch_batch_init(const MinSlot* ms, const int32_t* list, int64_t n, hipStream_t st);
hipError_t launch_batch_flags(const MinSlot* ms, const int32_t* list, int64_t n, SlotFlags* out, hipStream_t st);
hipError_t launch_batch_nk64(int d, int pt, int R1max, const EvalSlot* es, const BUnit* units, int64_t n, int gate,
                             hipStream_t st);
hipError_t launch_batch_nk2_64(const EvalSlot* es, const BUnit* units, int64_t n, int gate, hipStream_t st);
hipError_t launch_batch_combine64(const EvalSlot* es, const BUnit* units, int64_t n, int gate, hipStream_t st);
hipError_t launch_batch_grad64(int d, const EvalSlot* es, const BUnit* units, int64_t n, int gate, hipStream_t st);
hipError_t launch_batch_gcomb64(const EvalSlot* es, const BUnit* units, int64_t n, int which, int gate,
                                hipStream_t st);


namespace eng {

struct HostSlot {
  ss_problem prob;
  ss_min_opts opts;
  Plan* pl = nullptr;
  LaunchCfg c{};
  Plan::NkSched* sc = nullptr;
  Plan::Nk2Sched* s2 = nullptr;  // the tiled d = 2 n(k) pass (both precisions), or none
  int32_t* cb = nullptr;
  int64_t nv = 0;
  int m = 0, G = 0;
  size_t bytes = 0;  // workspace of this configuration (energy + minimiser)
  // unit counts of this configuration's grids
  int64_t n_table = 0, n_nk = 0, n_comb = 0, n_grad = 0, n_gcomb = 0, n_dots = 0, n_vec = 0;
  int64_t n_nk2 = 0;  // tiles x rows of the tiled pass (used when s2 is set)
  double work = 0.0;  // M N, for ordering
  int phase = 1;      // evaluation precision now: 0 FP64 (first stage or FP64 only), 1 double-double
};

// offsets and counts of each batched launch inside the unit array
struct Lists {
  struct Group {
    int d, pt, R1max;  // pt = 0: the tiled d = 2 pass
    int64_t off, n;
    double pairs;  // M N summed over the group's configurations
  };
  double table_work = 0.0;
  int64_t table_off = 0, table_n = 0, comb_off = 0, comb_n = 0, gcomb_off = 0, gcomb_n = 0;
  // configurations evaluating in FP64 (staged quenches before their switch)
  int64_t comb64_off = 0, comb64_n = 0, gcomb64_off = 0, gcomb64_n = 0;
  std::vector<Group> nk64, grad64;
  int64_t dots_off = 0, dots_n = 0, vec_off = 0, vec_n = 0;
  std::vector<Group> nk, grad;
  int64_t nlist = 0;
};

// the device arrays a batched launch reads
struct DevArrays {
  EvalSlot* es;
  MinSlot* ms;
  BUnit* units;
  int32_t* list;
  SlotFlags* flags;
};

size_t al256(size_t x);
int dot_blocks_of(int64_t nv);
size_t min_bytes(int64_t nv, int m, int G);
int setup_slot(ss_ctx* ctx, const ss_problem* p, const ss_min_opts* op, HostSlot* h);
void build_lists(const std::vector<HostSlot>& hs, std::vector<int> active, std::vector<BUnit>& U,
                 std::vector<int32_t>& list, Lists& L);
void fill_slot(const HostSlot& h, char* mem, double* x, const double* v, EvalSlot* E, MinSlot* C);
// the minimiser parameters of a configuration's current stage
MinParams stage_params(const HostSlot& h, int64_t iters_done);
// the most units a configuration contributes to one tick's lists (either precision)
int64_t max_units(const HostSlot& h);
// the starting evaluation and tests of every listed configuration
hipError_t launch_start(ss_ctx* ctx, const DevArrays& D, const Lists& L, hipStream_t st);
// one minimiser step of every listed configuration, ending with the gather of
// their running words into D.flags
hipError_t launch_tick(ss_ctx* ctx, const DevArrays& D, const Lists& L, hipStream_t st);

}  // namespace eng
}  // namespace ss
