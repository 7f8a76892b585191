// Host side of the C ABI declared in include/quadswarm.h: argument checks,
// the handle, the environment-to-workgroup partition and the launches.
#include <initializer_list>
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <algorithm>
#include <mutex>
#include <new>
#include <vector>

#include "quadswarm.h"
#include "qs_checks.h"
#include "qs_kernels.h"
#include "qs_rollout.h"

using qs::Consts;
using qs::Ptrs;

struct qs_handle {
  int dev = 0;
  int E = 0, Q = 0, Qp = 0, K = 0, OD = 0;
  int bs = 64, nblk = 0;
  int uniform_n = 0;  // every swarm holds this many quads (power of two), else 0
  Consts c{};
  Consts* d_c = nullptr;  // device copy of c, read by every kernel
  float* d_st = nullptr;
  float* d_par = nullptr;
  uint32_t* d_sw = nullptr;
  int2* d_blk = nullptr;
  int32_t* d_qenv = nullptr;
  unsigned long long* d_contacts = nullptr;
  int* d_err = nullptr;
  int* h_err = nullptr;  // pinned
  uint64_t t = 0;
  bool record = false;
  // adjoint scratch, grown on demand: tape [S][31][Q] (state and motor-noise
  // draws of the S substeps of the chunk of segments in flight), adjoint
  // [27][Q], parameter gradient [6][Q],
  // one checkpoint [27][Q]
  // uneven swarm sizes: work items of the persistent bucketed launch
  std::vector<int> env_start, env_n;  // host copy of the environments
  int4* d_items = nullptr;
  int2* d_item_envs = nullptr;
  int n_items = 0;
  int item_bs = 64;      // workgroup size of the bucketed launch
  int item_grid = 0;     // persistent grid size of the shared launch (0: one workgroup per item)
  // slot sizes (bit log2 N; 16 and 32) whose items take the partners in
  // chunks of four instead of one at a time
  uint32_t chunked = 0;
  // per slot size: swarms, and the times the autotuner measured for the
  // slot's items alone with each body (ns per call)
  int slot_swarms[7] = {0, 0, 0, 0, 0, 0, 0};
  float slot_ns_one[7] = {0, 0, 0, 0, 0, 0, 0};
  float slot_ns_chunked[7] = {0, 0, 0, 0, 0, 0, 0};
  bool bucketed = false;
  // graph-safe substep counter
  bool graph_mode = false;
  unsigned long long* d_t = nullptr;
  unsigned int* d_done = nullptr;
  float* d_tape = nullptr;
  size_t tape_cap = 0;
  float* d_lam = nullptr;
  float* d_gpar = nullptr;
  float* d_ck1 = nullptr;
};

namespace {

using qs_host::aligned;
using qs_host::check_desc;
using qs_host::finite;
using qs_host::outputs_overlap;
using qs_host::overlap;
using qs_host::Span;

// Workgroup size: one wavefront (64) unless every swarm is a single quad and
// the batch is large.  A one-wavefront workgroup needs no barrier for the
// in-swarm exchanges (32768 x 32: 128 -> 64 made the ten-substep step 4 %,
// the rollout 6 % and the backward 3 % faster); without exchanges, fewer
// and larger workgroups dispatch faster (1,048,576 x 1: 2 %).
int pick_block(int Q, int max_n) {
  if (const char* e = std::getenv("QS_BLOCK_SIZE")) {
    const int b = std::atoi(e);
    if (b == 64 || b == 128) return b;
  }
  if (max_n == 1 && Q >= 128 * 2048) return 128;
  return 64;
}

template <typename T>
int dalloc(T** p, size_t count) {
  if (count == 0) count = 1;
  if (hipMalloc((void**)p, count * sizeof(T)) != hipSuccess) {
    *p = nullptr;
    return QS_ERR_NOMEM;
  }
  return QS_OK;
}

void free_all(qs_handle* h) {
  (void)hipFree(h->d_st);
  (void)hipFree(h->d_par);
  (void)hipFree(h->d_sw);
  (void)hipFree(h->d_blk);
  (void)hipFree(h->d_qenv);
  (void)hipFree(h->d_contacts);
  (void)hipFree(h->d_err);
  (void)hipFree(h->d_tape);
  (void)hipFree(h->d_lam);
  (void)hipFree(h->d_gpar);
  (void)hipFree(h->d_ck1);
  (void)hipFree(h->d_items);
  (void)hipFree(h->d_item_envs);
  (void)hipFree(h->d_t);
  (void)hipFree(h->d_done);
  (void)hipFree(h->d_c);
  if (h->h_err) (void)hipHostFree(h->h_err);
}

Ptrs ptrs(qs_handle* h) {
  Ptrs p;
  p.st = h->d_st;
  p.par = h->d_par;
  p.sw = h->d_sw;
  p.blk = h->d_blk;
  p.contacts = h->record ? h->d_contacts : nullptr;
  p.err = h->d_err;
  p.Qp = h->Qp;
  p.Q = h->Q;
  p.items = h->d_items;
  p.item_envs = h->d_item_envs;
  return p;
}

// Greedy packing of whole environments into workgroups of at most bs quads:
// the workgroup table (first quad, count) and, per quad, its swarm's start
// within the workgroup and its size.  Sets bs and the workgroup count.
int build_table(qs_handle* h, int bs) {
  std::vector<int2> blk;
  std::vector<uint32_t> sw((size_t)h->Qp, 0u);
  int cur_begin = 0, cur_cnt = 0;
  for (size_t e = 0; e < h->env_n.size(); ++e) {
    const int q0 = h->env_start[e], n = h->env_n[e];
    if (cur_cnt + n > bs) {
      blk.push_back(make_int2(cur_begin, cur_cnt));
      cur_begin = q0;
      cur_cnt = 0;
    }
    for (int i = 0; i < n; ++i) sw[(size_t)q0 + i] = ((uint32_t)(q0 - cur_begin) << 8) | (uint32_t)n;
    cur_cnt += n;
  }
  blk.push_back(make_int2(cur_begin, cur_cnt));
  (void)hipFree(h->d_blk);
  (void)hipFree(h->d_sw);
  h->d_blk = nullptr;
  h->d_sw = nullptr;
  if (hipMalloc((void**)&h->d_blk, blk.size() * sizeof(int2)) != hipSuccess ||
      hipMalloc((void**)&h->d_sw, sw.size() * sizeof(uint32_t)) != hipSuccess)
    return QS_ERR_NOMEM;
  if (hipMemcpy(h->d_blk, blk.data(), blk.size() * sizeof(int2), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(h->d_sw, sw.data(), sw.size() * sizeof(uint32_t), hipMemcpyHostToDevice) != hipSuccess)
    return QS_ERR_HIP;
  h->bs = bs;
  h->nblk = (int)blk.size();
  return QS_OK;
}

// Work items of the bucketed launch: every swarm gets a slot of the next
// power of two >= its size; slots of one size are grouped bs/slot per item;
// items are ordered by slot size, largest first (heaviest work first).  An
// item's w field selects the chunked partner body (slot sizes in
// h->chunked).
int log2i(int n) {
  int k = 0;
  while ((1 << k) < n) ++k;
  return k;
}

// Slot sizes with a second, chunked body in the bucketed kernel.
constexpr uint32_t kChunkable = (1u << 4) | (1u << 5);

int build_items(qs_handle* h, int bs) {
  std::vector<int4> items;
  std::vector<int2> envs;
  for (int k = 0; k < 7; ++k) h->slot_swarms[k] = 0;
  for (size_t e = 0; e < h->env_n.size(); ++e) ++h->slot_swarms[log2i(h->env_n[e])];
  for (int N = 64; N >= 1; N >>= 1) {
    const int per = bs / N;
    const int w = (h->chunked & kChunkable) >> log2i(N) & 1u;
    int in_item = 0;
    for (size_t e = 0; e < h->env_n.size(); ++e) {
      const int n = h->env_n[e];
      if ((1 << log2i(n)) != N) continue;
      if (in_item == 0) items.push_back(make_int4(N, (int)envs.size(), 0, w));
      envs.push_back(make_int2(h->env_start[e], n));
      items.back().z += 1;
      if (++in_item == per) in_item = 0;
    }
  }
  (void)hipFree(h->d_items);
  (void)hipFree(h->d_item_envs);
  h->d_items = nullptr;
  h->d_item_envs = nullptr;
  if (hipMalloc((void**)&h->d_items, items.size() * sizeof(int4)) != hipSuccess ||
      hipMalloc((void**)&h->d_item_envs, envs.size() * sizeof(int2)) != hipSuccess)
    return QS_ERR_NOMEM;
  if (hipMemcpy(h->d_items, items.data(), items.size() * sizeof(int4), hipMemcpyHostToDevice) !=
          hipSuccess ||
      hipMemcpy(h->d_item_envs, envs.data(), envs.size() * sizeof(int2),
                hipMemcpyHostToDevice) != hipSuccess)
    return QS_ERR_HIP;
  h->n_items = (int)items.size();
  h->item_bs = bs;
  return QS_OK;
}

// Launch one instantiation.  Calls of several substeps on small batches run
// the motor part one substep ahead in a second wavefront (QS_STEP_PIPE=0/1
// forces it off/on).
bool use_step_pipe(const qs_handle* h) {
  if (const char* e = std::getenv("QS_STEP_PIPE")) return e[0] == '1';
  return h->nblk <= 1024;
}

// Observation rows per staging pass.  A grid of at most 2048 workgroups
// has at most two per SIMD, which LDS never limits: the whole workgroup's
// rows in one pass (fewest synchronisations; 4096 x 8: 6.7 us per launch
// against 7.0 us in two passes).  Larger grids keep the staging area and the
// exchange tile together within 10 KiB per wavefront of the workgroup
// (160 KiB of LDS over the four wavefronts per SIMD that the step's
// registers allow), so that LDS does not hold the resident workgroups below
// what the registers allow.  At 32768 x 32 (K = 6, 64-quad workgroups, a
// 6 KiB tile) that is 16 rows per pass: ten substeps per call 40.8 -> 50.9 G
// quad-steps/s against 32 rows (13.0 KiB per workgroup, three wavefronts
// per SIMD).  QS_STAGE_ROWS=n overrides (0: every lane stores its own row).
int stage_rows(int bs, int od, int nblk) {
  static const int forced = [] {
    const char* e = std::getenv("QS_STAGE_ROWS");
    return e ? std::atoi(e) : -1;
  }();
  if (forced >= 0 && forced <= bs && (forced & (forced - 1)) == 0) return forced;
  const size_t row = (size_t)od * sizeof(float);
  const size_t tile = 2 * qs::TILE_ROWS_CO * (size_t)bs * sizeof(float);
  const size_t budget = (size_t)(bs / 64) * 10 * 1024;
  size_t cap = budget > tile ? budget - tile : 0;
  if (nblk <= 2048) cap = 48 * 1024;
  int r = bs;
  while (r > 8 && (size_t)r * row > cap) r >>= 1;
  return r;
}

template <int BS, int KT, int N>
void go(qs_handle* h, const float* act, int nsub, const float* goals, float* obs,
        hipStream_t s, float* rw) {
  size_t dyn = 0;
  int stage = 0;
  if constexpr (KT >= 0) {
    stage = stage_rows(BS, 18 + 6 * KT, h->nblk);
    dyn = (size_t)stage * (18 + 6 * KT) * sizeof(float);
  }
  if constexpr (BS == 64 && N == 8 && (KT == 6 || KT == -2)) {
    if (nsub >= 2 && use_step_pipe(h)) {
      hipLaunchKernelGGL((qs::step_pipe_kernel<KT, N>), dim3(h->nblk), dim3(128), dyn, s,
                         h->d_st, h->d_par, act, goals, h->d_c, h->Qp, h->Q, nsub,
                         (unsigned long long)h->t, ptrs(h), obs, stage,
                         h->graph_mode ? h->d_t : nullptr, h->d_done, rw);
      return;
    }
  }
  hipLaunchKernelGGL((qs::step_kernel<BS, KT, N>), dim3(h->nblk), dim3(BS), dyn, s, h->d_st,
                     h->d_par, act, goals, h->d_c, h->Qp, h->Q, nsub, (unsigned long long)h->t,
                     ptrs(h), obs, stage, h->graph_mode ? h->d_t : nullptr, h->d_done, rw);
}

// One launch of the bucketed kernel over items [item0, item0 + count).
template <int BS, int KT>
void go_range(qs_handle* h, int item0, int count, int grid, const float* act, int nsub,
              const float* goals, float* obs, hipStream_t s, float* rw) {
  const size_t dyn = KT >= 0 ? (size_t)qs::BUCKET_STAGE_ROWS * (18 + 6 * KT) * sizeof(float) : 0;
  hipLaunchKernelGGL((qs::bucket_kernel<BS, KT>), dim3(std::max(grid, 1)), dim3(BS), dyn, s,
                     h->d_st, h->d_par, act, goals, h->d_c, h->Qp, h->Q, nsub,
                     (unsigned long long)h->t, ptrs(h), obs, item0, count,
                     h->graph_mode ? h->d_t : nullptr, h->d_done, rw);
}

template <int BS, int KT>
void go_items(qs_handle* h, const float* act, int nsub, const float* goals, float* obs,
              hipStream_t s, float* rw) {
  const int grid = h->item_grid > 0 ? std::min(h->item_grid, h->n_items) : h->n_items;
  go_range<BS, KT>(h, 0, h->n_items, grid, act, nsub, goals, obs, s, rw);
}

template <int BS>
void launch_items(qs_handle* h, const float* act, int nsub, const float* goals, float* obs,
                  bool with_obs, hipStream_t s, float* rw) {
  if (!with_obs)
    go_items<BS, -2>(h, act, nsub, goals, obs, s, rw);
  else if (h->K == 6)
    go_items<BS, 6>(h, act, nsub, goals, obs, s, rw);
  else if (h->K == 0)
    go_items<BS, 0>(h, act, nsub, goals, obs, s, rw);
  else
    go_items<BS, -1>(h, act, nsub, goals, obs, s, rw);
}

// One launch over an item range alone (autotuner trials; not in graph
// mode).
template <int BS>
void launch_range(qs_handle* h, int item0, int count, const float* act, int nsub,
                  const float* goals, float* obs, bool with_obs, hipStream_t s) {
  if (!with_obs)
    go_range<BS, -2>(h, item0, count, count, act, nsub, goals, obs, s, nullptr);
  else if (h->K == 6)
    go_range<BS, 6>(h, item0, count, count, act, nsub, goals, obs, s, nullptr);
  else if (h->K == 0)
    go_range<BS, 0>(h, item0, count, count, act, nsub, goals, obs, s, nullptr);
  else
    go_range<BS, -1>(h, item0, count, count, act, nsub, goals, obs, s, nullptr);
}

template <int BS, int KT>
void go_n(qs_handle* h, const float* act, int nsub, const float* goals, float* obs,
          hipStream_t s, float* rw) {
  switch (h->uniform_n) {
    case 1: go<BS, KT, 1>(h, act, nsub, goals, obs, s, rw); break;
    case 2: go<BS, KT, 2>(h, act, nsub, goals, obs, s, rw); break;
    case 4: go<BS, KT, 4>(h, act, nsub, goals, obs, s, rw); break;
    case 8: go<BS, KT, 8>(h, act, nsub, goals, obs, s, rw); break;
    case 16: go<BS, KT, 16>(h, act, nsub, goals, obs, s, rw); break;
    case 32: go<BS, KT, 32>(h, act, nsub, goals, obs, s, rw); break;
    case 64: go<BS, KT, 64>(h, act, nsub, goals, obs, s, rw); break;
    default: go<BS, KT, 0>(h, act, nsub, goals, obs, s, rw); break;
  }
}

template <int BS>
int launch_bs(qs_handle* h, const float* act, int nsub, const float* goals, float* obs,
              bool with_obs, hipStream_t s, float* rw) {
  if (!with_obs)
    go_n<BS, -2>(h, act, nsub, goals, obs, s, rw);
  else if (h->K == 6)
    go_n<BS, 6>(h, act, nsub, goals, obs, s, rw);
  else if (h->K == 0 && h->uniform_n == 1)
    go<BS, 0, 1>(h, act, nsub, goals, obs, s, rw);
  else if (h->K == 0)
    go<BS, 0, 0>(h, act, nsub, goals, obs, s, rw);
  else
    go<BS, -1, 0>(h, act, nsub, goals, obs, s, rw);
  return hipGetLastError() == hipSuccess ? QS_OK : QS_ERR_HIP;
}

int launch(qs_handle* h, const float* act, int nsub, const float* goals, float* obs,
           bool with_obs, hipStream_t s, float* rw = nullptr) {
  if (hipSetDevice(h->dev) != hipSuccess) return QS_ERR_HIP;
  int rc;
  if (h->bucketed) {
    if (h->item_bs == 128)
      launch_items<128>(h, act, nsub, goals, obs, with_obs, s, rw);
    else
      launch_items<64>(h, act, nsub, goals, obs, with_obs, s, rw);
    rc = hipGetLastError() == hipSuccess ? QS_OK : QS_ERR_HIP;
  } else {
    switch (h->bs) {
      case 128: rc = launch_bs<128>(h, act, nsub, goals, obs, with_obs, s, rw); break;
      default: rc = launch_bs<64>(h, act, nsub, goals, obs, with_obs, s, rw); break;
    }
  }
  if (rc == QS_OK) h->t += (uint64_t)nsub;
  return rc;
}

// ---- differentiable rollouts ------------------------------------------------
// The two-wavefront rollout (motor part one substep ahead) for small
// batches, as the reverse sweep (QS_ROLLOUT_PIPE=0/1 forces it off/on).
bool use_rollout_pipe(const qs_handle* h) {
  if (const char* e = std::getenv("QS_ROLLOUT_PIPE")) return e[0] == '1';
  return h->nblk <= 1024;
}

template <int BS, int N, bool PEN>
void go_roll(qs_handle* h, const float* act, int ncalls, int nsub, float* ckpt, int ce, float* pen,
             float beta, hipStream_t s) {
  if constexpr (BS == 64 && (N == 1 || N == 8)) {
    if (use_rollout_pipe(h)) {
      hipLaunchKernelGGL((qs::rollout_pipe_kernel<N, PEN>), dim3(h->nblk),
                         dim3(64 * qs::kRollWaves<N, PEN>), 0, s, h->d_c,
                         ptrs(h), act, ncalls, nsub, (unsigned long long)h->t, ckpt, ce, pen, beta);
      return;
    }
  }
  hipLaunchKernelGGL((qs::rollout_kernel<BS, N, PEN>), dim3(h->nblk), dim3(BS), 0, s, h->d_c, ptrs(h),
                     act, ncalls, nsub, (unsigned long long)h->t, ckpt, ce, pen, beta);
}

// Device scratch of one backward pass: the tape of the chunk of segments in
// flight ([S][31][Q]), the state adjoint ([27][Q]) and the parameter
// gradient ([6][Q]).
struct AdjScratch {
  float* tape;
  float* lam;
  float* gpar;
};

// The two-wavefront recompute (motor part one substep ahead) for small
// batches, as the rollout (QS_RECOMPUTE_PIPE=0/1 forces it off/on).
bool use_recompute_pipe(const qs_handle* h) {
  if (const char* e = std::getenv("QS_RECOMPUTE_PIPE")) return e[0] == '1';
  return h->nblk <= 1024;
}

template <int BS, int N, bool PEN>
void go_recompute(qs_handle* h, const AdjScratch& sc, const float* ckpt, const float* act,
                  int ncalls, int ce, int nsub, uint64_t t0, hipStream_t s) {
  const int nseg = (ncalls + ce - 1) / ce;
  if constexpr (BS == 64 && (N == 1 || N == 8)) {
    if (use_recompute_pipe(h)) {
      hipLaunchKernelGGL((qs::recompute_pipe_kernel<N>), dim3(h->nblk, nseg), dim3(128), 0, s,
                         h->d_c, ptrs(h), ckpt, act, ncalls, ce, nsub, (unsigned long long)t0,
                         sc.tape);
      return;
    }
  }
  hipLaunchKernelGGL((qs::recompute_kernel<BS, N>), dim3(h->nblk, nseg), dim3(BS), 0, s, h->d_c,
                     ptrs(h), ckpt, act, ncalls, ce, nsub, (unsigned long long)t0, sc.tape);
}

// The four-wavefront reverse sweep pays where the batch leaves SIMDs idle:
// up to 1024 workgroups of 64 quads (QS_REVERSE_PIPE=0/1 forces it off/on).
bool use_reverse_pipe(const qs_handle* h) {
  if (const char* e = std::getenv("QS_REVERSE_PIPE")) return e[0] == '1';
  return h->nblk <= 1024;
}

template <int N, bool PEN>
void go_reverse_pipe(qs_handle* h, const AdjScratch& sc, const float* act, int ncalls, int nsub,
                     uint64_t t0, const float* gpen, float beta, float* gact, hipStream_t s) {
  hipLaunchKernelGGL((qs::reverse_pipe_kernel<N, PEN>), dim3(h->nblk), dim3(256), 0, s, h->d_c,
                     ptrs(h), act, ncalls, nsub, (unsigned long long)t0, sc.tape, sc.lam, gpen,
                     beta, gact, sc.gpar);
}

template <int BS, int N, bool PEN>
void go_reverse(qs_handle* h, const AdjScratch& sc, const float* act, int ncalls, int nsub,
                uint64_t t0, const float* gpen, float beta, float* gact, hipStream_t s) {
  if constexpr (BS == 64 && (N == 1 || N == 8)) {
    if (use_reverse_pipe(h)) {
      go_reverse_pipe<N, PEN>(h, sc, act, ncalls, nsub, t0, gpen, beta, gact, s);
      return;
    }
  }
  hipLaunchKernelGGL((qs::reverse_kernel<BS, N, PEN>), dim3(h->nblk), dim3(BS), 0, s, h->d_c,
                     ptrs(h), act, ncalls, nsub, (unsigned long long)t0, sc.tape, sc.lam, gpen,
                     beta, gact, sc.gpar);
}

// Dispatch on (block size, uniform swarm size) for a launcher template F.
template <template <int, int, bool> class F, bool PEN, typename... A>
void dispatch(qs_handle* h, A... a) {
  if (h->bs == 128) {
    switch (h->uniform_n) {
      case 1: F<128, 1, PEN>::run(h, a...); break;
      case 8: F<128, 8, PEN>::run(h, a...); break;
      case 32: F<128, 32, PEN>::run(h, a...); break;
      default: F<128, 0, PEN>::run(h, a...); break;
    }
  } else {
    switch (h->uniform_n) {
      case 1: F<64, 1, PEN>::run(h, a...); break;
      case 8: F<64, 8, PEN>::run(h, a...); break;
      case 32: F<64, 32, PEN>::run(h, a...); break;
      default: F<64, 0, PEN>::run(h, a...); break;
    }
  }
}

template <int BS, int N, bool PEN>
struct RollF {
  static void run(qs_handle* h, const float* act, int ncalls, int nsub, float* ckpt, int ce,
                  float* pen, float beta, hipStream_t s) {
    go_roll<BS, N, PEN>(h, act, ncalls, nsub, ckpt, ce, pen, beta, s);
  }
};

template <int BS, int N, bool PEN>
struct RecF {
  static void run(qs_handle* h, const AdjScratch* sc, const float* ckpt, const float* act,
                  int ncalls, int ce, int nsub, uint64_t t0, hipStream_t s) {
    go_recompute<BS, N, PEN>(h, *sc, ckpt, act, ncalls, ce, nsub, t0, s);
  }
};

template <int BS, int N, bool PEN>
struct RevF {
  static void run(qs_handle* h, const AdjScratch* sc, const float* act, int ncalls, int nsub,
                  uint64_t t0, const float* gpen, float beta, float* gact, hipStream_t s) {
    go_reverse<BS, N, PEN>(h, *sc, act, ncalls, nsub, t0, gpen, beta, gact, s);
  }
};

int grow(float** p, size_t* cap, size_t need) {
  if (need <= *cap && *p) return QS_OK;
  (void)hipFree(*p);
  *p = nullptr;
  *cap = 0;
  if (hipMalloc((void**)p, need * sizeof(float)) != hipSuccess) {
    *p = nullptr;
    return QS_ERR_NOMEM;
  }
  *cap = need;
  return QS_OK;
}

int ensure_adjoint_scratch(qs_handle* h) {
  size_t cap_lam = h->d_lam ? 1 : 0, cap_g = h->d_gpar ? 1 : 0, cap_c = h->d_ck1 ? 1 : 0;
  int rc = QS_OK;
  if (!h->d_lam) rc = grow(&h->d_lam, &cap_lam, (size_t)qs::NSTATE * h->Q);
  if (rc == QS_OK && !h->d_gpar) rc = grow(&h->d_gpar, &cap_g, (size_t)6 * h->Q);
  if (rc == QS_OK && !h->d_ck1) rc = grow(&h->d_ck1, &cap_c, (size_t)qs::NSTATE * h->Q);
  return rc;
}

// Bytes of tape the backward pass may hold at once (QS_TAPE_BYTES overrides);
// at least one segment is always taped.
size_t tape_budget() {
  if (const char* e = std::getenv("QS_TAPE_BYTES")) {
    const long long b = std::atoll(e);
    if (b > 0) return (size_t)b;
  }
  return (size_t)8 << 30;
}

void convert(const float* src, float* dst, int Q, int rows, bool to_row_major, bool acc,
             hipStream_t s) {
  const long long n = (long long)Q * rows;
  const dim3 grid((unsigned)((n + 255) / 256)), block(256);
  if (to_row_major)
    hipLaunchKernelGGL(qs::fm_to_rm_kernel, grid, block, 0, s, src, dst, Q, rows, acc ? 1 : 0);
  else
    hipLaunchKernelGGL(qs::rm_to_fm_kernel, grid, block, 0, s, src, dst, Q, rows);
}

// Floats of tape one checkpoint segment needs.
size_t segment_tape_floats(const qs_handle* h, int n_calls, int nsub, int ce) {
  return (size_t)std::min(ce, n_calls) * nsub * qs::NTAPE * h->Q;
}

// Backward pass over n_calls calls with checkpoints every ce calls (ckpt:
// [27][Q] each); sc.lam and sc.gpar already hold the incoming adjoint and
// zeros, and sc.tape holds G segments.  Segments are taken in chunks of G,
// last chunk first: one launch recomputes every segment of the chunk in
// parallel, one launch sweeps the chunk in reverse.
int run_adjoint(qs_handle* h, const AdjScratch& sc, int G, const float* act, int n_calls,
                int nsub, int ce, const float* ckpt, uint64_t t0, const float* gpen, float beta,
                float* gact, hipStream_t s) {
  const int nseg = (n_calls + ce - 1) / ce;
  for (int hi = nseg; hi > 0; hi -= G) {
    const int g0 = std::max(0, hi - G);
    const int c0 = g0 * ce, nc = std::min(n_calls, hi * ce) - c0;
    const float* ck = ckpt + (size_t)g0 * qs::NSTATE * h->Q;
    const float* a = act + (size_t)c0 * h->Q * 4;
    float* ga = gact + (size_t)c0 * h->Q * 4;
    const uint64_t ts = t0 + (uint64_t)c0 * nsub;
    dispatch<RecF, false>(h, &sc, ck, a, nc, ce, nsub, ts, s);
    if (gpen)
      dispatch<RevF, true>(h, &sc, a, nc, nsub, ts, gpen, beta, ga, s);
    else
      dispatch<RevF, false>(h, &sc, a, nc, nsub, ts, gpen, beta, ga, s);
    if (hipGetLastError() != hipSuccess) return QS_ERR_HIP;
  }
  return QS_OK;
}

// Argument checks shared by the two forms of qs_step_backward.
int check_step_backward(const qs_handle* h, const float* d_state_in, const float* d_actions,
                        int32_t n_substeps, const float* d_gstate_out, const float* d_gstate_in,
                        const float* d_gactions, const float* d_gparams) {
  if (!h || !d_state_in || !d_actions || !d_gstate_out || !d_gstate_in || !d_gactions ||
      !d_gparams)
    return QS_ERR_NULL;
  if (n_substeps < 0) return QS_ERR_INVALID;
  if (h->c.flags & qs::F_DOWNWASH) return QS_ERR_UNSUPPORTED;
  if (!aligned(d_actions, 16) || !aligned(d_gactions, 16) || !aligned(d_state_in, 4) ||
      !aligned(d_gstate_out, 4) || !aligned(d_gstate_in, 4) || !aligned(d_gparams, 4))
    return QS_ERR_ALIGN;
  // d_gstate_in may be d_gstate_out itself (both are staged), not a part of it
  const size_t Q = (size_t)h->Q;
  const bool same = d_gstate_in == d_gstate_out;
  if (outputs_overlap({{d_gstate_in, Q * 108}, {d_gactions, Q * 16}, {d_gparams, Q * 24}},
                      {{d_state_in, Q * 108}, {d_actions, Q * 16},
                       {same ? nullptr : d_gstate_out, Q * 108}}))
    return QS_ERR_INVALID;
  return QS_OK;
}

// The launches of one qs_step_backward call on the given scratch: ck1 [27][Q]
// receives the state before the call, sc.lam the incoming adjoint, sc.gpar
// zeros (a fill kernel, not a memset, so the sequence can be captured), then
// the recompute and reverse sweeps of one segment, and the results are
// converted back to the caller's row-major layouts.
int step_backward_run(qs_handle* h, const AdjScratch& sc, float* ck1, const float* d_state_in,
                      const float* d_actions, int32_t n_substeps, uint64_t substep_index,
                      const float* d_gstate_out, float* d_gstate_in, float* d_gactions,
                      float* d_gparams, hipStream_t s) {
  convert(d_state_in, ck1, h->Q, qs::NSTATE, false, false, s);
  convert(d_gstate_out, sc.lam, h->Q, qs::NSTATE, false, false, s);
  hipLaunchKernelGGL(qs::fill_kernel, dim3((unsigned)((6LL * h->Q + 255) / 256)), dim3(256), 0, s,
                     sc.gpar, 6LL * h->Q, 0.0f);
  if (n_substeps > 0) {
    const int rc = run_adjoint(h, sc, 1, d_actions, 1, n_substeps, 1, ck1, substep_index, nullptr,
                               0.f, d_gactions, s);
    if (rc != QS_OK) return rc;
  } else {
    hipLaunchKernelGGL(qs::fill_kernel, dim3((unsigned)((4LL * h->Q + 255) / 256)), dim3(256), 0,
                       s, d_gactions, 4LL * h->Q, 0.0f);
  }
  convert(sc.lam, d_gstate_in, h->Q, qs::NSTATE, true, false, s);
  convert(sc.gpar, d_gparams, h->Q, 6, true, true, s);
  return hipGetLastError() == hipSuccess ? QS_OK : QS_ERR_HIP;
}

// ---- fixed scratch of the allocation-free entry point -------------------
// qs_step_backward_noalloc keeps its scratch in this array instead of
// allocating: 64 MiB, one copy on every device the library runs on, held
// until the process ends.  Host code never uses the array's name as an
// address (on the host it names a stand-in, not device memory): the device
// address comes from hipGetSymbolAddress, looked up once per device with
// that device current, and only that pointer is passed to kernels.
}  // namespace

constexpr size_t kNoAllocScratchFloats = (size_t)QS_NOALLOC_SCRATCH_BYTES / sizeof(float);
static __device__ __align__(256) float scratch[kNoAllocScratchFloats];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
float* g_scratch_ptr[kMaxDevices] = {};

// The device address of the scratch array on device dev (which must be
// current), looked up on first use and kept.
int noalloc_scratch(int dev, float** out) {
  if (dev < 0 || dev >= kMaxDevices) return QS_ERR_UNSUPPORTED;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return QS_ERR_HIP;
    g_scratch_ptr[dev] = static_cast<float*>(p);
  }
  *out = g_scratch_ptr[dev];
  return QS_OK;
}

}  // namespace

namespace {

// Autotuner trials: every trial starts from the saved state and substep
// counter; times come from HIP events around `reps` launches after 2 untimed
// ones.
struct Trial {
  qs_handle* h;
  const float *act, *goals;
  float* obs;
  int nsub;
  bool with_obs;
  hipStream_t s;
  float* saved;
  size_t st_bytes;
  uint64_t t_saved;
  hipEvent_t e0, e1;

  int restore() {
    h->t = t_saved;
    return hipMemcpyAsync(h->d_st, saved, st_bytes, hipMemcpyDeviceToDevice, s) == hipSuccess
               ? QS_OK : QS_ERR_HIP;
  }
  template <typename F>
  int time(F&& launch_once, float* ms_per_launch) {
    int rc = restore();
    for (int w = 0; rc == QS_OK && w < 2; ++w) rc = launch_once();
    if (rc != QS_OK) return rc;
    if (hipEventRecord(e0, s) != hipSuccess) return QS_ERR_HIP;
    const int reps = 5;
    for (int r = 0; rc == QS_OK && r < reps; ++r) rc = launch_once();
    float ms = 0.f;
    if (rc != QS_OK) return rc;
    if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
        hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
      return QS_ERR_HIP;
    *ms_per_launch = ms / reps;
    return QS_OK;
  }
  int call(float* ms) {
    return time([&] { return launch(h, act, nsub, goals, obs, with_obs, s); }, ms);
  }
  int range(int item0, int count, float* ms) {
    return time([&] {
      if (h->item_bs == 128)
        launch_range<128>(h, item0, count, act, nsub, goals, obs, with_obs, s);
      else
        launch_range<64>(h, item0, count, act, nsub, goals, obs, with_obs, s);
      return hipGetLastError() == hipSuccess ? QS_OK : QS_ERR_HIP;
    }, ms);
  }
};

// Launch configuration of a bucketed handle: workgroup size, persistent
// grid and the slot sizes that take the chunked partner body.
struct BucketConfig {
  int bs, grid;
  uint32_t chunked;
};

int apply(qs_handle* h, hipStream_t s, const BucketConfig& c) {
  // no launch may still read the tables that are about to be rebuilt
  if (hipStreamSynchronize(s) != hipSuccess) return QS_ERR_HIP;
  h->chunked = c.chunked;
  h->item_grid = c.grid;
  return build_items(h, c.bs);
}

// Bucketed handles: (1) workgroup sizes 64 and 128 and persistent grids,
// every slot size with the one-partner body; (2) per slot size with two
// bodies (16 and 32), its items alone with each body, at the workgroup size
// of (1); (3) the call with each slot size on its faster body, over the
// grids; the faster of (1) and (3) is kept.
int tune_buckets(Trial& tr, BucketConfig* best) {
  qs_handle* h = tr.h;
  float best_ms = 1e30f;
  int rc = QS_OK;
  for (int bs : {64, 128})
    for (int g : {0, 1024, 2048, 4096}) {
      const BucketConfig c{bs, g, 0u};
      float ms = 0.f;
      if ((rc = apply(h, tr.s, c)) != QS_OK || (rc = tr.call(&ms)) != QS_OK) return rc;
      if (ms < best_ms) {
        best_ms = ms;
        *best = c;
      }
    }
  for (int k = 0; k < 7; ++k) h->slot_ns_one[k] = h->slot_ns_chunked[k] = 0.f;
  uint32_t mask = 0u;
  for (int k = 0; k < 7; ++k) {
    if (!(kChunkable >> k & 1u) || h->slot_swarms[k] == 0) continue;
    float t[2] = {0.f, 0.f};
    for (int v = 0; v < 2; ++v) {
      if ((rc = apply(h, tr.s, {best->bs, 0, v ? 1u << k : 0u})) != QS_OK) return rc;
      // the slot's item range (items are ordered by slot size)
      std::vector<int4> items((size_t)h->n_items);
      if (hipMemcpy(items.data(), h->d_items, items.size() * sizeof(int4),
                    hipMemcpyDeviceToHost) != hipSuccess)
        return QS_ERR_HIP;
      int i0 = -1, i1 = -1;
      for (int i = 0; i < h->n_items; ++i)
        if (items[(size_t)i].x == (1 << k)) {
          if (i0 < 0) i0 = i;
          i1 = i + 1;
        }
      if (i0 < 0 || (rc = tr.range(i0, i1 - i0, &t[v])) != QS_OK) return rc;
    }
    h->slot_ns_one[k] = t[0] * 1e6f;
    h->slot_ns_chunked[k] = t[1] * 1e6f;
    if (t[1] < t[0]) mask |= 1u << k;
  }
  if (mask == 0u) return QS_OK;
  for (int g : {0, 1024, 2048, 4096}) {
    const BucketConfig c{best->bs, g, mask};
    float ms = 0.f;
    if ((rc = apply(h, tr.s, c)) != QS_OK || (rc = tr.call(&ms)) != QS_OK) return rc;
    if (ms < best_ms) {
      best_ms = ms;
      *best = c;
    }
  }
  return QS_OK;
}

}  // namespace

extern "C" {

int qs_create(const qs_desc* desc, const qs_quad_params* h_params, const float* h_state0,
              qs_handle** out) {
  if (!out) return QS_ERR_NULL;
  *out = nullptr;
  if (!h_params || !h_state0) return QS_ERR_NULL;
  int rc = check_desc(desc);
  if (rc != QS_OK) return rc;
  const int E = desc->n_envs;
  const int Q = desc->env_offsets[E];
  rc = qs_host::check_quads(Q, h_params, h_state0);
  if (rc != QS_OK) return rc;

  qs_handle* h = new (std::nothrow) qs_handle();
  if (!h) return QS_ERR_NOMEM;
  if (hipGetDevice(&h->dev) != hipSuccess) {
    delete h;
    return QS_ERR_HIP;
  }
  h->E = E;
  h->Q = Q;
  h->Qp = (Q + 63) / 64 * 64;
  h->K = desc->k_neighbors;
  h->OD = 18 + 6 * h->K;
  int max_n = 1;
  for (int e = 0; e < E; ++e)
    max_n = std::max(max_n, desc->env_offsets[e + 1] - desc->env_offsets[e]);
  h->bs = pick_block(Q, max_n);

  // constants (derived in double, rounded once)
  Consts& c = h->c;
  c.dt = desc->dt;
  c.g = desc->gravity;
  c.arm_d = (float)((double)desc->arm_length / std::sqrt(2.0));
  c.k_tau = desc->k_tau;
  c.drag = desc->drag_coef;
  c.mu = desc->floor_mu;
  c.a_nd = desc->motor_noise_decay;
  const double and_ = desc->motor_noise_decay;
  c.ns_scale = (float)((double)desc->motor_noise_std * std::sqrt(1.0 - and_ * and_));
  c.rmin0 = desc->room_min[0];
  c.rmin1 = desc->room_min[1];
  c.rmin2 = desc->room_min[2];
  c.rmax0 = desc->room_max[0];
  c.rmax1 = desc->room_max[1];
  c.rmax2 = desc->room_max[2];
  c.e_wall = desc->wall_restitution;
  c.dcol2 = (float)((double)desc->col_dist * (double)desc->col_dist);
  c.dcol = desc->col_dist;
  c.col_decay = desc->col_decay;
  c.col_nv = desc->col_noise_v;
  c.col_nw = desc->col_noise_w;
  c.flags = desc->flags;
  c.key0 = (uint32_t)desc->seed;
  c.key1 = (uint32_t)(desc->seed >> 32);
  c.K = h->K;
  c.obs_dim = h->OD;
  c.dw_k1 = desc->dw_k1;
  c.dw_k2 = desc->dw_k2;
  c.dw_b1 = desc->dw_b1;
  c.dw_r2 = (float)((double)desc->dw_radius * (double)desc->dw_radius);
  c.dw_h = desc->dw_height;
  c.dw_na = desc->dw_noise_a;
  c.dw_nw = desc->dw_noise_w;
  c.sn_x = desc->sn_x;
  c.sn_v = desc->sn_v;
  c.sn_w = desc->sn_w;
  for (int k = 0; k < 15; ++k) c.rw[k] = 0.f;
  c.rw[14] = 1.f;

  // environment -> workgroup partition (environments are never split)
  h->env_start.resize(E);
  h->env_n.resize(E);
  std::vector<int32_t> qenv((size_t)Q, 0);
  for (int e = 0; e < E; ++e) {
    const int q0 = desc->env_offsets[e], n = desc->env_offsets[e + 1] - q0;
    h->env_start[e] = q0;
    h->env_n[e] = n;
    for (int i = 0; i < n; ++i) qenv[(size_t)q0 + i] = e;
  }
  // uniform power-of-two swarms: the greedy packing is then exactly
  // "workgroup b owns quads [b bs, (b+1) bs)", which the specialised kernels use
  {
    const int n0 = desc->env_offsets[1] - desc->env_offsets[0];
    bool uni = (n0 & (n0 - 1)) == 0 && h->bs % n0 == 0;
    for (int e = 1; uni && e < E; ++e) uni = desc->env_offsets[e + 1] - desc->env_offsets[e] == n0;
    h->uniform_n = uni ? n0 : 0;
  }

  // derived per-quad parameters and SoA state
  std::vector<float> par((size_t)qs::NPARAM * h->Qp, 1.0f);
  std::vector<float> st((size_t)qs::NSTATE * h->Qp, 0.0f);
  for (int q = 0; q < Q; ++q) {
    const qs_quad_params& p = h_params[q];
    par[(size_t)qs::P_M * h->Qp + q] = p.mass;
    par[(size_t)qs::P_JX * h->Qp + q] = p.ixx;
    par[(size_t)qs::P_JY * h->Qp + q] = p.iyy;
    par[(size_t)qs::P_JZ * h->Qp + q] = p.izz;
    par[(size_t)qs::P_FMAX * h->Qp + q] =
        (float)(0.25 * (double)p.mass * (double)desc->gravity * (double)p.thrust_to_weight);
    par[(size_t)qs::P_ALAG * h->Qp + q] =
        (float)(1.0 - std::exp(-(double)desc->dt / (double)p.motor_tau));
    par[(size_t)qs::P_T2W * h->Qp + q] = p.thrust_to_weight;
    par[(size_t)qs::P_TAU * h->Qp + q] = p.motor_tau;
    for (int f = 0; f < qs::NSTATE; ++f)
      st[(size_t)f * h->Qp + q] = h_state0[(size_t)q * QS_STATE_DIM + f];
  }

  rc = QS_OK;
  if (rc == QS_OK) rc = dalloc(&h->d_st, st.size());
  if (rc == QS_OK) rc = dalloc(&h->d_par, par.size());
  if (rc == QS_OK) rc = dalloc(&h->d_qenv, qenv.size());
  if (rc == QS_OK) rc = dalloc(&h->d_contacts, (size_t)h->Qp);
  if (rc == QS_OK) rc = dalloc(&h->d_err, 1);
  if (rc == QS_OK) rc = build_table(h, h->bs);
  if (rc == QS_OK && hipMalloc((void**)&h->d_t, sizeof(unsigned long long)) != hipSuccess)
    rc = QS_ERR_NOMEM;
  if (rc == QS_OK &&
      hipMalloc((void**)&h->d_done, qs::DONE_WORDS * sizeof(unsigned int)) != hipSuccess)
    rc = QS_ERR_NOMEM;
  if (rc == QS_OK && hipMalloc((void**)&h->d_c, sizeof(Consts)) != hipSuccess) rc = QS_ERR_NOMEM;
  if (rc == QS_OK && h->uniform_n == 0) {
    const char* ev = std::getenv("QS_BUCKETED");
    h->bucketed = !(ev && ev[0] == '0');
    if (h->bucketed) rc = build_items(h, 64);
  }
  if (rc == QS_OK && hipHostMalloc((void**)&h->h_err, sizeof(int)) != hipSuccess) {
    h->h_err = nullptr;
    rc = QS_ERR_NOMEM;
  }
  if (rc == QS_OK) {
    bool ok = hipMemcpy(h->d_st, st.data(), st.size() * sizeof(float), hipMemcpyHostToDevice) == hipSuccess;
    ok = ok && hipMemcpy(h->d_par, par.data(), par.size() * sizeof(float), hipMemcpyHostToDevice) == hipSuccess;
    if (Q > 0)
      ok = ok && hipMemcpy(h->d_qenv, qenv.data(), qenv.size() * sizeof(int32_t), hipMemcpyHostToDevice) == hipSuccess;
    ok = ok && hipMemset(h->d_contacts, 0, (size_t)h->Qp * sizeof(unsigned long long)) == hipSuccess;
    ok = ok && hipMemset(h->d_err, 0, sizeof(int)) == hipSuccess;
    ok = ok && hipMemset(h->d_t, 0, sizeof(unsigned long long)) == hipSuccess;
    ok = ok && hipMemset(h->d_done, 0, qs::DONE_WORDS * sizeof(unsigned int)) == hipSuccess;
    ok = ok && hipMemcpy(h->d_c, &h->c, sizeof(Consts), hipMemcpyHostToDevice) == hipSuccess;
    ok = ok && hipDeviceSynchronize() == hipSuccess;
    if (!ok) rc = QS_ERR_HIP;
  }
  if (rc != QS_OK) {
    free_all(h);
    delete h;
    return rc;
  }
  *h->h_err = 0;
  // set-up of the allocation-free entry point's scratch address on this
  // device (its own first call retries if this lookup failed)
  float* unused = nullptr;
  (void)noalloc_scratch(h->dev, &unused);
  *out = h;
  return QS_OK;
}

int qs_destroy(qs_handle* h) {
  if (!h) return QS_OK;
  (void)hipSetDevice(h->dev);
  (void)hipDeviceSynchronize();
  free_all(h);
  delete h;
  return QS_OK;
}

int qs_sizes(const qs_handle* h, int32_t* n_quads, int32_t* n_envs, int32_t* obs_dim) {
  if (!h) return QS_ERR_NULL;
  if (n_quads) *n_quads = h->Q;
  if (n_envs) *n_envs = h->E;
  if (obs_dim) *obs_dim = h->OD;
  return QS_OK;
}

int qs_substep_index(const qs_handle* h, uint64_t* substep_index) {
  if (!h || !substep_index) return QS_ERR_NULL;
  if (h->graph_mode) {
    unsigned long long v = 0;
    if (hipSetDevice(h->dev) != hipSuccess || hipDeviceSynchronize() != hipSuccess ||
        hipMemcpy(&v, h->d_t, sizeof(v), hipMemcpyDeviceToHost) != hipSuccess)
      return QS_ERR_HIP;
    *substep_index = v;
    return QS_OK;
  }
  *substep_index = h->t;
  return QS_OK;
}

int qs_set_graph_mode(qs_handle* h, int32_t enable, void* stream) {
  if (!h) return QS_ERR_NULL;
  if (hipSetDevice(h->dev) != hipSuccess) return QS_ERR_HIP;
  hipStream_t s = (hipStream_t)stream;
  if (hipStreamSynchronize(s) != hipSuccess) return QS_ERR_HIP;
  if (enable && !h->graph_mode) {
    hipLaunchKernelGGL(qs::set_counter_kernel, dim3(1), dim3(64), 0, s, h->d_t, h->d_done,
                       (unsigned long long)h->t);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s) != hipSuccess)
      return QS_ERR_HIP;
    h->graph_mode = true;
  } else if (!enable && h->graph_mode) {
    unsigned long long v = 0;
    if (hipMemcpy(&v, h->d_t, sizeof(v), hipMemcpyDeviceToHost) != hipSuccess) return QS_ERR_HIP;
    h->t = v;
    h->graph_mode = false;
  }
  return QS_OK;
}

int qs_set_launch(qs_handle* h, int32_t block, int32_t grid) {
  if (!h) return QS_ERR_NULL;
  if ((block != 64 && block != 128) || grid < 0) return QS_ERR_INVALID;
  if (hipSetDevice(h->dev) != hipSuccess || hipDeviceSynchronize() != hipSuccess) return QS_ERR_HIP;
  int rc = QS_OK;
  if (h->bucketed) {
    if (block != h->item_bs) rc = build_items(h, block);
    h->item_grid = grid;
  } else if (block != h->bs) {
    if (h->uniform_n > 64 || block % std::max(h->uniform_n, 1) != 0) return QS_ERR_INVALID;
    rc = build_table(h, block);
  }
  return rc;
}

int qs_set_partner_chunks(qs_handle* h, uint32_t slot_mask) {
  if (!h) return QS_ERR_NULL;
  if (slot_mask & ~kChunkable) return QS_ERR_INVALID;
  if (hipSetDevice(h->dev) != hipSuccess || hipDeviceSynchronize() != hipSuccess) return QS_ERR_HIP;
  h->chunked = slot_mask;
  return h->bucketed ? build_items(h, h->item_bs) : QS_OK;
}

int qs_launch_plan(const qs_handle* h, int32_t* plan, int32_t* n_rows) {
  if (!h || !plan || !n_rows) return QS_ERR_NULL;
  int r = 0;
  for (int k = 6; k >= 0; --k) {
    if (h->slot_swarms[k] == 0) continue;
    int32_t* row = plan + 5 * r++;
    row[0] = 1 << k;
    row[1] = h->slot_swarms[k];
    row[2] = h->bucketed && ((h->chunked & kChunkable) >> k & 1u) ? 1 : 0;
    row[3] = (int32_t)std::lround(h->slot_ns_one[k]);
    row[4] = (int32_t)std::lround(h->slot_ns_chunked[k]);
  }
  *n_rows = r;
  return QS_OK;
}

int qs_autotune(qs_handle* h, const float* d_actions, int32_t n_substeps, const float* d_goals,
                float* d_obs, int32_t* choice, void* stream) {
  if (!h || !d_actions) return QS_ERR_NULL;
  if (n_substeps < 1 || (d_goals == nullptr) != (d_obs == nullptr)) return QS_ERR_INVALID;
  if (!aligned(d_actions, 16) || (d_obs && !aligned(d_obs, 8))) return QS_ERR_ALIGN;
  if (hipSetDevice(h->dev) != hipSuccess) return QS_ERR_HIP;
  if (h->graph_mode) return QS_ERR_UNSUPPORTED;
  hipStream_t s = (hipStream_t)stream;
  // the trials must not change the simulation: every candidate starts from
  // the saved state, and the state, substep counter and sticky error word
  // are restored afterwards
  float* saved = nullptr;
  const size_t st_bytes = (size_t)qs::NSTATE * h->Qp * sizeof(float);
  if (hipMalloc((void**)&saved, st_bytes + 256) != hipSuccess) return QS_ERR_NOMEM;
  int* saved_err = reinterpret_cast<int*>(reinterpret_cast<char*>(saved) + st_bytes);
  Trial tr{h, d_actions, d_goals, d_obs, (int)n_substeps, d_obs != nullptr, s, saved, st_bytes,
           h->t, nullptr, nullptr};
  int rc = hipMemcpyAsync(saved, h->d_st, st_bytes, hipMemcpyDeviceToDevice, s) == hipSuccess &&
                   hipMemcpyAsync(saved_err, h->d_err, sizeof(int), hipMemcpyDeviceToDevice, s) ==
                       hipSuccess
               ? QS_OK : QS_ERR_HIP;
  if (rc == QS_OK && (hipEventCreate(&tr.e0) != hipSuccess || hipEventCreate(&tr.e1) != hipSuccess))
    rc = QS_ERR_HIP;
  if (rc == QS_OK) {
    if (h->bucketed) {
      BucketConfig best{h->item_bs, h->item_grid, h->chunked};
      rc = tune_buckets(tr, &best);
      if (rc == QS_OK) rc = apply(h, s, best);
    } else if (h->uniform_n > 0) {
      // uniform power-of-two swarms: workgroup size 64 or 128
      int best_bs = h->bs;
      float best_ms = 1e30f;
      for (int bs : {64, 128}) {
        if (bs % h->uniform_n != 0) continue;
        float ms = 0.f;
        if (hipStreamSynchronize(s) != hipSuccess) { rc = QS_ERR_HIP; break; }
        if (bs != h->bs && (rc = build_table(h, bs)) != QS_OK) break;
        if ((rc = tr.call(&ms)) != QS_OK) break;
        if (ms < best_ms) {
          best_ms = ms;
          best_bs = bs;
        }
      }
      if (rc == QS_OK && hipStreamSynchronize(s) != hipSuccess) rc = QS_ERR_HIP;
      if (rc == QS_OK && best_bs != h->bs) rc = build_table(h, best_bs);
    }
  }
  if (hipMemcpyAsync(h->d_st, saved, st_bytes, hipMemcpyDeviceToDevice, s) != hipSuccess ||
      hipMemcpyAsync(h->d_err, saved_err, sizeof(int), hipMemcpyDeviceToDevice, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    rc = QS_ERR_HIP;
  h->t = tr.t_saved;
  if (tr.e0) (void)hipEventDestroy(tr.e0);
  if (tr.e1) (void)hipEventDestroy(tr.e1);
  (void)hipFree(saved);
  if (rc == QS_OK && choice) {
    choice[0] = h->bucketed ? h->item_bs : h->bs;
    choice[1] = h->bucketed ? h->item_grid : h->nblk;
    choice[2] = h->bucketed ? 1 : 0;
  }
  return rc;
}

int qs_step(qs_handle* h, const float* d_actions, int32_t n_substeps, void* stream) {
  if (!h || !d_actions) return QS_ERR_NULL;
  if (n_substeps < 0) return QS_ERR_INVALID;
  if (!aligned(d_actions, 16)) return QS_ERR_ALIGN;
  if (n_substeps == 0) return QS_OK;
  return launch(h, d_actions, n_substeps, nullptr, nullptr, false, (hipStream_t)stream);
}

int qs_observe(qs_handle* h, const float* d_goals, float* d_obs, void* stream) {
  if (!h || !d_goals || !d_obs) return QS_ERR_NULL;
  if (!aligned(d_goals, 4) || !aligned(d_obs, 8)) return QS_ERR_ALIGN;
  const size_t Q = (size_t)h->Q;
  if (outputs_overlap({{d_obs, Q * h->OD * 4}}, {{d_goals, Q * 12}})) return QS_ERR_INVALID;
  return launch(h, nullptr, 0, d_goals, d_obs, true, (hipStream_t)stream);
}

int qs_step_observe(qs_handle* h, const float* d_actions, int32_t n_substeps,
                    const float* d_goals, float* d_obs, void* stream) {
  if (!h || !d_actions || !d_goals || !d_obs) return QS_ERR_NULL;
  if (n_substeps < 0) return QS_ERR_INVALID;
  if (!aligned(d_actions, 16) || !aligned(d_goals, 4) || !aligned(d_obs, 8)) return QS_ERR_ALIGN;
  const size_t Q = (size_t)h->Q;
  if (outputs_overlap({{d_obs, Q * h->OD * 4}}, {{d_actions, Q * 16}, {d_goals, Q * 12}}))
    return QS_ERR_INVALID;
  return launch(h, d_actions, n_substeps, d_goals, d_obs, true, (hipStream_t)stream);
}

int qs_set_reward_weights(qs_handle* h, const float* h_w) {
  if (!h || !h_w) return QS_ERR_NULL;
  for (int k = 0; k < 15; ++k)
    if (!finite(h_w[k])) return QS_ERR_INVALID;
  if (!(h_w[14] > 0.f)) return QS_ERR_INVALID;
  if (hipSetDevice(h->dev) != hipSuccess) return QS_ERR_HIP;
  // enqueued calls still read the previous weights from the device copy
  if (hipDeviceSynchronize() != hipSuccess) return QS_ERR_HIP;
  for (int k = 0; k < 15; ++k) h->c.rw[k] = h_w[k];
  if (hipMemcpy(h->d_c, &h->c, sizeof(Consts), hipMemcpyHostToDevice) != hipSuccess)
    return QS_ERR_HIP;
  return QS_OK;
}

int qs_step_observe_reward(qs_handle* h, const float* d_actions, int32_t n_substeps,
                           const float* d_goals, float* d_obs, float* d_reward, void* stream) {
  if (!h || !d_actions || !d_goals || !d_obs || !d_reward) return QS_ERR_NULL;
  if (n_substeps < 1) return QS_ERR_INVALID;
  if (!aligned(d_actions, 16) || !aligned(d_goals, 4) || !aligned(d_obs, 8) ||
      !aligned(d_reward, 4))
    return QS_ERR_ALIGN;
  const size_t Q = (size_t)h->Q;
  if (outputs_overlap({{d_obs, Q * h->OD * 4}, {d_reward, Q * 4}},
                      {{d_actions, Q * 16}, {d_goals, Q * 12}}))
    return QS_ERR_INVALID;
  return launch(h, d_actions, n_substeps, d_goals, d_obs, true, (hipStream_t)stream, d_reward);
}

int qs_get_state(qs_handle* h, float* d_state, uint64_t* substep_index, void* stream) {
  if (!h || !d_state) return QS_ERR_NULL;
  if (!aligned(d_state, 4)) return QS_ERR_ALIGN;
  if (hipSetDevice(h->dev) != hipSuccess) return QS_ERR_HIP;
  const long long n = (long long)h->Q * qs::NSTATE;
  const int tb = 256;
  hipLaunchKernelGGL(qs::get_state_kernel, dim3((unsigned)((n + tb - 1) / tb)), dim3(tb), 0,
                     (hipStream_t)stream, h->d_st, h->Qp, h->Q, d_state);
  if (hipGetLastError() != hipSuccess) return QS_ERR_HIP;
  if (substep_index) *substep_index = h->t;
  return QS_OK;
}

int qs_set_state(qs_handle* h, const float* d_state, uint64_t substep_index,
                 const uint8_t* d_env_mask, void* stream) {
  if (!h || !d_state) return QS_ERR_NULL;
  if (!aligned(d_state, 4)) return QS_ERR_ALIGN;
  if (hipSetDevice(h->dev) != hipSuccess) return QS_ERR_HIP;
  const long long n = (long long)h->Q * qs::NSTATE;
  const int tb = 256;
  hipLaunchKernelGGL(qs::set_state_kernel, dim3((unsigned)((n + tb - 1) / tb)), dim3(tb), 0,
                     (hipStream_t)stream, h->d_st, h->Qp, h->Q, d_state, h->d_qenv, d_env_mask);
  if (hipGetLastError() != hipSuccess) return QS_ERR_HIP;
  h->t = substep_index;
  if (h->graph_mode)
    hipLaunchKernelGGL(qs::set_counter_kernel, dim3(1), dim3(64), 0, (hipStream_t)stream, h->d_t,
                       h->d_done, (unsigned long long)substep_index);
  return hipGetLastError() == hipSuccess ? QS_OK : QS_ERR_HIP;
}

int qs_record_contacts(qs_handle* h, int32_t enable) {
  if (!h) return QS_ERR_NULL;
  h->record = enable != 0;
  return QS_OK;
}

int qs_debug_contacts(qs_handle* h, uint64_t* d_mask, void* stream) {
  if (!h || !d_mask) return QS_ERR_NULL;
  if (!aligned(d_mask, 8)) return QS_ERR_ALIGN;
  if (hipSetDevice(h->dev) != hipSuccess) return QS_ERR_HIP;
  if (hipMemcpyAsync(d_mask, h->d_contacts, (size_t)h->Q * sizeof(uint64_t),
                     hipMemcpyDeviceToDevice, (hipStream_t)stream) != hipSuccess)
    return QS_ERR_HIP;
  return QS_OK;
}

int qs_sync(qs_handle* h, void* stream) {
  if (!h) return QS_ERR_NULL;
  if (hipSetDevice(h->dev) != hipSuccess) return QS_ERR_HIP;
  hipStream_t s = (hipStream_t)stream;
  if (hipMemcpyAsync(h->h_err, h->d_err, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess)
    return QS_ERR_HIP;
  if (hipStreamSynchronize(s) != hipSuccess) return QS_ERR_HIP;
  const int bits = *h->h_err;
  if (bits != 0) {
    *h->h_err = 0;
    if (hipMemsetAsync(h->d_err, 0, sizeof(int), s) != hipSuccess) return QS_ERR_HIP;
    if (hipStreamSynchronize(s) != hipSuccess) return QS_ERR_HIP;
    return (bits & (qs::ERRBIT_STATE | qs::ERRBIT_ACTION)) ? QS_ERR_NONFINITE : QS_ERR_INVALID;
  }
  return QS_OK;
}

int qs_set_params(qs_handle* h, const float* d_params, const uint8_t* d_env_mask, void* stream) {
  if (!h || !d_params) return QS_ERR_NULL;
  if (!aligned(d_params, 4)) return QS_ERR_ALIGN;
  if (hipSetDevice(h->dev) != hipSuccess) return QS_ERR_HIP;
  const int tb = 256;
  hipLaunchKernelGGL(qs::set_params_kernel, dim3((unsigned)((h->Q + tb - 1) / tb)), dim3(tb), 0,
                     (hipStream_t)stream, h->d_par, h->Qp, h->Q, d_params, h->d_qenv, d_env_mask,
                     h->c.dt, h->c.g, h->d_err);
  return hipGetLastError() == hipSuccess ? QS_OK : QS_ERR_HIP;
}

int qs_debug_philox(uint64_t seed, uint32_t noise_stream, uint32_t draw, uint64_t substep_index,
                    uint32_t quad0, int32_t n, uint32_t* d_words, float* d_normals,
                    void* stream) {
  if (!d_words) return QS_ERR_NULL;
  if (n < 0 || noise_stream > 0xffffffu || draw > 0xffu ||
      (uint64_t)quad0 + (uint64_t)n > 0x100000000ull)
    return QS_ERR_INVALID;
  if (!aligned(d_words, 4) || (d_normals && !aligned(d_normals, 4))) return QS_ERR_ALIGN;
  if (d_normals && overlap({d_words, (size_t)n * 16}, {d_normals, (size_t)n * 16}))
    return QS_ERR_INVALID;
  if (n == 0) return QS_OK;
  const int tb = 256;
  hipLaunchKernelGGL(qs::philox_debug_kernel, dim3((unsigned)((n + tb - 1) / tb)), dim3(tb), 0,
                     (hipStream_t)stream, (uint32_t)seed, (uint32_t)(seed >> 32), noise_stream,
                     draw, (unsigned long long)substep_index, quad0, (int)n, d_words, d_normals);
  return hipGetLastError() == hipSuccess ? QS_OK : QS_ERR_HIP;
}

int qs_rollout(qs_handle* h, const float* d_actions, int32_t n_calls, int32_t n_substeps,
               int32_t ckpt_every, float* d_ckpt, float* d_penalty, float beta, void* stream) {
  if (!h || !d_actions) return QS_ERR_NULL;
  if (n_calls < 0 || n_substeps < 0) return QS_ERR_INVALID;
  if (d_ckpt && ckpt_every < 1) return QS_ERR_INVALID;
  if (d_penalty && !(beta > 0.f && std::isfinite(beta))) return QS_ERR_INVALID;
  if (!aligned(d_actions, 16) || (d_ckpt && !aligned(d_ckpt, 4)) ||
      (d_penalty && !aligned(d_penalty, 4)))
    return QS_ERR_ALIGN;
  if (n_calls == 0 || n_substeps == 0) return QS_OK;
  {
    const size_t Q = (size_t)h->Q, n_ck = d_ckpt ? (n_calls + ckpt_every - 1) / ckpt_every : 0;
    if (outputs_overlap({{d_ckpt, n_ck * qs::NSTATE * Q * 4}, {d_penalty, Q * 4}},
                        {{d_actions, (size_t)n_calls * Q * 16}}))
      return QS_ERR_INVALID;
  }
  if (hipSetDevice(h->dev) != hipSuccess) return QS_ERR_HIP;
  hipStream_t s = (hipStream_t)stream;
  if (d_penalty)
    dispatch<RollF, true>(h, d_actions, (int)n_calls, (int)n_substeps, d_ckpt, (int)ckpt_every,
                          d_penalty, beta, s);
  else
    dispatch<RollF, false>(h, d_actions, (int)n_calls, (int)n_substeps, d_ckpt,
                           (int)std::max(ckpt_every, 1), d_penalty, beta, s);
  if (hipGetLastError() != hipSuccess) return QS_ERR_HIP;
  h->t += (uint64_t)n_calls * (uint64_t)n_substeps;
  return QS_OK;
}

int qs_rollout_backward(qs_handle* h, const float* d_actions, int32_t n_calls,
                        int32_t n_substeps, int32_t ckpt_every, const float* d_ckpt,
                        uint64_t substep_index0, float* d_gstate, const float* d_gpenalty,
                        float beta, float* d_gactions, float* d_gparams, void* stream) {
  if (!h || !d_actions || !d_ckpt || !d_gstate || !d_gactions || !d_gparams) return QS_ERR_NULL;
  if (n_calls < 0 || n_substeps < 0 || ckpt_every < 1) return QS_ERR_INVALID;
  if (h->c.flags & qs::F_DOWNWASH) return QS_ERR_UNSUPPORTED;
  if (d_gpenalty && !(beta > 0.f && std::isfinite(beta))) return QS_ERR_INVALID;
  if (!aligned(d_actions, 16) || !aligned(d_gactions, 16) || !aligned(d_ckpt, 4) ||
      !aligned(d_gstate, 4) || !aligned(d_gparams, 4) || (d_gpenalty && !aligned(d_gpenalty, 4)))
    return QS_ERR_ALIGN;
  {
    const size_t Q = (size_t)h->Q, nc = (size_t)std::max(n_calls, 0);
    const size_t n_ck = (nc + ckpt_every - 1) / ckpt_every;
    if (outputs_overlap({{d_gactions, nc * Q * 16}, {d_gparams, Q * 24}, {d_gstate, Q * 108}},
                        {{d_actions, nc * Q * 16}, {d_ckpt, n_ck * qs::NSTATE * Q * 4},
                         {d_gpenalty, Q * 4}}))
      return QS_ERR_INVALID;
  }
  if (n_calls == 0 || n_substeps == 0) return QS_OK;
  if (hipSetDevice(h->dev) != hipSuccess) return QS_ERR_HIP;
  int rc = ensure_adjoint_scratch(h);
  if (rc != QS_OK) return rc;
  hipStream_t s = (hipStream_t)stream;
  convert(d_gstate, h->d_lam, h->Q, qs::NSTATE, false, false, s);
  hipLaunchKernelGGL(qs::fill_kernel, dim3((unsigned)((6LL * h->Q + 255) / 256)), dim3(256), 0, s,
                     h->d_gpar, 6LL * h->Q, 0.0f);
  // segments per chunk: as many as fit the tape budget (also the recompute
  // grid's y extent, at most 65535), at least one
  const int nseg = (n_calls + ckpt_every - 1) / ckpt_every;
  const size_t seg = segment_tape_floats(h, n_calls, n_substeps, ckpt_every);
  const size_t fit = tape_budget() / (seg * sizeof(float));
  const int G = (int)std::max<size_t>(1, std::min<size_t>({(size_t)nseg, fit, (size_t)65535}));
  rc = grow(&h->d_tape, &h->tape_cap, (size_t)G * seg);
  if (rc != QS_OK) return rc;
  const AdjScratch sc{h->d_tape, h->d_lam, h->d_gpar};
  rc = run_adjoint(h, sc, G, d_actions, n_calls, n_substeps, ckpt_every, d_ckpt, substep_index0,
                   d_gpenalty, beta, d_gactions, s);
  if (rc != QS_OK) return rc;
  convert(h->d_lam, d_gstate, h->Q, qs::NSTATE, true, false, s);
  convert(h->d_gpar, d_gparams, h->Q, 6, true, true, s);
  return hipGetLastError() == hipSuccess ? QS_OK : QS_ERR_HIP;
}

int qs_step_backward(qs_handle* h, const float* d_state_in, const float* d_actions,
                     int32_t n_substeps, uint64_t substep_index, const float* d_gstate_out,
                     float* d_gstate_in, float* d_gactions, float* d_gparams, void* stream) {
  int rc = check_step_backward(h, d_state_in, d_actions, n_substeps, d_gstate_out, d_gstate_in,
                               d_gactions, d_gparams);
  if (rc != QS_OK) return rc;
  if (hipSetDevice(h->dev) != hipSuccess) return QS_ERR_HIP;
  rc = ensure_adjoint_scratch(h);
  if (rc == QS_OK && n_substeps > 0)
    rc = grow(&h->d_tape, &h->tape_cap, segment_tape_floats(h, 1, n_substeps, 1));
  if (rc != QS_OK) return rc;
  const AdjScratch sc{h->d_tape, h->d_lam, h->d_gpar};
  return step_backward_run(h, sc, h->d_ck1, d_state_in, d_actions, n_substeps, substep_index,
                           d_gstate_out, d_gstate_in, d_gactions, d_gparams, (hipStream_t)stream);
}

int qs_step_backward_noalloc(qs_handle* h, const float* d_state_in, const float* d_actions,
                             int32_t n_substeps, uint64_t substep_index,
                             const float* d_gstate_out, float* d_gstate_in, float* d_gactions,
                             float* d_gparams, void* stream) {
  int rc = check_step_backward(h, d_state_in, d_actions, n_substeps, d_gstate_out, d_gstate_in,
                               d_gactions, d_gparams);
  if (rc != QS_OK) return rc;
  // parts of the fixed scratch, each rounded up to 64 floats (256 bytes)
  auto part = [](size_t n) { return (n + 63) / 64 * 64; };
  const size_t Q = (size_t)h->Q;
  const size_t n_ck = part(qs::NSTATE * Q), n_lam = part(qs::NSTATE * Q), n_g = part(6 * Q);
  const size_t n_tape = n_substeps > 0 ? part(segment_tape_floats(h, 1, n_substeps, 1)) : 0;
  if (n_ck + n_lam + n_g + n_tape > kNoAllocScratchFloats) return QS_ERR_TOO_LARGE;
  if (hipSetDevice(h->dev) != hipSuccess) return QS_ERR_HIP;
  float* base = nullptr;
  rc = noalloc_scratch(h->dev, &base);
  if (rc != QS_OK) return rc;
  const AdjScratch sc{base + n_ck + n_lam + n_g, base + n_ck, base + n_ck + n_lam};
  return step_backward_run(h, sc, base, d_state_in, d_actions, n_substeps, substep_index,
                           d_gstate_out, d_gstate_in, d_gactions, d_gparams, (hipStream_t)stream);
}

const char* qs_error_string(int code) {
  switch (code) {
    case QS_OK: return "ok";
    case QS_ERR_NULL: return "a required pointer is NULL";
    case QS_ERR_INVALID: return "a count, size or constant is out of range";
    case QS_ERR_ENV_SIZE: return "env_offsets is not CSR or a swarm has 0 or more than 64 quads";
    case QS_ERR_HIP: return "a HIP runtime call failed";
    case QS_ERR_NONFINITE: return "a non-finite action or state value was produced on the device";
    case QS_ERR_NOMEM: return "allocation failed";
    case QS_ERR_ALIGN: return "a device pointer is misaligned";
    case QS_ERR_UNSUPPORTED: return "request not supported by this build";
    case QS_ERR_TOO_LARGE:
      return "request exceeds the fixed scratch of the allocation-free entry point";
    default: return "unknown error code";
  }
}

}  // extern "C"
