// Pipelines: the per-block sequence of one plan over many SNP blocks
// (clak_pipeline_*), and several plans (cohorts) in one submission
// (clak_batch_*), the streaming of the X_R blocks of section 3.
//
// Every schedule runs on three streams of its own, whatever the number of
// plans: a side stream for the genotype ingest and two compute streams.
// Work goes in rounds: round r takes block r of every plan that has one.
// Each plan's block of round r uses that plan's workspace slot r % 3, which
// is refilled once round r - 3 has finished, so the ingest runs up to two
// rounds ahead of the rotation and the memory-bound ingest overlaps the
// MFMA-bound kernels without waiting on the round just before.  Rounds
// alternate between the two compute streams, so the kernels of round r + 1
// start while the last work-groups of round r drain (every buffer a round
// writes belongs to its slots or to its own outputs).  The three streams and
// the launch stream stay within the four hardware queues a process gets.
//
// A round of several plans is one launch per kernel (ingest, rotation,
// digit encoding, grid contraction) over all of them when their kernels
// agree (batch_compatible: mixed precision, several traits, the same
// p_L <= 3 and output form): each launch's grid is the plans' grids one after
// the other, the plan with the most work per block first (cost
// n (2 n + 10 (p_L + 2) t) per SNP, the rotation's and the grid's products),
// so that the smaller plans' work-groups fill in behind it.  Other plans run
// their per-block launches in the same rounds and order.
//
// With the serial stage profiler on, one compute stream serves every round
// and the ingest runs on it too, so that no two kernels overlap; a batched
// launch is timed once, under the round's first plan.  A launch enqueues the
// whole schedule from the host, forked from the launch stream by an event and
// joined back to it.
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <functional>
#include <numeric>
#include <vector>

#include "clak_internal.hpp"

using namespace clak;

namespace {

constexpr int NCOMPUTE = 2;  // compute streams of a schedule

struct Schedule {
  std::vector<Plan*> plans;
  std::vector<int64_t> first, count;  // plan k: blocks [first[k], first[k] + count[k]) of `blocks`
  std::vector<clak_block> blocks;
  std::vector<std::vector<int>> rounds;  // plans of round r, costliest first
  bool batched = false;                  // one launch per kernel and round over all plans
  int g_dtype = CLAK_G_U8, out_dtype = CLAK_OUT_F32;
  hipStream_t s_in = nullptr, s_main[NCOMPUTE] = {};
  hipEvent_t fork = nullptr, joined_in = nullptr, joined_main[NCOMPUTE] = {};
  hipEvent_t ingested[NSLOTS] = {}, done[NSLOTS] = {};
};

void release(Schedule* g) {
  if (!g) return;
  for (int k = 0; k < NCOMPUTE; ++k)
    if (g->s_main[k]) (void)hipStreamSynchronize(g->s_main[k]);
  if (g->s_in) (void)hipStreamSynchronize(g->s_in);
  for (int k = 0; k < NSLOTS; ++k) {
    if (g->ingested[k]) (void)hipEventDestroy(g->ingested[k]);
    if (g->done[k]) (void)hipEventDestroy(g->done[k]);
  }
  for (int k = 0; k < NCOMPUTE; ++k) {
    if (g->joined_main[k]) (void)hipEventDestroy(g->joined_main[k]);
    if (g->s_main[k]) (void)hipStreamDestroy(g->s_main[k]);
  }
  if (g->joined_in) (void)hipEventDestroy(g->joined_in);
  if (g->fork) (void)hipEventDestroy(g->fork);
  if (g->s_in) (void)hipStreamDestroy(g->s_in);
  delete g;
}

#define CK(expr, what)                                                                      \
  do {                                                                                      \
    hipError_t e_ = (expr);                                                                 \
    if (e_ != hipSuccess) return fail(CLAK_E_DEVICE, "%s: %s: %s", what, #expr, hipGetErrorString(e_)); \
  } while (0)

// MFMA work of one SNP of a plan's block: rotation (n^2) and grid sums
// (10 digit products of p_L + 2 sums per trait).
double plan_cost(const Plan* p) { return (double)p->n * (2.0 * p->n + 10.0 * (p->pL + 2) * p->t); }

bool serial_profile(const Schedule& g) {
  for (Plan* p : g.plans)
    if (p->profiling == CLAK_PROFILE_SERIAL) return true;
  return false;
}

clak_status make_schedule(Schedule* g, const std::vector<Plan*>& plans, const std::vector<int64_t>& n_blocks,
                          const clak_block* blocks, int g_dtype, int out_dtype, const char* what) {
  g->plans = plans;
  g->g_dtype = g_dtype;
  g->out_dtype = out_dtype;
  int64_t total = 0;
  for (int64_t c : n_blocks) {
    g->first.push_back(total);
    g->count.push_back(c);
    total += c;
  }
  if (blocks) g->blocks.assign(blocks, blocks + total);
  // rounds, costliest plan first
  std::vector<int> order(plans.size());
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(),
                   [&](int a, int b) { return plan_cost(plans[a]) > plan_cost(plans[b]); });
  const int64_t nr = *std::max_element(n_blocks.begin(), n_blocks.end());
  g->rounds.resize((size_t)nr);
  for (int64_t r = 0; r < nr; ++r)
    for (int k : order)
      if (r < n_blocks[k]) g->rounds[r].push_back(k);
  g->batched = plans.size() > 1 && plans.size() <= (size_t)MAX_BATCH;
  for (size_t k = 1; k < plans.size() && g->batched; ++k) g->batched = batch_compatible(*plans[0], *plans[k]);
  CK(hipEventCreateWithFlags(&g->fork, hipEventDisableTiming), what);
  CK(hipEventCreateWithFlags(&g->joined_in, hipEventDisableTiming), what);
  CK(hipStreamCreateWithFlags(&g->s_in, hipStreamNonBlocking), what);
  for (int q = 0; q < NCOMPUTE; ++q) {
    CK(hipStreamCreateWithFlags(&g->s_main[q], hipStreamNonBlocking), what);
    CK(hipEventCreateWithFlags(&g->joined_main[q], hipEventDisableTiming), what);
  }
  for (int q = 0; q < NSLOTS; ++q) {
    CK(hipEventCreateWithFlags(&g->ingested[q], hipEventDisableTiming), what);
    CK(hipEventCreateWithFlags(&g->done[q], hipEventDisableTiming), what);
  }
  return CLAK_OK;
}

// Brackets one launch with the stage profiler's events on stream s under plan p.
hipError_t timed(Plan* p, int stage, hipStream_t s, const std::function<hipError_t()>& launch) {
  if (!p->profiling) return launch();
  hipEvent_t a = take_event(p), b = take_event(p);
  if (!a || !b) return hipErrorOutOfMemory;
  hipError_t e = hipEventRecord(a, s);
  if (e == hipSuccess) e = launch();
  if (e == hipSuccess) e = hipEventRecord(b, s);
  p->pending.push_back({stage, a, b});
  return e;
}

// Enqueues round r: ingest on the side stream (after round r - 3 has released
// the slots), the rest on the round's compute stream.  get(k) gives plan k's
// block of this round.
clak_status enqueue_round(Schedule* g, int64_t r, const std::function<clak_status(int, clak_block*)>& get,
                          const char* what) {
  const int slot = (int)(r % NSLOTS);
  const bool serial = serial_profile(*g);
  const hipStream_t sm = serial ? g->s_main[0] : g->s_main[r % NCOMPUTE];
  const hipStream_t si = serial ? sm : g->s_in;
  if (r >= NSLOTS) CK(hipStreamWaitEvent(si, g->done[slot], 0), what);
  const std::vector<int>& plans = g->rounds[(size_t)r];
  if (!g->batched) {
    for (size_t q = 0; q < plans.size(); ++q) {
      Plan* p = g->plans[plans[q]];
      clak_block B{};
      clak_status s = get(plans[q], &B);
      if (s) return s;
      // each plan's compute waits for its own ingest (the event is re-recorded per plan)
      s = enqueue_block(p, slot, si, sm, g->ingested[slot], B.m_blk, B.G, g->g_dtype, B.ldg,
                        cell_out(B.b, B.se, B.pval, B.flags, B.ldo, g->out_dtype));
      if (s) return s;
    }
  } else {
    BatchItem items[MAX_BATCH];
    const int n = (int)plans.size();
    for (int q = 0; q < n; ++q) {
      clak_block B{};
      clak_status s = get(plans[q], &B);
      if (s) return s;
      items[q].p = g->plans[plans[q]];
      items[q].slot = slot;
      items[q].m_blk = B.m_blk;
      items[q].G = B.G;
      items[q].ldg = B.ldg;
      items[q].out = cell_out(B.b, B.se, B.pval, B.flags, B.ldo, g->out_dtype);
    }
    Plan* p0 = items[0].p;  // the batched launches are timed under the round's first plan
    CK(timed(p0, CLAK_STAGE_INGEST, si, [&] { return launch_ingest_batch(items, n, g->g_dtype, si); }), what);
    CK(hipEventRecord(g->ingested[slot], si), what);
    if (si != sm) CK(hipStreamWaitEvent(sm, g->ingested[slot], 0), what);
    CK(timed(p0, CLAK_STAGE_ROTATE, sm, [&] { return launch_rotate_batch(items, n, sm); }), what);
    CK(timed(p0, CLAK_STAGE_ENCODE, sm, [&] { return launch_encode_batch(items, n, sm); }), what);
    CK(timed(p0, CLAK_STAGE_GRID, sm, [&] { return launch_grid_batch(items, n, sm); }), what);
  }
  CK(hipEventRecord(g->done[slot], sm), what);
  return CLAK_OK;
}

// Forks the schedule's streams from `origin`.
clak_status fork_from(Schedule* g, hipStream_t origin, const char* what) {
  CK(hipEventRecord(g->fork, origin), what);
  CK(hipStreamWaitEvent(g->s_in, g->fork, 0), what);
  for (int q = 0; q < NCOMPUTE; ++q) CK(hipStreamWaitEvent(g->s_main[q], g->fork, 0), what);
  return CLAK_OK;
}

// Joins the schedule's streams back to `origin`.
clak_status join_to(Schedule* g, hipStream_t origin, const char* what) {
  CK(hipEventRecord(g->joined_in, g->s_in), what);
  CK(hipStreamWaitEvent(origin, g->joined_in, 0), what);
  for (int q = 0; q < NCOMPUTE; ++q) {
    CK(hipEventRecord(g->joined_main[q], g->s_main[q]), what);
    CK(hipStreamWaitEvent(origin, g->joined_main[q], 0), what);
  }
  return CLAK_OK;
}

// Enqueues the whole schedule, forked from and joined back to `origin`.
clak_status run_schedule(Schedule* g, hipStream_t origin, const char* what) {
  clak_status s = fork_from(g, origin, what);
  if (s) return s;
  for (int64_t r = 0; r < (int64_t)g->rounds.size(); ++r) {
    s = enqueue_round(g, r, [&](int k, clak_block* B) {
      *B = g->blocks[(size_t)(g->first[k] + r)];
      return CLAK_OK;
    }, what);
    if (s) return s;
  }
  return join_to(g, origin, what);
}

clak_status check_blocks(Plan* p, int64_t n, const clak_block* blocks, int g_dtype, int out_dtype) {
  for (int64_t b = 0; b < n; ++b) {
    const clak_block& B = blocks[b];
    clak_status s = validate_block(p, B.m_blk, B.G, g_dtype, B.ldg, B.b, B.se, out_dtype, B.ldo, B.flags, B.pval);
    if (s) return s;
  }
  return CLAK_OK;
}

}  // namespace

namespace clak {

// Streams n_blocks blocks of one plan through the slot ring and compute
// streams of a pipeline, asking `get` for each block just before it is
// enqueued (it may wait, e.g. for a file read) and calling `after` with the
// ingest stream once the block's ingest is enqueued (e.g. to record when its
// input buffer may be reused).  Forked from and joined back to the plan's
// stream; returns after the plan's stream has finished the work.
clak_status stream_blocks(Plan* p, int64_t n_blocks, int g_dtype, int out_dtype,
                          const std::function<clak_status(int64_t, clak_block*)>& get,
                          const std::function<clak_status(int64_t, hipStream_t)>& after, const char* what) {
  Schedule* g = new Schedule();
  clak_status s = make_schedule(g, {p}, {n_blocks}, nullptr, g_dtype, out_dtype, what);
  auto done = [&](clak_status st) {
    release(g);
    return st;
  };
  if (s) return done(s);
  if ((s = fork_from(g, p->stream, what))) return done(s);
  clak_status result = CLAK_OK;
  for (int64_t j = 0; j < n_blocks && result == CLAK_OK; ++j) {
    result = enqueue_round(g, j, [&](int, clak_block* B) {
      clak_status st = get(j, B);
      if (st) return st;
      return validate_block(p, B->m_blk, B->G, g_dtype, B->ldg, B->b, B->se, out_dtype, B->ldo, B->flags, B->pval);
    }, what);
    if (!result) result = after(j, serial_profile(*g) ? g->s_main[0] : g->s_in);
  }
  // join everything enqueued so far back to the plan's stream and wait for it
  clak_status js = join_to(g, p->stream, what);
  if (!js && hipStreamSynchronize(p->stream) != hipSuccess) js = fail(CLAK_E_DEVICE, "%s: synchronise", what);
  return done(result ? result : js);
}

// The launch parameters of the mixed path chosen by timing a pipelined pass
// over the caller's blocks (all on the plan's stream through the pipeline's
// streams, as clak_pipeline_launch runs them) for each candidate: the
// rotation's tile configuration and XCD row groups first (with the grid at
// its built-in choice), then the grid kernel and its XCD grouping (the
// selection rule is at `choose` below).  Every candidate computes the same bits, so the caller's outputs hold the result
// whichever is chosen (the last pass runs with the choice).  A cache file
// line per shape (device architecture, n_pad, p_L, t, block size, number of
// blocks, flags) replaces the timing when present.
clak_status autotune_blocks(Plan* p, int64_t n_blocks, const clak_block* blocks, int g_dtype, int out_dtype,
                            const char* cache_path, const char* what) {
  if (n_blocks < 1 || !blocks) return fail(CLAK_E_ARG, "%s: need at least one block", what);
  clak_status s = check_blocks(p, n_blocks, blocks, g_dtype, out_dtype);
  if (s) return s;
  Schedule* g = new Schedule();
  s = make_schedule(g, {p}, {n_blocks}, blocks, g_dtype, out_dtype, what);
  auto done = [&](clak_status st) {
    release(g);
    return st;
  };
  if (s) return done(s);
  const int prof = p->profiling;
  p->profiling = CLAK_PROFILE_OFF;
  auto finish = [&](clak_status st) {
    p->profiling = prof;
    if (!st) st = run_schedule(g, p->stream, what);  // the outputs, with the chosen parameters
    return done(st);
  };
  if (p->prec != CLAK_PREC_MIXED) return finish(CLAK_OK);  // nothing to tune on the FP64 path
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, p->device) != hipSuccess) return finish(fail(CLAK_E_DEVICE, "%s: device", what));
  char arch[64];
  std::snprintf(arch, sizeof arch, "%s", prop.gcnArchName);
  for (char* c = arch; *c; ++c)
    if (*c == ' ' || *c == ':') *c = '_';
  char key[256];
  std::snprintf(key, sizeof key, "%s n_pad=%lld p_L=%lld t=%lld m_blk=%lld blocks=%lld flags=0x%x", arch,
                (long long)p->n_pad, (long long)p->pL, (long long)p->t, (long long)blocks[0].m_blk,
                (long long)n_blocks, p->flags);
  if (cache_path) {
    if (FILE* f = std::fopen(cache_path, "r")) {
      char line[512];
      bool found = false;
      while (!found && std::fgets(line, sizeof line, f)) {
        const size_t kl = std::strlen(key);
        if (std::strncmp(line, key, kl) != 0 || line[kl] != ' ') continue;
        int cfg = 0, rg = 0, tt = 0, xt = 0;
        if (std::sscanf(line + kl, " rot_cfg=%d rot_rg=%d grid_tt=%d grid_xt=%d", &cfg, &rg, &tt, &xt) == 4 &&
            clak_plan_set_tuning(reinterpret_cast<clak_plan_t>(p), cfg, rg, tt, xt) == CLAK_OK)
          found = true;
      }
      std::fclose(f);
      if (found) return finish(CLAK_OK);
    }
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    return finish(fail(CLAK_E_DEVICE, "%s: event creation failed", what));
  }
  clak_status err = CLAK_OK;
  auto measure = [&]() -> float {
    float best = 1e30f;
    for (int rep = 0; rep < 4 && !err; ++rep) {
      if (hipEventRecord(e0, p->stream) != hipSuccess) err = fail(CLAK_E_DEVICE, "%s: event", what);
      if (!err) err = run_schedule(g, p->stream, what);
      if (!err && (hipEventRecord(e1, p->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess))
        err = fail(CLAK_E_DEVICE, "%s: timing", what);
      float ms = 0.0f;
      if (!err && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) err = fail(CLAK_E_DEVICE, "%s: timing", what);
      if (!err && rep > 0 && ms < best) best = ms;  // the first pass warms caches and code
    }
    return best;
  };
  // One family of candidates (candidate 0 is the built-in choice): every
  // candidate is timed once, then the built-in one and the three fastest
  // others again in three interleaved rounds, each keeping its best time.  The
  // fastest finalist wins only if it beats the built-in choice by MARGIN; of
  // the finalists within TIE of the winner the first in candidate order is
  // taken, so that near-equal candidates do not trade places from run to run.
  constexpr float MARGIN = 0.98f, TIE = 1.01f;
  auto choose = [&](const std::vector<std::pair<int, int>>& cand, auto set) -> std::pair<int, int> {
    std::vector<float> ms(cand.size(), 1e30f);
    for (size_t c = 0; c < cand.size() && !err; ++c) {
      set(cand[c]);
      ms[c] = measure();
    }
    std::vector<size_t> order(cand.size());
    for (size_t c = 0; c < order.size(); ++c) order[c] = c;
    std::stable_sort(order.begin() + 1, order.end(), [&](size_t a, size_t b) { return ms[a] < ms[b]; });
    order.resize(std::min<size_t>(order.size(), 4));
    for (int round = 0; round < 3 && !err; ++round)
      for (size_t c : order) {
        set(cand[c]);
        ms[c] = std::min(ms[c], measure());
      }
    size_t win = 0;
    for (size_t c : order)
      if (ms[c] < ms[win]) win = c;
    if (!(ms[win] < MARGIN * ms[0])) return cand[0];
    size_t pick = win;
    for (size_t c : order)
      if (c < pick && ms[c] <= TIE * ms[win] && ms[c] < MARGIN * ms[0]) pick = c;
    return cand[pick];
  };
  const int pow2[4] = {1, 2, 4, 8};
  p->rot_cfg = p->rot_rg = p->grid_tt = p->grid_xt = 0;
  // rotation: tile configuration x XCD row groups
  std::vector<std::pair<int, int>> cand = {{0, 0}};
  for (int cfg = 0; cfg < ROT_CONFIGS; ++cfg)
    for (int rg : pow2)
      if (cfg != 10 || rg == 1) cand.push_back({cfg, rg});  // the Z-resident kernel has its own XCD map
  const auto rot = choose(cand, [&](std::pair<int, int> c) { p->rot_cfg = c.first, p->rot_rg = c.second; });
  p->rot_cfg = rot.first;
  p->rot_rg = rot.second;
  // grid (several traits): the ring kernel's XCD grouping, the two-stage
  // kernel's trait tile and XCD trait groups (no variants for the full
  // vector with p_L > 3)
  if (!p->fused_t1 && (p->pL <= 3 || !(p->flags & CLAK_OUT_FULL)) && !err) {
    cand.assign(1, {0, 0});
    for (int tt : {0, 32, 64})
      for (int xt : pow2)
        if (tt != 0 || p->pL <= 3) cand.push_back({tt, xt});  // the ring kernel takes p_L <= 3
    const auto grid = choose(cand, [&](std::pair<int, int> c) { p->grid_tt = c.first, p->grid_xt = c.second; });
    p->grid_tt = grid.first;
    p->grid_xt = grid.second;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (err) return finish(err);
  if (cache_path) {
    if (FILE* f = std::fopen(cache_path, "a")) {
      std::fprintf(f, "%s rot_cfg=%d rot_rg=%d grid_tt=%d grid_xt=%d\n", key, p->rot_cfg, p->rot_rg, p->grid_tt,
                   p->grid_xt);
      std::fclose(f);
    }
  }
  return finish(CLAK_OK);
}

}  // namespace clak

struct clak_pipeline_s {
  Schedule* run;
  Plan* plan;
};

struct clak_batch_s {
  Schedule* run;
};

extern "C" {

clak_status clak_pipeline_create(clak_pipeline_t* out, clak_plan_t plan, int64_t n_blocks, const clak_block* blocks,
                                 int g_dtype, int out_dtype) {
  if (!out) return fail(CLAK_E_ARG, "pipeline_create: null output pointer");
  *out = nullptr;
  Plan* p = reinterpret_cast<Plan*>(plan);
  clak_status s = need_state(p, ST_READY, "pipeline_create");
  if (s) return s;
  if (n_blocks < 1 || !blocks) return fail(CLAK_E_ARG, "pipeline_create: need at least one block");
  s = check_blocks(p, n_blocks, blocks, g_dtype, out_dtype);
  if (s) return s;
  Schedule* g = new Schedule();
  s = make_schedule(g, {p}, {n_blocks}, blocks, g_dtype, out_dtype, "pipeline_create");
  if (s) {
    release(g);
    return s;
  }
  *out = new clak_pipeline_s{g, p};
  return ok();
}

clak_status clak_pipeline_launch(clak_pipeline_t pipe) {
  if (!pipe) return fail(CLAK_E_ARG, "pipeline_launch: null pipeline");
  clak_status s = need_state(pipe->plan, ST_READY, "pipeline_launch");
  if (s) return s;
  s = run_schedule(pipe->run, pipe->plan->stream, "pipeline_launch");
  if (s) return s;
  return ok();
}

clak_status clak_pipeline_destroy(clak_pipeline_t pipe) {
  if (!pipe) return fail(CLAK_E_ARG, "pipeline_destroy: null pipeline");
  release(pipe->run);
  delete pipe;
  return ok();
}

clak_status clak_autotune_pipeline(clak_plan_t plan, int64_t n_blocks, const clak_block* blocks, int g_dtype,
                                   int out_dtype, const char* cache_path) {
  Plan* p = reinterpret_cast<Plan*>(plan);
  clak_status s = need_state(p, ST_READY, "autotune_pipeline");
  if (s) return s;
  s = autotune_blocks(p, n_blocks, blocks, g_dtype, out_dtype, cache_path, "autotune_pipeline");
  return s ? s : ok();
}

clak_status clak_batch_create(clak_batch_t* out, int n_plans, const clak_plan_t* plans, const int64_t* n_blocks,
                              const clak_block* blocks, int g_dtype, int out_dtype) {
  if (!out) return fail(CLAK_E_ARG, "batch_create: null output pointer");
  *out = nullptr;
  if (n_plans < 1 || !plans || !n_blocks || !blocks) return fail(CLAK_E_ARG, "batch_create: empty batch");
  std::vector<Plan*> ps;
  std::vector<int64_t> nb;
  int64_t off = 0;
  for (int k = 0; k < n_plans; ++k) {
    Plan* p = reinterpret_cast<Plan*>(plans[k]);
    clak_status s = need_state(p, ST_READY, "batch_create");
    if (s) return s;
    for (Plan* q : ps)
      if (q == p) return fail(CLAK_E_ARG, "batch_create: plan %d listed twice", k);
    if (!ps.empty() && p->device != ps[0]->device) return fail(CLAK_E_ARG, "batch_create: plans on different devices");
    if (n_blocks[k] < 1) return fail(CLAK_E_ARG, "batch_create: plan %d has no blocks", k);
    s = check_blocks(p, n_blocks[k], blocks + off, g_dtype, out_dtype);
    if (s) return s;
    ps.push_back(p);
    nb.push_back(n_blocks[k]);
    off += n_blocks[k];
  }
  Schedule* g = new Schedule();
  clak_status s = make_schedule(g, ps, nb, blocks, g_dtype, out_dtype, "batch_create");
  if (s) {
    release(g);
    return s;
  }
  *out = new clak_batch_s{g};
  return ok();
}

clak_status clak_batch_launch(clak_batch_t batch, void* hip_stream) {
  if (!batch) return fail(CLAK_E_ARG, "batch_launch: null batch");
  for (Plan* p : batch->run->plans) {
    clak_status s = need_state(p, ST_READY, "batch_launch");
    if (s) return s;
  }
  clak_status s = run_schedule(batch->run, (hipStream_t)hip_stream, "batch_launch");
  if (s) return s;
  return ok();
}

clak_status clak_batch_get_info(clak_batch_t batch, int* batched, int64_t* rounds, int* streams) {
  if (!batch) return fail(CLAK_E_ARG, "batch_get_info: null batch");
  if (batched) *batched = batch->run->batched ? 1 : 0;
  if (rounds) *rounds = (int64_t)batch->run->rounds.size();
  if (streams) *streams = 1 + NCOMPUTE;
  return ok();
}

clak_status clak_batch_destroy(clak_batch_t batch) {
  if (!batch) return fail(CLAK_E_ARG, "batch_destroy: null batch");
  release(batch->run);
  delete batch;
  return ok();
}

}  // extern "C"
