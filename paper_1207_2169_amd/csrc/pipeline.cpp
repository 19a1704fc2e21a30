// Pipelines: the per-block sequence of one plan over many SNP blocks
// (clak_pipeline_*), and several plans (cohorts) in one submission
// (clak_batch_*).
//
// Within a plan, blocks go round the NSLOTS (three) workspace slots: block b
// is ingested on a side stream into slot b % 3 once block b - 3, the previous
// user of that slot, has finished, so the ingest runs up to two blocks ahead
// of the rotation and the memory-bound ingest overlaps the MFMA-bound
// rotation without waiting on the block just before.  Blocks alternate
// between two compute streams, so the kernels of block b + 1 start while the
// last work-groups of block b drain (every buffer a block writes belongs to
// its slot or to its own outputs; a slot is reused only after the wait on its
// last user, whichever stream ran it).  Two compute streams and the side
// stream, with the launch stream, stay within four hardware queues.  With the
// stage profiler on, one compute stream serves every block so that
// per-kernel times are not shared.  A launch enqueues the whole schedule from
// the host: the side and compute streams are forked from the launch stream by
// an event and joined back to it at the end, so the launch stream sees the
// pipeline as one unit of work.
// Cohorts of a batch get their own streams and run concurrently.
#include <functional>
#include <vector>

#include "clak_internal.hpp"

using namespace clak;

namespace {

constexpr int NCOMPUTE = 2;  // compute streams per plan

struct PlanStreams {
  Plan* plan = nullptr;
  hipStream_t s_main[NCOMPUTE] = {}, s_in = nullptr;
  hipEvent_t ingested[NSLOTS] = {};
  hipEvent_t done[NSLOTS] = {};
  hipEvent_t joined_in = nullptr, joined_main[NCOMPUTE] = {};
  int64_t first = 0, count = 0;  // blocks [first, first + count) of the block list
};

struct Schedule {
  std::vector<PlanStreams> ps;
  std::vector<clak_block> blocks;
  int g_dtype = CLAK_G_U8, out_dtype = CLAK_OUT_F32;
  hipEvent_t fork = nullptr;
};

void release(Schedule* g) {
  if (!g) return;
  for (auto& c : g->ps) {
    for (int k = 0; k < NCOMPUTE; ++k)
      if (c.s_main[k]) (void)hipStreamSynchronize(c.s_main[k]);
    if (c.s_in) (void)hipStreamSynchronize(c.s_in);
    for (int k = 0; k < NSLOTS; ++k) {
      if (c.ingested[k]) (void)hipEventDestroy(c.ingested[k]);
      if (c.done[k]) (void)hipEventDestroy(c.done[k]);
    }
    for (int k = 0; k < NCOMPUTE; ++k) {
      if (c.joined_main[k]) (void)hipEventDestroy(c.joined_main[k]);
      if (c.s_main[k]) (void)hipStreamDestroy(c.s_main[k]);
    }
    if (c.joined_in) (void)hipEventDestroy(c.joined_in);
    if (c.s_in) (void)hipStreamDestroy(c.s_in);
  }
  if (g->fork) (void)hipEventDestroy(g->fork);
  delete g;
}

// The compute stream of block j.  While the serial stage profiler runs,
// every block uses one, so that each kernel's bracketed time is its own
// (consecutive blocks do not overlap).
hipStream_t compute_stream(const Plan* p, const PlanStreams& c, int64_t j) {
  return p->profiling == CLAK_PROFILE_SERIAL ? c.s_main[0] : c.s_main[j % NCOMPUTE];
}

#define CK(expr, what)                                                                      \
  do {                                                                                      \
    hipError_t e_ = (expr);                                                                 \
    if (e_ != hipSuccess) return fail(CLAK_E_DEVICE, "%s: %s: %s", what, #expr, hipGetErrorString(e_)); \
  } while (0)

clak_status make_schedule(Schedule* g, const std::vector<Plan*>& plans, const std::vector<int64_t>& off,
                          const clak_block* blocks, int g_dtype, int out_dtype, const char* what) {
  g->g_dtype = g_dtype;
  g->out_dtype = out_dtype;
  g->blocks.assign(blocks, blocks + off.back());
  g->ps.resize(plans.size());
  CK(hipEventCreateWithFlags(&g->fork, hipEventDisableTiming), what);
  for (size_t k = 0; k < plans.size(); ++k) {
    PlanStreams& c = g->ps[k];
    c.plan = plans[k];
    c.first = off[k];
    c.count = off[k + 1] - off[k];
    CK(hipStreamCreateWithFlags(&c.s_in, hipStreamNonBlocking), what);
    for (int q = 0; q < NCOMPUTE; ++q) {
      CK(hipStreamCreateWithFlags(&c.s_main[q], hipStreamNonBlocking), what);
      CK(hipEventCreateWithFlags(&c.joined_main[q], hipEventDisableTiming), what);
    }
    for (int q = 0; q < NSLOTS; ++q) {
      CK(hipEventCreateWithFlags(&c.ingested[q], hipEventDisableTiming), what);
      CK(hipEventCreateWithFlags(&c.done[q], hipEventDisableTiming), what);
    }
    CK(hipEventCreateWithFlags(&c.joined_in, hipEventDisableTiming), what);
  }
  return CLAK_OK;
}

// Enqueues the whole schedule, forked from and joined back to `origin`.
clak_status run_schedule(Schedule* g, hipStream_t origin, const char* what) {
  CK(hipEventRecord(g->fork, origin), what);
  for (auto& c : g->ps) {
    Plan* p = c.plan;
    // compute streams this launch uses (one for a single block or while profiling)
    const int nmain = (p->profiling == CLAK_PROFILE_SERIAL || c.count < 2) ? 1 : NCOMPUTE;
    for (int q = 0; q < nmain; ++q) CK(hipStreamWaitEvent(c.s_main[q], g->fork, 0), what);
    CK(hipStreamWaitEvent(c.s_in, g->fork, 0), what);
    for (int64_t j = 0; j < c.count; ++j) {
      const int slot = (int)(j % NSLOTS);
      const hipStream_t sm = compute_stream(p, c, j);
      // while profiling serially the ingest runs on the compute stream too, so
      // that every stage is timed without a concurrent kernel
      const hipStream_t si = p->profiling == CLAK_PROFILE_SERIAL ? sm : c.s_in;
      if (j >= NSLOTS) CK(hipStreamWaitEvent(si, c.done[slot], 0), what);
      const clak_block& B = g->blocks[c.first + j];
      clak_status st = enqueue_block(p, slot, si, sm, c.ingested[slot], B.m_blk, B.G, g->g_dtype,
                                     B.ldg, cell_out(B.b, B.se, B.pval, B.flags, B.ldo, g->out_dtype));
      if (st) return st;
      CK(hipEventRecord(c.done[slot], sm), what);
    }
    CK(hipEventRecord(c.joined_in, c.s_in), what);
    CK(hipStreamWaitEvent(origin, c.joined_in, 0), what);
    for (int q = 0; q < nmain; ++q) {
      CK(hipEventRecord(c.joined_main[q], c.s_main[q]), what);
      CK(hipStreamWaitEvent(origin, c.joined_main[q], 0), what);
    }
  }
  return CLAK_OK;
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
  std::vector<clak_block> placeholder((size_t)n_blocks);
  Schedule* g = new Schedule();
  clak_status s = make_schedule(g, {p}, {0, n_blocks}, placeholder.data(), g_dtype, out_dtype, what);
  auto done = [&](clak_status st) {
    release(g);
    return st;
  };
  if (s) return done(s);
  PlanStreams& c = g->ps[0];
  auto ck = [&](hipError_t e) -> clak_status {
    return e == hipSuccess ? CLAK_OK : fail(CLAK_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
  };
  if ((s = ck(hipEventRecord(g->fork, p->stream)))) return done(s);
  for (int q = 0; q < NCOMPUTE; ++q)
    if ((s = ck(hipStreamWaitEvent(c.s_main[q], g->fork, 0)))) return done(s);
  if ((s = ck(hipStreamWaitEvent(c.s_in, g->fork, 0)))) return done(s);
  clak_status result = CLAK_OK;
  for (int64_t j = 0; j < n_blocks && result == CLAK_OK; ++j) {
    const int slot = (int)(j % NSLOTS);
    clak_block B{};
    if ((result = get(j, &B))) break;
    if ((result = validate_block(p, B.m_blk, B.G, g_dtype, B.ldg, B.b, B.se, out_dtype, B.ldo, B.flags, B.pval))) break;
    const hipStream_t sm = compute_stream(p, c, j);
    const hipStream_t si = p->profiling == CLAK_PROFILE_SERIAL ? sm : c.s_in;  // as in run_schedule
    if (j >= NSLOTS && (result = ck(hipStreamWaitEvent(si, c.done[slot], 0)))) break;
    if ((result = enqueue_block(p, slot, si, sm, c.ingested[slot], B.m_blk, B.G, g_dtype, B.ldg,
                                cell_out(B.b, B.se, B.pval, B.flags, B.ldo, out_dtype))))
      break;
    if ((result = after(j, si))) break;
    result = ck(hipEventRecord(c.done[slot], sm));
  }
  // join everything enqueued so far back to the plan's stream and wait for it
  clak_status js = ck(hipEventRecord(c.joined_in, c.s_in));
  if (!js) js = ck(hipStreamWaitEvent(p->stream, c.joined_in, 0));
  for (int q = 0; q < NCOMPUTE && !js; ++q) {
    js = ck(hipEventRecord(c.joined_main[q], c.s_main[q]));
    if (!js) js = ck(hipStreamWaitEvent(p->stream, c.joined_main[q], 0));
  }
  if (!js) js = ck(hipStreamSynchronize(p->stream));
  return done(result ? result : js);
}

}  // namespace clak

struct clak_pipeline_s {
  Schedule* run;
  Plan* plan;
};

struct clak_batch_s {
  Schedule* run;
  std::vector<Plan*> plans;
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
  s = make_schedule(g, {p}, {0, n_blocks}, blocks, g_dtype, out_dtype, "pipeline_create");
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

clak_status clak_batch_create(clak_batch_t* out, int n_plans, const clak_plan_t* plans, const int64_t* n_blocks,
                              const clak_block* blocks, int g_dtype, int out_dtype) {
  if (!out) return fail(CLAK_E_ARG, "batch_create: null output pointer");
  *out = nullptr;
  if (n_plans < 1 || !plans || !n_blocks || !blocks) return fail(CLAK_E_ARG, "batch_create: empty batch");
  std::vector<Plan*> ps;
  std::vector<int64_t> off{0};
  for (int k = 0; k < n_plans; ++k) {
    Plan* p = reinterpret_cast<Plan*>(plans[k]);
    clak_status s = need_state(p, ST_READY, "batch_create");
    if (s) return s;
    for (Plan* q : ps)
      if (q == p) return fail(CLAK_E_ARG, "batch_create: plan %d listed twice", k);
    if (n_blocks[k] < 1) return fail(CLAK_E_ARG, "batch_create: plan %d has no blocks", k);
    s = check_blocks(p, n_blocks[k], blocks + off.back(), g_dtype, out_dtype);
    if (s) return s;
    ps.push_back(p);
    off.push_back(off.back() + n_blocks[k]);
  }
  Schedule* g = new Schedule();
  clak_status s = make_schedule(g, ps, off, blocks, g_dtype, out_dtype, "batch_create");
  if (s) {
    release(g);
    return s;
  }
  *out = new clak_batch_s{g, ps};
  return ok();
}

clak_status clak_batch_launch(clak_batch_t batch, void* hip_stream) {
  if (!batch) return fail(CLAK_E_ARG, "batch_launch: null batch");
  for (Plan* p : batch->plans) {
    clak_status s = need_state(p, ST_READY, "batch_launch");
    if (s) return s;
  }
  clak_status s = run_schedule(batch->run, (hipStream_t)hip_stream, "batch_launch");
  if (s) return s;
  return ok();
}

clak_status clak_batch_destroy(clak_batch_t batch) {
  if (!batch) return fail(CLAK_E_ARG, "batch_destroy: null batch");
  release(batch->run);
  delete batch;
  return ok();
}

}  // extern "C"
