// Host-side checks of libclak's argument validation, call-order checks,
// genotype-file validation and workspace carving, compiled with
// AddressSanitizer and UndefinedBehaviorSanitizer and run where no GPU is
// needed: every call below returns before any device work.  Where the
// library would need a device (plan creation, pinned buffers) the check
// accepts CLAK_E_DEVICE when none is present.
//
// Usage: abi_checks <scratch directory>.  Prints one line per failed check
// and "abi_checks: N checks, F failed"; exit status 1 if any failed.
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "clak.h"
#include "clak_internal.hpp"

using namespace clak;

static int g_checks = 0, g_failed = 0;

static void check(bool ok, const char* what) {
  ++g_checks;
  if (!ok) {
    ++g_failed;
    std::printf("FAILED: %s (last error: %s)\n", what, clak_last_error());
  }
}

static void expect(clak_status got, clak_status want, const char* what) {
  char buf[256];
  std::snprintf(buf, sizeof buf, "%s: status %d, expected %d", what, (int)got, (int)want);
  check(got == want && (want == CLAK_OK || std::strlen(clak_last_error()) > 0), buf);
}

static void write_file(const std::string& path, const std::vector<unsigned char>& bytes) {
  FILE* f = std::fopen(path.c_str(), "wb");
  if (!f) {
    check(false, "cannot write a scratch file");
    return;
  }
  if (!bytes.empty()) std::fwrite(bytes.data(), 1, bytes.size(), f);
  std::fclose(f);
}

// Null handles and invalid arguments of every entry point.
static void null_handles() {
  double d = 0.0;
  size_t sz = 0;
  int64_t i64 = 0;
  int i = 0;
  expect(clak_plan_create(nullptr, 100, 3, 1, 10, CLAK_PREC_MIXED, 0), CLAK_E_ARG, "plan_create null output");
  clak_plan_t h = reinterpret_cast<clak_plan_t>(&d);
  expect(clak_plan_create(&h, 100, 0, 1, 10, CLAK_PREC_MIXED, 0), CLAK_E_ARG, "plan_create p_L = 0");
  check(h == nullptr, "plan_create clears its output on error");
  expect(clak_plan_create(&h, 3, 3, 1, 10, CLAK_PREC_MIXED, 0), CLAK_E_ARG, "plan_create n <= p_L");
  expect(clak_plan_create(&h, 100, 3, 0, 10, CLAK_PREC_MIXED, 0), CLAK_E_ARG, "plan_create t = 0");
  expect(clak_plan_create(&h, 100, 3, 1, 0, CLAK_PREC_MIXED, 0), CLAK_E_ARG, "plan_create max_block = 0");
  expect(clak_plan_create(&h, 100, 3, 1, 10, 7, 0), CLAK_E_ARG, "plan_create unknown precision");
  expect(clak_plan_create(&h, 100, 3, 1, 10, CLAK_PREC_MIXED, 1u << 30), CLAK_E_ARG, "plan_create unknown flag");
  expect(clak_plan_create(&h, 100, 3, 2, 10, CLAK_PREC_MIXED, CLAK_CHOL), CLAK_E_ARG, "plan_create CHOL, t = 2");
  expect(clak_plan_create(&h, 100, 9, 1, 10, CLAK_PREC_MIXED, 0), CLAK_E_UNSUPPORTED, "plan_create mixed p_L = 9");
  expect(clak_plan_create(&h, (int64_t)1 << 21, 3, 1, 10, CLAK_PREC_FP64, 0), CLAK_E_UNSUPPORTED,
         "plan_create n too large");
  // a valid plan needs a device: without one, CLAK_E_DEVICE and no handle
  clak_status s = clak_plan_create(&h, 100, 3, 1, 10, CLAK_PREC_MIXED, 0);
  if (s == CLAK_OK) {
    expect(clak_plan_destroy(h), CLAK_OK, "plan_destroy");
  } else {
    expect(s, CLAK_E_DEVICE, "plan_create without a device");
    check(h == nullptr, "plan_create without a device leaves no handle");
  }

  clak_plan_t np = nullptr;
  expect(clak_plan_workspace_size(np, &sz), CLAK_E_ARG, "workspace_size null plan");
  expect(clak_plan_set_workspace(np, &d, 8), CLAK_E_ARG, "set_workspace null plan");
  expect(clak_plan_set_stream(np, nullptr), CLAK_E_ARG, "set_stream null plan");
  expect(clak_set_kinship(np, &d, 1), CLAK_E_ARG, "set_kinship null plan");
  expect(clak_set_eigen(np, &d, 1, &d), CLAK_E_ARG, "set_eigen null plan");
  expect(clak_set_covariates(np, &d, 1), CLAK_E_ARG, "set_covariates null plan");
  expect(clak_set_traits(np, &d, 1, &d, &d), CLAK_E_ARG, "set_traits null plan");
  expect(clak_estimate_vc(np, &d, 1, CLAK_VC_REML, &d, &d, nullptr), CLAK_E_ARG, "estimate_vc null plan");
  expect(clak_run_block(np, 1, &d, CLAK_G_U8, 1, &d, &d, CLAK_OUT_F32, 1, nullptr, nullptr), CLAK_E_ARG,
         "run_block null plan");
  expect(clak_run_block_static(np, 1, &d, CLAK_G_U8, 1, &d, &d, CLAK_OUT_F32, 1, nullptr, nullptr), CLAK_E_ARG,
         "run_block_static null plan");
  expect(clak_plan_block_scratch_size(np, &sz), CLAK_E_ARG, "block_scratch_size null plan");
  expect(clak_autotune(np, 1, &d, CLAK_G_U8, 1, &d, &d, CLAK_OUT_F32, 1, nullptr, nullptr), CLAK_E_ARG,
         "autotune null plan");
  clak_block blk = {1, &d, 1, &d, &d, 1, nullptr, nullptr};
  expect(clak_autotune_pipeline(np, 1, &blk, CLAK_G_U8, CLAK_OUT_F32, nullptr), CLAK_E_ARG,
         "autotune_pipeline null plan");
  expect(clak_plan_set_tuning(np, 0, 0, 0, 0), CLAK_E_ARG, "set_tuning null plan");
  expect(clak_plan_get_shape(np, &i64, &i64, &i64, &i64, &i, nullptr), CLAK_E_ARG, "get_shape null plan");
  expect(clak_plan_get_tuning(np, &i, &i, &i, &i), CLAK_E_ARG, "get_tuning null plan");
  expect(clak_plan_set_profiling(np, CLAK_PROFILE_OFF), CLAK_E_ARG, "set_profiling null plan");
  expect(clak_plan_get_profile(np, &d, &i64), CLAK_E_ARG, "get_profile null plan");
  expect(clak_plan_get_busy(np, &d), CLAK_E_ARG, "get_busy null plan");

  clak_pipeline_t pipe = nullptr;
  expect(clak_pipeline_create(nullptr, np, 1, &blk, CLAK_G_U8, CLAK_OUT_F32), CLAK_E_ARG,
         "pipeline_create null output");
  expect(clak_pipeline_create(&pipe, np, 1, &blk, CLAK_G_U8, CLAK_OUT_F32), CLAK_E_ARG, "pipeline_create null plan");
  expect(clak_pipeline_launch(nullptr), CLAK_E_ARG, "pipeline_launch null");
  expect(clak_pipeline_destroy(nullptr), CLAK_E_ARG, "pipeline_destroy null");

  clak_batch_t batch = nullptr;
  int64_t nb = 1;
  expect(clak_batch_create(nullptr, 1, &np, &nb, &blk, CLAK_G_U8, CLAK_OUT_F32), CLAK_E_ARG,
         "batch_create null output");
  expect(clak_batch_create(&batch, 0, &np, &nb, &blk, CLAK_G_U8, CLAK_OUT_F32), CLAK_E_ARG, "batch_create no plans");
  expect(clak_batch_create(&batch, 1, &np, &nb, &blk, CLAK_G_U8, CLAK_OUT_F32), CLAK_E_ARG,
         "batch_create null plan");
  expect(clak_batch_launch(nullptr, nullptr), CLAK_E_ARG, "batch_launch null");
  expect(clak_batch_get_info(nullptr, &i, &i64, &i), CLAK_E_ARG, "batch_get_info null");
  expect(clak_batch_destroy(nullptr), CLAK_E_ARG, "batch_destroy null");

  expect(clak_bed_scan(nullptr, np, &d, &d, CLAK_OUT_F32, 1, nullptr, nullptr), CLAK_E_ARG, "bed_scan null reader");
  expect(clak_bed_close(nullptr), CLAK_E_ARG, "bed_close null");
}

// Call order and argument checks on a plan that has its sizes but no device
// state (a host-only Plan object; none of these calls reach the device).
static void call_order() {
  Plan p;
  init_shape(p, 1000, 3, 20, 4096, CLAK_PREC_MIXED, 0);
  clak_plan_t h = reinterpret_cast<clak_plan_t>(&p);
  double d = 0.0;
  expect(clak_set_kinship(h, &d, 1000), CLAK_E_STATE, "set_kinship before a workspace");
  expect(clak_set_eigen(h, &d, 1000, &d), CLAK_E_STATE, "set_eigen before a workspace");
  expect(clak_set_covariates(h, &d, 1000), CLAK_E_STATE, "set_covariates before the eigenvectors");
  expect(clak_set_traits(h, &d, 1000, &d, &d), CLAK_E_STATE, "set_traits before the covariates");
  expect(clak_estimate_vc(h, &d, 1000, CLAK_VC_REML, &d, &d, nullptr), CLAK_E_STATE, "estimate_vc before the covariates");
  expect(clak_run_block(h, 1, &d, CLAK_G_U8, 1000, &d, &d, CLAK_OUT_F32, 1, nullptr, nullptr), CLAK_E_STATE,
         "run_block before the traits");
  expect(clak_run_block_static(h, 1, &d, CLAK_G_U8, 1000, &d, &d, CLAK_OUT_F32, 1, nullptr, nullptr),
         CLAK_E_STATE, "run_block_static before the traits");
  expect(clak_plan_set_workspace(h, nullptr, 0), CLAK_E_WORKSPACE, "set_workspace null workspace");
  expect(clak_plan_set_workspace(h, reinterpret_cast<void*>(uintptr_t(4096 + 8)), 1 << 30), CLAK_E_WORKSPACE,
         "set_workspace misaligned");
  expect(clak_plan_set_tuning(h, 99, 0, 0, 0), CLAK_E_ARG, "set_tuning rotation configuration out of range");
  expect(clak_plan_set_tuning(h, 0, 3, 0, 0), CLAK_E_ARG, "set_tuning row grouping not a divisor of 8");
  expect(clak_plan_set_tuning(h, 0, 0, 48, 0), CLAK_E_ARG, "set_tuning grid tile width");
  expect(clak_plan_set_profiling(h, 7), CLAK_E_ARG, "set_profiling unknown mode");
  int64_t n = 0, pl = 0, t = 0, mb = 0;
  int prec = -1;
  uint32_t fl = 1;
  expect(clak_plan_get_shape(h, &n, &pl, &t, &mb, &prec, &fl), CLAK_OK, "get_shape");
  check(n == 1000 && pl == 3 && t == 20 && mb == 4096 && prec == CLAK_PREC_MIXED && fl == 0, "get_shape values");
  size_t ws = 0, scratch = 0;
  expect(clak_plan_workspace_size(h, &ws), CLAK_OK, "workspace_size");
  expect(clak_plan_block_scratch_size(h, &scratch), CLAK_OK, "block_scratch_size");
  check(ws > 3 * scratch && scratch > 0, "three block slots inside the workspace");
  clak_block blk = {1, &d, 1000, &d, &d, 1, nullptr, nullptr};
  clak_pipeline_t pipe = nullptr;
  expect(clak_pipeline_create(&pipe, h, 1, &blk, CLAK_G_U8, CLAK_OUT_F32), CLAK_E_STATE,
         "pipeline_create before the traits");
  clak_batch_t batch = nullptr;
  int64_t nb = 1;
  expect(clak_batch_create(&batch, 1, &h, &nb, &blk, CLAK_G_U8, CLAK_OUT_F32), CLAK_E_STATE,
         "batch_create before the traits");
}

// Genotype-file validation of the reader (no device call before the file checks pass).
static void bed_files(const std::string& dir) {
  clak_bed_t r = nullptr;
  const std::string good = dir + "/good.bed", magic = dir + "/magic.bed", shortf = dir + "/short.bed",
                    empty = dir + "/empty.bed";
  const int64_t n = 10, m = 7, row = (n + 3) / 4;
  std::vector<unsigned char> bytes = {0x6c, 0x1b, 0x01};
  for (int64_t k = 0; k < m * row; ++k) bytes.push_back((unsigned char)(37 * k + 11));
  write_file(good, bytes);
  std::vector<unsigned char> bad = bytes;
  bad[2] = 0x00;  // individual-major files are not read
  write_file(magic, bad);
  write_file(shortf, std::vector<unsigned char>(bytes.begin(), bytes.end() - 1));
  write_file(empty, {});
  expect(clak_bed_open(nullptr, good.c_str(), n, m, 4, 4), CLAK_E_ARG, "bed_open null output");
  expect(clak_bed_open(&r, nullptr, n, m, 4, 4), CLAK_E_ARG, "bed_open null path");
  expect(clak_bed_open(&r, good.c_str(), 0, m, 4, 4), CLAK_E_ARG, "bed_open n = 0");
  expect(clak_bed_open(&r, good.c_str(), n, m, 0, 4), CLAK_E_ARG, "bed_open block = 0");
  expect(clak_bed_open(&r, good.c_str(), n, m, 4, 1), CLAK_E_ARG, "bed_open depth 1");
  expect(clak_bed_open(&r, good.c_str(), n, m, 4, 17), CLAK_E_ARG, "bed_open depth 17");
  expect(clak_bed_open(&r, (dir + "/missing.bed").c_str(), n, m, 4, 4), CLAK_E_ARG, "bed_open missing file");
  expect(clak_bed_open(&r, magic.c_str(), n, m, 4, 4), CLAK_E_ARG, "bed_open wrong magic");
  expect(clak_bed_open(&r, shortf.c_str(), n, m, 4, 4), CLAK_E_ARG, "bed_open truncated file");
  expect(clak_bed_open(&r, empty.c_str(), n, m, 4, 4), CLAK_E_ARG, "bed_open empty file");
  expect(clak_bed_open(&r, good.c_str(), n + 4, m, 4, 4), CLAK_E_ARG, "bed_open size for another n");
  check(r == nullptr, "bed_open leaves no reader on error");
  // a valid file needs pinned buffers: without a device, CLAK_E_DEVICE and the partial reader is released
  clak_status s = clak_bed_open(&r, good.c_str(), n, m, 4, 4);
  if (s == CLAK_OK) {
    expect(clak_bed_close(r), CLAK_OK, "bed_close");
  } else {
    expect(s, CLAK_E_DEVICE, "bed_open without a device");
    check(r == nullptr, "bed_open without a device leaves no reader");
  }
}

// Every region the workspace carving hands out lies inside the workspace, is
// 256-byte aligned, and follows the previous one without overlap; the three
// block slots are equal and the per-block pointers name slot 0.
static void carving() {
  const int64_t ns[] = {4, 127, 128, 129, 1000, 4099, 10000};
  const int64_t pls[] = {1, 3, 8};
  const int64_t ts[] = {1, 2, 129, 1000};
  const int64_t mbs[] = {1, 255, 10000, 20000};
  const uint32_t flagsets[] = {0, CLAK_OUT_FULL, CLAK_STAGE_GENOTYPES, CLAK_CHOL};
  char* const base = reinterpret_cast<char*>(uintptr_t(1) << 40);  // never dereferenced
  int plans = 0;
  for (int prec : {CLAK_PREC_FP64, CLAK_PREC_MIXED})
    for (int64_t n : ns)
      for (int64_t pl : pls)
        for (int64_t t : ts)
          for (int64_t mb : mbs)
            for (uint32_t fl : flagsets) {
              if (n <= pl || ((fl & CLAK_CHOL) && t != 1)) continue;
              Plan p;
              init_shape(p, n, pl, t, mb, prec, fl);
              ++plans;
              char what[160];
              std::snprintf(what, sizeof what, "carving prec=%d n=%lld p_L=%lld t=%lld block=%lld flags=0x%x", prec,
                            (long long)n, (long long)pl, (long long)t, (long long)mb, fl);
              const size_t size = workspace_bytes(p, nullptr, nullptr);
              Workspace w;
              const size_t again = workspace_bytes(p, &w, base);
              const size_t sb = slot_bytes(p, nullptr, nullptr);
              bool ok = again == size && size % 256 == 0 && sb % 256 == 0 && 3 * sb < size;
              const void* regions[] = {w.Zt, w.w, w.evE, w.dstat, w.QL, w.Rm, w.Rinv, w.XLt, w.Qt, w.Yt, w.tpar,
                                       w.Phi, w.XL, w.V64, w.D64, w.Zd, w.zs, w.Cq, w.Vd, w.Dd, w.vs, w.ds};
              const char* prev = nullptr;
              for (const void* r : regions) {
                if (!r) continue;
                const char* c = static_cast<const char*>(r);
                ok = ok && c >= base && c < base + size && (uintptr_t)c % 256 == 0 && (!prev || c > prev);
                prev = c;
              }
              for (int k = 0; k < NSLOTS; ++k) {
                const Slot& S = w.slot[k];
                const char* start = reinterpret_cast<const char*>(S.Gp);
                ok = ok && start > prev && start + sb <= base + size;
                if (k) ok = ok && start == reinterpret_cast<const char*>(w.slot[k - 1].Gp) + sb;
                const void* parts[] = {S.Gp, S.sstat, S.ipart, S.part, S.X64, S.Xd, S.Gh};
                const char* q = nullptr;
                for (const void* r : parts) {
                  if (!r) continue;
                  const char* c = static_cast<const char*>(r);
                  ok = ok && c >= start && c < start + sb && (uintptr_t)c % 256 == 0 && (!q || c > q);
                  q = c;
                }
                ok = ok && ((S.Gh != nullptr) == ((fl & CLAK_STAGE_GENOTYPES) != 0));
                ok = ok && ((S.Xd != nullptr) == (prec == CLAK_PREC_MIXED && t > 1));
              }
              ok = ok && w.Gp == w.slot[0].Gp && w.sstat == w.slot[0].sstat && w.X64 == w.slot[0].X64 &&
                   w.Xd == w.slot[0].Xd && w.part == w.slot[0].part;
              ok = ok && p.n_pad % 128 == 0 && p.n_pad >= n && p.mb_pad % 256 == 0 && p.mb_pad >= mb &&
                   p.t_pad % 128 == 0 && p.t_pad >= t && p.zrows >= p.n_pad;
              check(ok, what);
            }
  check(plans > 500, "carving: plan shapes covered");
}

int main(int argc, char** argv) {
  if (argc < 2) {
    std::fprintf(stderr, "usage: abi_checks <scratch directory>\n");
    return 2;
  }
  check(std::strlen(clak_version()) > 0, "version string");
  null_handles();
  call_order();
  bed_files(argv[1]);
  carving();
  std::printf("abi_checks: %d checks, %d failed\n", g_checks, g_failed);
  return g_failed ? 1 : 0;
}
