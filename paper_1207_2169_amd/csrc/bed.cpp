// Out-of-core genotype input: a PLINK 1 binary genotype file (SNP-major) read
// block by block by a host thread into a ring of pinned buffers, and a scan
// that streams those buffers through a plan's block pipeline (the ingest reads
// the 2-bit rows straight from pinned host memory over PCIe, or through the
// copy engine with CLAK_STAGE_GENOTYPES), so that disk reads, PCIe transfers
// and the per-block kernels overlap (supplementary notes, section 3: the SNP
// blocks of X_R are streamed from disk while earlier blocks are processed).
#include <fcntl.h>
#include <unistd.h>

#include <algorithm>
#include <condition_variable>
#include <cstdio>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "clak_internal.hpp"

using namespace clak;

struct clak_bed_s {
  int fd = -1;
  int64_t n = 0, m = 0, block = 0, row = 0, nblocks = 0;
  int depth = 0;
  std::vector<uint8_t*> buf;       // pinned host buffers, block * row bytes each
  std::vector<hipEvent_t> freed;   // per buffer: recorded after the ingest that read it
  std::vector<char> armed;         // freed[k] has been recorded (guarded by mu)
  std::vector<int64_t> holds;      // block whose rows buffer k holds, -1 while being filled (guarded by mu)
  std::vector<std::thread> readers;
  std::mutex mu;
  std::condition_variable cv;
  int64_t claimed = 0;   // blocks handed to reader threads so far (in order)
  int64_t released = 0;  // blocks whose buffer the scan has handed back
  bool stop = false;
  std::string err;
};

namespace {

constexpr unsigned char BED_MAGIC[3] = {0x6c, 0x1b, 0x01};

// Reader threads claim blocks in order; block b goes to buffer b % depth once
// block b - depth has been released by the scan and its ingest has finished.
void reader_main(clak_bed_s* r) {
  for (;;) {
    int64_t b;
    bool busy;
    {
      std::unique_lock<std::mutex> lk(r->mu);
      r->cv.wait(lk, [&] { return r->stop || (r->claimed < r->nblocks && r->claimed - r->released < r->depth); });
      if (r->stop) return;
      b = r->claimed++;
      busy = r->armed[b % r->depth] != 0;
    }
    const int k = (int)(b % r->depth);
    if (busy) {
      // the GPU may still be reading this buffer
      if (hipEventSynchronize(r->freed[k]) != hipSuccess) {
        std::lock_guard<std::mutex> lk(r->mu);
        r->err = "bed reader: hipEventSynchronize failed";
        r->cv.notify_all();
        return;
      }
    }
    const int64_t first = b * r->block, count = std::min(r->block, r->m - first);
    size_t done = 0, want = (size_t)(count * r->row);
    while (done < want) {
      const ssize_t got = pread(r->fd, r->buf[k] + done, want - done, (off_t)(3 + first * r->row + (int64_t)done));
      if (got <= 0) break;
      done += (size_t)got;
    }
    std::lock_guard<std::mutex> lk(r->mu);
    if (done != want) {
      r->err = "bed reader: short read at SNP " + std::to_string(first);
      r->cv.notify_all();
      return;
    }
    r->holds[k] = b;
    r->cv.notify_all();
  }
}

void close_bed(clak_bed_s* r) {
  if (!r) return;
  {
    std::lock_guard<std::mutex> lk(r->mu);
    r->stop = true;
  }
  r->cv.notify_all();
  for (auto& t : r->readers)
    if (t.joinable()) t.join();
  for (size_t k = 0; k < r->freed.size(); ++k) {
    if (r->armed[k]) (void)hipEventSynchronize(r->freed[k]);
    if (r->freed[k]) (void)hipEventDestroy(r->freed[k]);
  }
  for (uint8_t* p : r->buf)
    if (p) (void)hipHostFree(p);
  if (r->fd >= 0) close(r->fd);
  delete r;
}

}  // namespace

extern "C" {

clak_status clak_bed_open(clak_bed_t* out, const char* path, int64_t n, int64_t m, int64_t block, int depth) {
  if (!out || !path) return fail(CLAK_E_ARG, "bed_open: null argument");
  *out = nullptr;
  if (n < 1 || m < 1 || block < 1) return fail(CLAK_E_ARG, "bed_open: n, m and block must be positive");
  if (depth < 2 || depth > 16) return fail(CLAK_E_ARG, "bed_open: depth=%d outside [2, 16]", depth);
  const int fd = open(path, O_RDONLY);
  if (fd < 0) return fail(CLAK_E_ARG, "bed_open: cannot open %s", path);
  unsigned char magic[3] = {0, 0, 0};
  const int64_t row = (n + 3) / 4;
  const off_t size = lseek(fd, 0, SEEK_END);
  if (pread(fd, magic, 3, 0) != 3 || magic[0] != BED_MAGIC[0] || magic[1] != BED_MAGIC[1] ||
      magic[2] != BED_MAGIC[2]) {
    close(fd);
    return fail(CLAK_E_ARG, "bed_open: %s is not a SNP-major PLINK 1 binary genotype file", path);
  }
  if ((int64_t)size != 3 + m * row) {
    close(fd);
    return fail(CLAK_E_ARG, "bed_open: %s holds %lld bytes, %lld expected for n=%lld, m=%lld", path,
                (long long)size, (long long)(3 + m * row), (long long)n, (long long)m);
  }
  clak_bed_s* r = new clak_bed_s();
  r->fd = fd;
  r->n = n;
  r->m = m;
  r->block = block;
  r->row = row;
  r->nblocks = (m + block - 1) / block;
  r->depth = depth;
  r->buf.assign(depth, nullptr);
  r->freed.assign(depth, nullptr);
  r->armed.assign(depth, 0);
  r->holds.assign(depth, -1);
  for (int k = 0; k < depth; ++k) {
    if (hipHostMalloc((void**)&r->buf[k], (size_t)(block * row), hipHostMallocDefault) != hipSuccess ||
        hipEventCreateWithFlags(&r->freed[k], hipEventDisableTiming) != hipSuccess) {
      (void)hipGetLastError();
      close_bed(r);
      return fail(CLAK_E_DEVICE, "bed_open: pinned buffer or event allocation failed");
    }
  }
  // a few positional readers keep the ring full (one thread reads about as fast as the rotation consumes)
  const int nthreads = std::max(1, std::min(4, depth / 2));
  for (int k = 0; k < nthreads; ++k) r->readers.emplace_back(reader_main, r);
  *out = r;
  return ok();
}

clak_status clak_bed_scan(clak_bed_t r, clak_plan_t h, void* d_b, void* d_se, int out_dtype, int64_t ldo,
                          uint8_t* d_flags, void* d_pval) {
  Plan* p = reinterpret_cast<Plan*>(h);
  if (!r) return fail(CLAK_E_ARG, "bed_scan: null reader");
  clak_status s = need_state(p, ST_READY, "bed_scan");
  if (s) return s;
  if (r->n != p->n) return fail(CLAK_E_ARG, "bed_scan: the file has n=%lld, the plan n=%lld", (long long)r->n,
                                (long long)p->n);
  if (r->block > p->max_block)
    return fail(CLAK_E_ARG, "bed_scan: block=%lld > max_block=%lld", (long long)r->block, (long long)p->max_block);
  if (ldo < r->m) return fail(CLAK_E_ARG, "bed_scan: ldo=%lld < m=%lld", (long long)ldo, (long long)r->m);
  if (!d_b || !d_se) return fail(CLAK_E_ARG, "bed_scan: null b or se");
  {
    // a finished scan rewinds the reader: the next one reads the file again from the start
    std::lock_guard<std::mutex> lk(r->mu);
    if (!r->err.empty()) return fail(CLAK_E_ARG, "bed_scan: %s", r->err.c_str());
    if (r->released == r->nblocks) {
      r->claimed = 0;
      r->released = 0;
      for (auto& held : r->holds) held = -1;
      r->cv.notify_all();
    } else if (r->released != 0) {
      return fail(CLAK_E_STATE, "bed_scan: an earlier scan of this reader did not finish (open the file again)");
    }
  }
  const size_t esz = out_dtype == CLAK_OUT_F64 ? 8 : 4;
  const int64_t pw = (p->flags & CLAK_OUT_FULL) ? p->pL + 1 : 1;
  auto get = [&](int64_t b, clak_block* B) -> clak_status {
    std::unique_lock<std::mutex> lk(r->mu);
    r->cv.wait(lk, [&] { return r->holds[b % r->depth] == b || !r->err.empty(); });
    if (!r->err.empty()) return fail(CLAK_E_ARG, "bed_scan: %s", r->err.c_str());
    const int64_t first = b * r->block;
    B->m_blk = std::min(r->block, r->m - first);
    B->G = r->buf[b % r->depth];
    B->ldg = r->row;
    B->b = (char*)d_b + (size_t)first * pw * esz;
    B->se = (char*)d_se + (size_t)first * esz;
    B->ldo = ldo;
    B->flags = d_flags ? d_flags + first : nullptr;
    B->pval = d_pval ? (char*)d_pval + (size_t)first * esz : nullptr;
    return CLAK_OK;
  };
  auto after = [&](int64_t b, hipStream_t s_in) -> clak_status {
    const int k = (int)(b % r->depth);
    if (hipEventRecord(r->freed[k], s_in) != hipSuccess) return fail(CLAK_E_DEVICE, "bed_scan: hipEventRecord");
    std::lock_guard<std::mutex> lk(r->mu);
    r->armed[k] = 1;
    r->holds[k] = -1;
    r->released = b + 1;
    r->cv.notify_all();
    return CLAK_OK;
  };
  s = stream_blocks(p, r->nblocks, CLAK_G_P2, out_dtype, get, after, "bed_scan");
  if (s) return s;
  return ok();
}

clak_status clak_bed_close(clak_bed_t r) {
  if (!r) return fail(CLAK_E_ARG, "bed_close: null reader");
  close_bed(r);
  return ok();
}

}  // extern "C"
