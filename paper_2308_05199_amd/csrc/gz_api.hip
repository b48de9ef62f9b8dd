// gz_api.hip -- host runtime and C ABI (include/gzccl.h).
//
// The context owns every temporary device buffer, allocated once: the
// control block (tickets, epoch, sticky status), one look-back word per
// strip, one chain word per job, the batch descriptor arena and the selector
// weights.  Single calls pass their job descriptor as a kernel argument;
// batched calls stage descriptors through a small ring of pinned host
// buffers and one async copy.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "gz_common.h"
#include "gz_kernels.h"
#include "gz_select.h"
#include "gzccl.h"

using gzk::Ctl;
using gzk::Ctrl;
using gzk::Job;
using gzk::job_ptr;

namespace {

constexpr int STAGE_SLOTS = 4;
constexpr uint64_t MAX_CHAIN_DW = (1ull << 34) - 1;  // look-back value field

struct Tuned {
  uint32_t tpb = 0, grid = 0;
};

// First-fit ranges of a context-owned device array (plan descriptors), so
// that creating and destroying plans never allocates device memory.
struct Arena {
  uint64_t cap = 0;
  std::vector<std::pair<uint64_t, uint64_t>> used;  // (offset, length), by offset
  bool take(uint64_t len, uint64_t& off) {
    if (len == 0 || len > cap) return false;
    uint64_t at = 0;
    size_t i = 0;
    for (; i < used.size(); ++i) {
      if (used[i].first - at >= len) break;
      at = used[i].first + used[i].second;
    }
    if (i == used.size() && cap - at < len) return false;
    used.insert(used.begin() + (long)i, {at, len});
    off = at;
    return true;
  }
  void give(uint64_t off) {
    for (size_t i = 0; i < used.size(); ++i)
      if (used[i].first == off) {
        used.erase(used.begin() + (long)i);
        return;
      }
  }
};

}  // namespace

struct gz_ctx {
  int device = 0;
  int cus = 0;
  size_t lds_max = 0;  // LDS one workgroup may allocate
  uint64_t max_elems = 0;
  uint32_t max_jobs = 0;
  uint64_t max_strips = 0;
  Ctrl* ctrl = nullptr;
  unsigned long long* status = nullptr;
  unsigned long long* jobbase = nullptr;
  uint8_t* blob = nullptr;
  bool blob_loaded = false;
  Job* d_jobs = nullptr;
  uint32_t* d_map = nullptr;
  uint8_t* stage[STAGE_SLOTS] = {};
  hipEvent_t stage_ev[STAGE_SLOTS] = {};
  bool stage_used[STAGE_SLOTS] = {};
  int stage_next = 0;
  size_t stage_bytes = 0;
  Tuned tuned[3][2][3];  // single calls: [op][dtype][log2L-5]
  Tuned batch_tuned[4][2];  // batched launches: [op][batch holds fp64]
  uint32_t best_L[2] = {0, 0};  // tuned block length per dtype (0: untuned, 32)
  uint64_t wait_ticks = 0;    // wait bound in ticks of the constant-rate clock (1 s default)
  uint64_t wclk_khz = 0;      // that clock's rate
  float* train_ws = nullptr;  // selector training: per-sample backward terms
  // plan arena: descriptors and strip maps of live plans (allocated once)
  Job* plan_jobs = nullptr;
  uint32_t* plan_map = nullptr;
  Arena plan_jobs_arena, plan_map_arena;
  std::vector<gz_plan*> live_plans;
  Ctl ctl() const { return Ctl{ctrl, status, jobbase, blob, wait_ticks}; }
};

struct gz_plan {
  gz_ctx* ctx = nullptr;  // null once the context is destroyed
  uint32_t op = 0;
  Job* d_jobs = nullptr;      // in the context's plan arena
  uint32_t* d_map = nullptr;  // in the context's plan arena
  uint64_t jobs_off = 0, map_off = 0;
  uint32_t total = 0;
  uint32_t njobs = 0;  // uniform batch: the kernels derive (job, strip)
  uint32_t tpb = 0, grid = 0;
  bool wide = false;
  bool wave = false;  // per-wave encoding kernels (total = njobs x rounds)
  bool wave_dec = false;  // per-wave decoding kernels (total = superblocks)
  bool has_map = false;   // wave_dec: d_map lists (job, superblock) pairs
  uint32_t jw = 0;        // wave_dec: d_map holds jw per-wave job shares
  uint32_t log2L = 5;
};

struct gz_graph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

uint64_t cdiv(uint64_t a, uint64_t b) { return (a + b - 1) / b; }
uint64_t round4(uint64_t a) { return (a + 3) & ~3ull; }
uint32_t esize(uint32_t dt) { return dt == GZ_F32 ? 4u : 8u; }

bool valid_L(uint32_t L) { return L == 32 || L == 64 || L == 128; }
uint32_t log2_of(uint32_t L) { return L == 32 ? 5u : L == 64 ? 6u : 7u; }

uint64_t bound_of(uint64_t n, uint32_t dt, uint32_t L) {
  return gzk::HDR + 4 * cdiv(n, gzk::SUPER) + round4(cdiv(n, L)) + n * esize(dt);
}
uint64_t fixed_of(uint64_t n, uint32_t L) {
  return gzk::HDR + 4 * cdiv(n, gzk::SUPER) + round4(cdiv(n, L));
}

// Step t, its reciprocal and the largest float not above eb.
bool set_bound(Job& J, uint32_t dtype, double eb) {
  if (!(eb > 0.0) || !isfinite(eb)) return false;
  J.eb = eb;
  const double two = 2.0 * eb;
  if (dtype == GZ_F32) {
    float t = (float)two;
    if (!isfinite(t) || t == 0.0f) return false;
    J.t32 = t;
    J.rinv = 1.0 / (double)t;
    float e = (float)eb;
    if ((double)e > eb) e = nextafterf(e, 0.0f);
    J.eblo = e;
    J.t64 = (double)t;
  } else {
    if (!isfinite(two) || two == 0.0) return false;
    J.t64 = two;
    J.t32 = 0;
    J.rinv = 0;
    J.eblo = 0;
  }
  return true;
}

void set_geom(Job& J, uint64_t n, uint32_t L, uint32_t tpb) {
  J.n = n;
  J.log2L = log2_of(L);
  J.B = cdiv(n, L);
  J.NS = cdiv(n, gzk::SUPER);
  J.hdr_off = gzk::HDR + 4 * J.NS;
  J.pay_off = J.hdr_off + round4(J.B);
  const uint64_t segs = J.B * L / gzk::SEG;
  uint64_t ns = cdiv(segs, tpb);
  J.nstrips = (uint32_t)(ns ? ns : 1);
}

bool overlaps(const void* a, uint64_t na, const void* b, uint64_t nb) {
  if (!na || !nb) return false;
  uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
  return x < y + nb && y < x + na;
}

bool tile_mode(const gz_params* p);

// Workgroup size: the caller's, else the tuned one (1D streams), else the
// measured default.  fp32 1D encoding and the fused step take 1024 threads
// (a quarter of the per-strip ticket, barrier and look-back cost per element
// of 256), fp32 decoding 512 (measured faster than 1024), fp64 and tiles 256.
// Operations 0-3 as gz_op; decode-and-accumulate (3) shares decoding's tuning.
uint32_t tune_op(uint32_t op) { return op == 3 ? 1u : op; }

// threads = 64 (one wave) asks for the per-wave kernels.
constexpr uint32_t WAVE_TPB = 64;

uint32_t pick_tpb(const gz_ctx* c, uint32_t op, uint32_t dt, uint32_t L, const gz_params* p) {
  if (p && p->threads) return p->threads;
  if (!tile_mode(p)) {
    const Tuned& t = c->tuned[tune_op(op)][dt][log2_of(L) - 5];
    if (t.tpb && t.tpb != WAVE_TPB) return t.tpb;
  }
  if (dt != GZ_F32 || tile_mode(p)) return 256;
  for (uint32_t t = tune_op(op) == 1 ? 512u : 1024u; t > 256; t /= 2)
    if (gzk::lds_bytes(0, t) <= c->lds_max) return t;
  return 256;
}

uint32_t pick_grid(const gz_ctx* c, uint32_t op, uint32_t dt, uint32_t L, uint32_t tpb,
                   uint64_t strips, const gz_params* p) {
  uint64_t g;
  if (p && p->grid) {
    g = p->grid;
  } else {
    const Tuned& t = c->tuned[tune_op(op)][dt][log2_of(L) - 5];
    if (t.grid && t.tpb == tpb && op != 3) {
      g = t.grid;
    } else {
      int occ = gzk::occupancy_blocks(op == 3 ? gzk::OCC_ACCUM : op, dt, log2_of(L), tpb);
      g = (uint64_t)c->cus * (uint64_t)occ;
    }
  }
  g = std::min<uint64_t>(g, strips);
  return (uint32_t)std::max<uint64_t>(g, 1);
}

uint32_t pick_tile_grid(const gz_ctx* c, uint32_t op, uint32_t tpb, uint64_t strips,
                        const gz_params* p) {
  uint64_t g = (p && p->grid) ? p->grid
                              : (uint64_t)c->cus * gzk::occupancy_blocks(op, 0, 6, tpb);
  return (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(g, strips));
}

bool tpb_ok(uint32_t t) {
  return t == 0 || t == WAVE_TPB || t == 128 || t == 256 || t == 512 || t == 1024;
}

// The strip kernel is built for tpb threads (1024 only for fp32 1D kernels)
// and the workgroup's LDS fits the device (512-thread fp64 strips may not).
bool tpb_fits(const gz_ctx* c, bool wide, bool tile, uint32_t tpb) {
  if (tpb < 128) return false;
  if (tpb > ((wide || tile) ? gzk::MAX_TPB_WIDE : gzk::MAX_TPB)) return false;
  return gzk::lds_bytes(wide ? 1u : 0u, tpb) <= c->lds_max;
}

bool params_ok(const gz_params* p, uint32_t& L) {
  L = (p && p->block_len) ? p->block_len : (p && p->mode == 1 ? 64 : 32);
  if (!valid_L(L)) return false;
  if (p) {
    if (!tpb_ok(p->threads)) return false;
    if (p->mode > 1) return false;
    if (p->mode == 0 && p->nx != 0) return false;
    if (p->mode == 1 && (L != 64 || p->nx == 0 || p->nx % 8 != 0 || p->select > 2)) return false;
  }
  return true;
}

bool tile_mode(const gz_params* p) { return p && p->mode == 1; }

// Per-wave kernels exist for 1D decoding of either type (op 1), fp32 1D
// encoding, the fused step and decode-and-accumulate (ops 0, 2, 3), and
// need their LDS.
bool wave_fits(const gz_ctx* c, uint32_t op, uint32_t dt) {
  if (op == 1) return gzk::wave_decode_lds(dt) <= c->lds_max;
  if (op == 3) return dt == GZ_F32 && gzk::wave_decode_lds(GZ_F32) <= c->lds_max;
  return (op == 0 || op == 2) && dt == GZ_F32 && gzk::wave_encode_lds() <= c->lds_max;
}

// Measured defaults: the per-wave kernels for decoding (single streams and
// batches) and the fused step; strips for compression and decode-and-
// accumulate (1 GiB: 417 vs 455 us and 436 vs 478 us; there four waves per
// SIMD hide the input and accumulator loads, where the per-wave kernels
// have two) and for scatter decoding (an offset read per superblock).
bool wave_default(uint32_t op) { return op == 1 || op == 2; }

// Whether a single 1D call takes the per-wave kernel: asked for (threads
// 64), tuned, or by default (no threads, grid or tuned shape).
bool wave_wanted(const gz_ctx* c, uint32_t op, uint32_t dt, uint32_t L, const gz_params* p) {
  if (p && p->threads) return p->threads == WAVE_TPB;
  if (p && p->grid) return false;
  const Tuned& t = c->tuned[tune_op(op)][dt][log2_of(L) - 5];
  return t.tpb ? t.tpb == WAVE_TPB : wave_default(op);
}

gz_status hip_status(hipError_t e) { return e == hipSuccess ? GZ_OK : GZ_EHIP; }

// Copies descriptors and the strip map into the context arena on `st`.
gz_status stage_upload(gz_ctx* c, const std::vector<Job>& jobs,
                       const std::vector<uint32_t>& map, hipStream_t st) {
  const size_t jb = jobs.size() * sizeof(Job), mb = map.size() * sizeof(uint32_t);
  if (jb + mb > c->stage_bytes) return GZ_ENOSPC;
  const int k = c->stage_next;
  c->stage_next = (k + 1) % STAGE_SLOTS;
  if (c->stage_used[k] && hipEventSynchronize(c->stage_ev[k]) != hipSuccess) return GZ_EHIP;
  memcpy(c->stage[k], jobs.data(), jb);
  memcpy(c->stage[k] + jb, map.data(), mb);
  if (hipMemcpyAsync(c->d_jobs, c->stage[k], jb, hipMemcpyHostToDevice, st) != hipSuccess ||
      hipMemcpyAsync(c->d_map, c->stage[k] + jb, mb, hipMemcpyHostToDevice, st) != hipSuccess ||
      hipEventRecord(c->stage_ev[k], st) != hipSuccess)
    return GZ_EHIP;
  c->stage_used[k] = true;
  return GZ_OK;
}

// Ticket order of a batch's strips as (job, strip) pairs.  Jobs that are
// chains of their own are interleaved round-robin (strip r of every job
// before strip r + 1 of any), which keeps each chain's in-flight depth
// small; a chain running through several jobs keeps job order.  Either way
// a strip's look-back predecessors hold earlier tickets.
void fill_map(const std::vector<Job>& jobs, bool interleave, std::vector<uint32_t>& map) {
  uint64_t total = 0;
  for (const Job& J : jobs) total += J.nstrips;
  map.resize(2 * total);
  size_t k = 0;
  if (!interleave) {
    for (uint32_t j = 0; j < (uint32_t)jobs.size(); ++j)
      for (uint64_t r = 0; r < jobs[j].nstrips; ++r) {
        map[k++] = j;
        map[k++] = (uint32_t)r;
      }
    return;
  }
  std::vector<uint32_t> live;
  for (uint32_t j = 0; j < (uint32_t)jobs.size(); ++j)
    if (jobs[j].nstrips) live.push_back(j);
  for (uint64_t r = 0; !live.empty(); ++r) {
    size_t keep = 0;
    for (uint32_t j : live) {
      map[k++] = j;
      map[k++] = (uint32_t)r;
      if (r + 1 < jobs[j].nstrips) live[keep++] = j;
    }
    live.resize(keep);
  }
}

// Job count when all jobs have the same number of strips (the kernels then
// derive a ticket's job and strip from the interleaved order), else 0.
uint32_t uniform_jobs(const std::vector<Job>& jobs) {
  for (const Job& J : jobs)
    if (J.nstrips != jobs[0].nstrips) return 0;
  return (uint32_t)jobs.size();
}

// Per-wave shares of an fp32 1D decoding batch of `total` superblocks:
// (job, first superblock, stride) triples, each job given waves in
// proportion to its superblocks (at least one) out of the waves the
// per-wave decoder is launched with; empty where that does not apply
// (accumulation, fp64, tiles, more jobs than waves), and the (job,
// superblock) map is used instead.
std::vector<uint32_t> wave_job_shares(const gz_ctx* c, gz_op op, const std::vector<Job>& jobs,
                                      bool wide, uint64_t total) {
  std::vector<uint32_t> m;
  if (op != GZ_OP_DECOMPRESS || wide || jobs.empty() || total == 0) return m;
  for (const Job& J : jobs)
    if (J.dtype != 0 || J.mode != 0 || J.NS == 0) return m;
  constexpr uint64_t WV = gzk::DEC_WAVES_F32;  // the launch: one workgroup per CU at most
  const uint64_t W = std::min<uint64_t>((uint64_t)c->cus, (total + WV - 1) / WV) * WV;
  if (jobs.size() > W) return m;
  std::vector<uint64_t> cnt(jobs.size());
  uint64_t sum = 0;
  for (size_t j = 0; j < jobs.size(); ++j) {
    cnt[j] = std::max<uint64_t>(1, W * jobs[j].NS / total);
    sum += cnt[j];
  }
  while (sum > W) {  // the minimum of one wave per job may overshoot
    auto it = std::max_element(cnt.begin(), cnt.end());
    if (*it <= 1) return m;
    --*it;
    --sum;
  }
  m.reserve(3 * sum);
  for (size_t j = 0; j < jobs.size(); ++j)
    for (uint64_t i = 0; i < cnt[j]; ++i) {
      m.push_back((uint32_t)j);
      m.push_back((uint32_t)i);
      m.push_back((uint32_t)cnt[j]);
    }
  return m;
}

// Builds the jobs of a request batch; fills the strip map.
gz_status build_requests(gz_ctx* c, gz_op op, const gz_request* r, uint32_t nreq, uint32_t tpb,
                         std::vector<Job>& jobs, std::vector<uint32_t>& map) {
  if (!r || nreq == 0 || nreq > c->max_jobs) return GZ_EINVAL;
  jobs.resize(nreq);
  uint64_t strip = 0;
  for (uint32_t j = 0; j < nreq; ++j) {
    const gz_request& q = r[j];
    Job J;
    memset(&J, 0, sizeof J);
    if (q.dtype != GZ_F32 && q.dtype != GZ_F64) return GZ_EINVAL;
    // block length 0: the context's tuned length for the dtype (gz_tune);
    // a decoded stream must declare the length it was written with
    const uint32_t L = q.block_len ? q.block_len : (c->best_L[q.dtype] ? c->best_L[q.dtype] : 32);
    if (!valid_L(L)) return GZ_EINVAL;
    if ((op == GZ_OP_FUSED || op == GZ_OP_ACCUMULATE) && q.dtype != GZ_F32)
      return GZ_EUNSUPPORTED;
    if (q.n && (!q.in || !q.out)) return GZ_EINVAL;
    if (q.n * (uint64_t)esize(q.dtype) >= (1ull << 34)) return GZ_EINVAL;
    J.dtype = q.dtype;
    J.in = job_ptr(q.in);
    J.out = job_ptr(q.out);
    J.local = job_ptr(q.local);
    J.out_bytes = job_ptr((unsigned long long*)q.d_out_bytes);
    J.in_bytes = q.in_bytes;
    J.job = j;
    set_geom(J, q.n, L, tpb);
    if (op == GZ_OP_ACCUMULATE) {
      if (!q.in || overlaps(q.in, q.in_bytes, q.out, q.n * 4)) return GZ_EINVAL;
    } else if (op != GZ_OP_DECOMPRESS) {
      if (!set_bound(J, q.dtype, q.eb)) return GZ_EINVAL;
      if (q.out_cap < bound_of(q.n, q.dtype, L)) return GZ_ENOSPC;
      if (op == GZ_OP_FUSED && q.n && !q.local) return GZ_EINVAL;
      if (overlaps(q.in, op == GZ_OP_FUSED ? q.in_bytes : q.n * esize(q.dtype), q.out, q.out_cap))
        return GZ_EINVAL;
    } else {
      if (!q.in) return GZ_EINVAL;
    }
    J.strip0 = J.chain0 = strip;
    strip += J.nstrips;
    jobs[j] = J;
  }
  if (strip > c->max_strips || strip >= (1ull << 32)) return GZ_ENOSPC;
  fill_map(jobs, true, map);
  return GZ_OK;
}

// Workgroup size of a batched launch: the caller's, else the tuned one for
// (op, batch holds fp64) (gz_tune_batch), else the single-call default of
// the widest element type.
uint32_t batch_tpb(const gz_ctx* c, gz_op op, const gz_request* r, uint32_t nreq,
                   const gz_params* p, bool& wide) {
  wide = false;
  for (uint32_t j = 0; j < nreq; ++j) wide = wide || r[j].dtype == GZ_F64;
  if (p && p->threads && p->threads != WAVE_TPB) return p->threads;
  const Tuned& t = c->batch_tuned[op][wide ? 1 : 0];
  if (t.tpb && t.tpb != WAVE_TPB) return t.tpb;
  return pick_tpb(c, op, wide ? GZ_F64 : GZ_F32, 32, nullptr);
}

// A batch the per-wave encoding kernels take: compression or the fused
// step, every job fp32 with the same block length and superblock count.
bool batch_wave_ok(const gz_ctx* c, gz_op op, const std::vector<Job>& jobs) {
  if ((op != GZ_OP_COMPRESS && op != GZ_OP_FUSED) || jobs.empty() || !wave_fits(c, op, GZ_F32))
    return false;
  for (const Job& J : jobs)
    if (J.dtype != GZ_F32 || J.log2L != jobs[0].log2L || J.NS != jobs[0].NS || J.NS == 0)
      return false;
  const uint64_t total = jobs.size() * gzk::wave_rounds(jobs[0].NS);
  return total <= c->max_strips && total < (1ull << 32);
}

// Whether a batch takes the per-wave kernels when it can: asked for
// (threads 64), tuned, or by default.
bool batch_wave_wanted(const gz_ctx* c, gz_op op, const gz_params* p, bool wide = false) {
  if (p && p->threads) return p->threads == WAVE_TPB;
  if (p && p->grid) return false;
  const Tuned& t = c->batch_tuned[op][wide ? 1 : 0];
  return t.tpb ? t.tpb == WAVE_TPB : wave_default(op);
}

// The superblocks of a per-wave decoding batch as (job, superblock) pairs,
// job by job; none when every job has the same superblock count (the kernel
// then derives them).  Returns the number of superblocks.
uint64_t wave_decode_map(const std::vector<Job>& jobs, std::vector<uint32_t>& map) {
  map.clear();
  uint64_t total = 0;
  bool uniform = true;
  for (const Job& J : jobs) {
    total += J.NS;
    uniform = uniform && J.NS == jobs[0].NS;
  }
  if (uniform || total > (1ull << 31)) return total;
  map.reserve(2 * total);
  for (uint32_t j = 0; j < (uint32_t)jobs.size(); ++j)
    for (uint64_t sb = 0; sb < jobs[j].NS; ++sb) {
      map.push_back(j);
      map.push_back((uint32_t)sb);
    }
  return total;
}

// A batch the per-wave decoders take: decoding, or fp32 decode-and-
// accumulate, every job with at least one superblock (an empty stream's
// header is checked by a strip), within the context's map capacity.
bool batch_decode_wave_ok(const gz_ctx* c, gz_op op, const std::vector<Job>& jobs, bool wide,
                          uint64_t total) {
  if (op != GZ_OP_DECOMPRESS && op != GZ_OP_ACCUMULATE) return false;
  if (!wave_fits(c, op, wide ? GZ_F64 : GZ_F32)) return false;
  for (const Job& J : jobs)
    if (J.NS == 0) return false;
  return total > 0 && total <= c->max_strips && total < (1ull << 32);
}

uint32_t batch_grid(const gz_ctx* c, gz_op op, bool wide, uint32_t tpb, uint64_t total,
                    const gz_params* p) {
  uint64_t g;
  const Tuned& t = c->batch_tuned[op][wide ? 1 : 0];
  if (p && p->grid) g = p->grid;
  else if (t.grid && t.tpb == tpb) g = t.grid;
  else g = (uint64_t)c->cus * gzk::occupancy_blocks(gzk::OCC_BATCH + (uint32_t)op, wide, 5, tpb);
  return (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(g, total));
}

}  // namespace

extern "C" {

const char* gz_status_str(gz_status s) {
  switch (s) {
    case GZ_OK: return "ok";
    case GZ_EINVAL: return "invalid argument";
    case GZ_ENOSPC: return "insufficient capacity";
    case GZ_ECORRUPT: return "corrupt or mismatching stream";
    case GZ_EHIP: return "HIP runtime error";
    case GZ_ENOMEM: return "out of memory";
    case GZ_EUNSUPPORTED: return "unsupported combination";
    case GZ_ETIMEOUT: return "device wait timed out";
  }
  return "unknown status";
}

uint64_t gz_compress_bound(uint64_t n, gz_dtype dtype, uint32_t block_len) {
  if (!valid_L(block_len) || (dtype != GZ_F32 && dtype != GZ_F64)) return 0;
  return bound_of(n, dtype, block_len);
}

gz_status gz_ctx_create(gz_ctx** out, int device, uint64_t max_elems, uint32_t max_requests) {
  if (!out) return GZ_EINVAL;
  *out = nullptr;
  if (max_requests == 0) max_requests = 1;
  if (hipSetDevice(device) != hipSuccess) return GZ_EHIP;
  gz_ctx* c = new (std::nothrow) gz_ctx();
  if (!c) return GZ_ENOMEM;
  c->device = device;
  if (hipDeviceGetAttribute(&c->cus, hipDeviceAttributeMultiprocessorCount, device) !=
      hipSuccess) {
    delete c;
    return GZ_EHIP;
  }
  int wclk_khz = 0;
  if (hipDeviceGetAttribute(&wclk_khz, hipDeviceAttributeWallClockRate, device) != hipSuccess ||
      wclk_khz <= 0)
    wclk_khz = 100000;
  c->wclk_khz = (uint64_t)wclk_khz;
  c->wait_ticks = (uint64_t)wclk_khz * 1000ull;
  int lds = 0;
  if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device) != hipSuccess ||
      lds <= 0)
    lds = 65536;
  c->lds_max = (size_t)lds;
  c->max_elems = max_elems;
  c->max_jobs = max_requests;
  // strips of the smallest workgroup (128 lanes = 4096 elements), plus one
  // partial strip per request
  c->max_strips = cdiv(max_elems, 128 * gzk::SEG) + max_requests + 1;
  bool ok = true;
  ok = ok && hipMalloc((void**)&c->ctrl, sizeof(Ctrl)) == hipSuccess;
  ok = ok && hipMalloc((void**)&c->status, c->max_strips * 8) == hipSuccess;
  ok = ok && hipMalloc((void**)&c->jobbase, (size_t)max_requests * 8) == hipSuccess;
  ok = ok && hipMalloc((void**)&c->blob, 1024) == hipSuccess;
  ok = ok && hipMalloc((void**)&c->d_jobs, (size_t)max_requests * sizeof(Job)) == hipSuccess;
  ok = ok && hipMalloc((void**)&c->d_map, c->max_strips * 8) == hipSuccess;
  ok = ok && hipMalloc((void**)&c->train_ws, gzs::mlp_workspace_bytes()) == hipSuccess;
  // live plans may hold up to 16 batches' worth of descriptors and maps
  c->plan_jobs_arena.cap = 16ull * max_requests + 64;
  c->plan_map_arena.cap = 16ull * 2 * c->max_strips + 1024;
  ok = ok && hipMalloc((void**)&c->plan_jobs, c->plan_jobs_arena.cap * sizeof(Job)) == hipSuccess;
  ok = ok && hipMalloc((void**)&c->plan_map, c->plan_map_arena.cap * 4) == hipSuccess;
  c->stage_bytes = (size_t)max_requests * sizeof(Job) + c->max_strips * 8;
  for (int k = 0; ok && k < STAGE_SLOTS; ++k) {
    ok = hipHostMalloc((void**)&c->stage[k], c->stage_bytes, hipHostMallocDefault) == hipSuccess &&
         hipEventCreateWithFlags(&c->stage_ev[k], hipEventDisableTiming) == hipSuccess;
  }
  if (ok) {
    Ctrl init;
    memset(&init, 0, sizeof init);
    init.epoch = 1;
    ok = hipMemcpy(c->ctrl, &init, sizeof init, hipMemcpyHostToDevice) == hipSuccess &&
         hipMemset(c->status, 0, c->max_strips * 8) == hipSuccess &&
         hipMemset(c->jobbase, 0, (size_t)max_requests * 8) == hipSuccess &&
         hipMemset(c->blob, 0, 1024) == hipSuccess && hipDeviceSynchronize() == hipSuccess;
  }
  if (!ok) {
    gz_ctx_destroy(c);
    return GZ_ENOMEM;
  }
  *out = c;
  return GZ_OK;
}

void gz_ctx_destroy(gz_ctx* c) {
  if (!c) return;
  for (gz_plan* pl : c->live_plans) pl->ctx = nullptr;  // orphaned: destroy only
  for (int k = 0; k < STAGE_SLOTS; ++k) {
    if (c->stage_ev[k]) {
      (void)hipEventSynchronize(c->stage_ev[k]);
      (void)hipEventDestroy(c->stage_ev[k]);
    }
    if (c->stage[k]) (void)hipHostFree(c->stage[k]);
  }
  (void)hipFree(c->ctrl);
  (void)hipFree(c->status);
  (void)hipFree(c->jobbase);
  (void)hipFree(c->blob);
  (void)hipFree(c->d_jobs);
  (void)hipFree(c->d_map);
  (void)hipFree(c->train_ws);
  (void)hipFree(c->plan_jobs);
  (void)hipFree(c->plan_map);
  delete c;
}

gz_status gz_ctx_status(gz_ctx* c, gz_stream_t stream, gz_status* dev) {
  if (!c || !dev) return GZ_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  // the word is read after the stream's work, on the stream, into pageable
  // host memory (a synchronous copy) -- only this stream is waited for
  uint32_t err = 0;
  if (hipStreamSynchronize(st) != hipSuccess ||
      hipMemcpyAsync(&err, &c->ctrl->err, 4, hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return GZ_EHIP;
  *dev = (err & gzk::ERRF_CORRUPT) ? GZ_ECORRUPT : (err & gzk::ERRF_TIMEOUT) ? GZ_ETIMEOUT : GZ_OK;
  if (err) {
    static const uint32_t z = 0;
    if (hipMemcpyAsync(&c->ctrl->err, &z, 4, hipMemcpyHostToDevice, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      return GZ_EHIP;
  }
  return GZ_OK;
}

gz_status gz_ctx_reset(gz_ctx* c, gz_stream_t stream) {
  if (!c) return GZ_EINVAL;
  return hip_status(gzk::launch_reset(c->ctl(), (hipStream_t)stream));
}

gz_status gz_ctx_set_wait(gz_ctx* c, uint64_t usec) {
  if (!c || usec > (1ull << 40)) return GZ_EINVAL;
  c->wait_ticks = usec * c->wclk_khz / 1000ull;
  return GZ_OK;
}

gz_status gz_quantize(gz_ctx* c, const void* d_in, uint64_t n, gz_dtype dtype, double eb,
                      int32_t* d_q, uint8_t* d_fail, gz_stream_t stream) {
  if (!c || (dtype != GZ_F32 && dtype != GZ_F64)) return GZ_EINVAL;
  if (n && (!d_in || !d_q || !d_fail)) return GZ_EINVAL;
  Job J;
  memset(&J, 0, sizeof J);
  J.dtype = dtype;
  if (!set_bound(J, dtype, eb)) return GZ_EINVAL;
  if (!n) return GZ_OK;
  return hip_status(gzk::launch_quantize(d_in, n, J, d_q, d_fail, (hipStream_t)stream));
}

}  // extern "C"

namespace {

// Validates a compression and enqueues its one launch on the context's
// workspace (a real context, or the device-resident one of
// gz_compress_noalloc).
gz_status compress_impl(gz_ctx* c, const void* d_in, uint64_t n, gz_dtype dtype, double eb,
                        const gz_params* p, void* d_out, uint64_t out_cap,
                        uint64_t* d_out_bytes, gz_stream_t stream) {
  uint32_t L;
  if (!c || !d_out || (dtype != GZ_F32 && dtype != GZ_F64) || !params_ok(p, L))
    return GZ_EINVAL;
  if (n && !d_in) return GZ_EINVAL;
  if (n * (uint64_t)esize(dtype) >= (1ull << 34)) return GZ_EINVAL;
  if (out_cap < bound_of(n, dtype, L)) return GZ_ENOSPC;
  if (overlaps(d_in, n * esize(dtype), d_out, out_cap)) return GZ_EINVAL;
  Job J;
  memset(&J, 0, sizeof J);
  J.dtype = dtype;
  if (!set_bound(J, dtype, eb)) return GZ_EINVAL;
  // per-wave encoding takes one look-back word per round of 8 superblocks; a
  // stream with more rounds than the workspace has words falls back to
  // strips unless the caller asked for waves
  if (!tile_mode(p) && n && wave_wanted(c, 0, dtype, L, p) && wave_fits(c, 0, dtype)) {
    set_geom(J, n, L, gzk::MAX_TPB);
    if (gzk::wave_rounds(J.NS) <= c->max_strips) {
      J.in = job_ptr(d_in);
      J.out = job_ptr(d_out);
      J.out_bytes = job_ptr((unsigned long long*)d_out_bytes);
      return hip_status(gzk::launch_encode_wave(0, nullptr, J, 1,
                                                (uint32_t)gzk::wave_rounds(J.NS), J.log2L,
                                                c->ctl(), (uint32_t)c->cus,
                                                (hipStream_t)stream));
    }
    if (p && p->threads == WAVE_TPB) return GZ_ENOSPC;
  }
  gz_params q;  // an empty stream asked for waves: one default strip writes its header
  if (!n && p && p->threads == WAVE_TPB && !tile_mode(p) && wave_fits(c, 0, dtype)) {
    q = *p;
    q.threads = q.grid = 0;
    p = &q;
  }
  const uint32_t tpb = pick_tpb(c, 0, dtype, L, p);
  if (!tpb_fits(c, dtype == GZ_F64, tile_mode(p), tpb)) return GZ_EUNSUPPORTED;
  set_geom(J, n, L, tpb);
  if (J.nstrips > c->max_strips) return GZ_ENOSPC;
  J.in = job_ptr(d_in);
  J.out = job_ptr(d_out);
  J.out_bytes = job_ptr((unsigned long long*)d_out_bytes);
  if (tile_mode(p)) {
    if (dtype != GZ_F32) return GZ_EUNSUPPORTED;
    if (n % (8ull * p->nx) != 0) return GZ_EINVAL;
    if (p->select == 0 && !c->blob_loaded) return GZ_EINVAL;
    J.mode = 1;
    J.nx = p->nx;
    J.select = p->select;
    const uint32_t grid = pick_tile_grid(c, gzk::OCC_TILE_C, tpb, J.nstrips, p);
    return hip_status(gzk::launch_tiles(0, J, c->ctl(), tpb, grid, (hipStream_t)stream));
  }
  const uint32_t grid = pick_grid(c, 0, dtype, L, tpb, J.nstrips, p);
  return hip_status(gzk::launch_single(0, J, c->ctl(), tpb, grid, (hipStream_t)stream));
}

}  // namespace

extern "C" {

gz_status gz_compress(gz_ctx* c, const void* d_in, uint64_t n, gz_dtype dtype, double eb,
                      const gz_params* p, void* d_out, uint64_t out_cap, uint64_t* d_out_bytes,
                      gz_stream_t stream) {
  return compress_impl(c, d_in, n, dtype, eb, p, d_out, out_cap, d_out_bytes, stream);
}

gz_status gz_decompress(gz_ctx* c, const void* d_in, uint64_t in_bytes, uint64_t n,
                        gz_dtype dtype, const gz_params* p, void* d_out, gz_stream_t stream) {
  uint32_t L;
  if (!c || !d_in || (dtype != GZ_F32 && dtype != GZ_F64) || !params_ok(p, L)) return GZ_EINVAL;
  if (n && !d_out) return GZ_EINVAL;
  if (n * (uint64_t)esize(dtype) >= (1ull << 34)) return GZ_EINVAL;
  if (overlaps(d_in, in_bytes, d_out, n * esize(dtype))) return GZ_EINVAL;
  Job J;
  memset(&J, 0, sizeof J);
  J.dtype = dtype;
  if (!tile_mode(p) && wave_wanted(c, 1, dtype, L, p) && wave_fits(c, 1, dtype)) {
    set_geom(J, n, L, gzk::MAX_TPB);
    J.in = job_ptr(d_in);
    J.in_bytes = in_bytes;
    J.out = job_ptr(d_out);
    return hip_status(gzk::launch_decompress_wave(J, c->ctl(), (uint32_t)c->cus,
                                                  (hipStream_t)stream));
  }
  const uint32_t tpb = pick_tpb(c, 1, dtype, L, p);
  if (!tpb_fits(c, dtype == GZ_F64, tile_mode(p), tpb)) return GZ_EUNSUPPORTED;
  set_geom(J, n, L, tpb);
  if (J.nstrips > c->max_strips) return GZ_ENOSPC;
  J.in = job_ptr(d_in);
  J.in_bytes = in_bytes;
  J.out = job_ptr(d_out);
  if (tile_mode(p)) {
    if (dtype != GZ_F32) return GZ_EUNSUPPORTED;
    if (n % (8ull * p->nx) != 0) return GZ_EINVAL;
    J.mode = 1;
    J.nx = p->nx;
    const uint32_t grid = pick_tile_grid(c, gzk::OCC_TILE_D, tpb, J.nstrips, p);
    return hip_status(gzk::launch_tiles(1, J, c->ctl(), tpb, grid, (hipStream_t)stream));
  }
  const uint32_t grid = pick_grid(c, 1, dtype, L, tpb, J.nstrips, p);
  return hip_status(gzk::launch_single(1, J, c->ctl(), tpb, grid, (hipStream_t)stream));
}

gz_status gz_fused_reduce_step(gz_ctx* c, const void* d_cmp_in, uint64_t in_bytes,
                               const float* d_local, uint64_t n, double eb, const gz_params* p,
                               void* d_cmp_out, uint64_t out_cap, uint64_t* d_out_bytes,
                               gz_stream_t stream) {
  uint32_t L;
  if (!c || !d_cmp_in || !d_cmp_out || !params_ok(p, L) || tile_mode(p)) return GZ_EINVAL;
  if (n && !d_local) return GZ_EINVAL;
  if (n * 4ull >= (1ull << 34)) return GZ_EINVAL;
  if (out_cap < bound_of(n, GZ_F32, L)) return GZ_ENOSPC;
  if (overlaps(d_cmp_in, in_bytes, d_cmp_out, out_cap) ||
      overlaps(d_local, n * 4, d_cmp_out, out_cap))
    return GZ_EINVAL;
  Job J;
  memset(&J, 0, sizeof J);
  J.dtype = GZ_F32;
  if (!set_bound(J, GZ_F32, eb)) return GZ_EINVAL;
  J.in = job_ptr(d_cmp_in);
  J.in_bytes = in_bytes;
  J.local = job_ptr(d_local);
  J.out = job_ptr(d_cmp_out);
  J.out_bytes = job_ptr((unsigned long long*)d_out_bytes);
  if (n && wave_wanted(c, 2, GZ_F32, L, p) && wave_fits(c, 2, GZ_F32)) {
    set_geom(J, n, L, gzk::MAX_TPB);
    if (gzk::wave_rounds(J.NS) <= c->max_strips)
      return hip_status(gzk::launch_encode_wave(2, nullptr, J, 1,
                                                (uint32_t)gzk::wave_rounds(J.NS), J.log2L,
                                                c->ctl(), (uint32_t)c->cus,
                                                (hipStream_t)stream));
    if (p && p->threads == WAVE_TPB) return GZ_ENOSPC;
  }
  gz_params q;  // an empty stream asked for waves: one default strip writes its header
  if (!n && p && p->threads == WAVE_TPB) {
    q = *p;
    q.threads = q.grid = 0;
    p = &q;
  }
  const uint32_t tpb = pick_tpb(c, 2, GZ_F32, L, p);
  if (!tpb_fits(c, false, false, tpb)) return GZ_EUNSUPPORTED;
  set_geom(J, n, L, tpb);
  if (J.nstrips > c->max_strips) return GZ_ENOSPC;
  const uint32_t grid = pick_grid(c, 2, GZ_F32, L, tpb, J.nstrips, p);
  return hip_status(gzk::launch_single(2, J, c->ctl(), tpb, grid, (hipStream_t)stream));
}

gz_status gz_decompress_add(gz_ctx* c, const void* d_in, uint64_t in_bytes, uint64_t n,
                            const gz_params* p, float* d_acc, gz_stream_t stream) {
  uint32_t L;
  if (!c || !d_in || !params_ok(p, L) || tile_mode(p)) return GZ_EINVAL;
  if (n && !d_acc) return GZ_EINVAL;
  if (n * 4ull >= (1ull << 34)) return GZ_EINVAL;
  if (overlaps(d_in, in_bytes, d_acc, n * 4)) return GZ_EINVAL;
  Job J;
  memset(&J, 0, sizeof J);
  J.dtype = GZ_F32;
  J.in = job_ptr(d_in);
  J.in_bytes = in_bytes;
  J.out = job_ptr(d_acc);
  if (wave_wanted(c, 3, GZ_F32, L, p) && wave_fits(c, 3, GZ_F32)) {
    set_geom(J, n, L, gzk::MAX_TPB);
    return hip_status(gzk::launch_accum_wave(J, c->ctl(), (uint32_t)c->cus, (hipStream_t)stream));
  }
  const uint32_t tpb = pick_tpb(c, 3, GZ_F32, L, p);
  if (!tpb_fits(c, false, false, tpb)) return GZ_EUNSUPPORTED;
  set_geom(J, n, L, tpb);
  if (J.nstrips > c->max_strips) return GZ_ENOSPC;
  const uint32_t grid = pick_grid(c, 3, GZ_F32, L, tpb, J.nstrips, p);
  return hip_status(gzk::launch_single(3, J, c->ctl(), tpb, grid, (hipStream_t)stream));
}

gz_status gz_scatter_compress(gz_ctx* c, const void* d_root, gz_dtype dtype,
                              const uint64_t* h_counts, const uint64_t* h_displs,
                              uint32_t nchunks, double eb, const gz_params* p, void* d_out,
                              uint64_t out_cap, uint64_t* d_chunk_bytes,
                              uint64_t* d_chunk_offsets, gz_stream_t stream) {
  uint32_t L;
  if (!c || !d_root || !d_out || !h_counts || !h_displs || !d_chunk_bytes || !d_chunk_offsets ||
      (dtype != GZ_F32 && dtype != GZ_F64) || !params_ok(p, L) || tile_mode(p) || nchunks == 0)
    return GZ_EINVAL;
  if (nchunks > c->max_jobs) return GZ_ENOSPC;
  const uint32_t tpb = pick_tpb(c, 0, dtype, L, p);
  if (!tpb_fits(c, dtype == GZ_F64, false, tpb)) return GZ_EUNSUPPORTED;
  std::vector<Job> jobs(nchunks);
  Job proto;
  memset(&proto, 0, sizeof proto);
  proto.dtype = dtype;
  if (!set_bound(proto, dtype, eb)) return GZ_EINVAL;
  uint64_t strip = 0, fixed = 0, need = 0, pay = 0, span = 0;
  for (uint32_t j = 0; j < nchunks; ++j) {
    Job J = proto;
    const uint64_t n = h_counts[j];
    if (n * (uint64_t)esize(dtype) >= (1ull << 34)) return GZ_EINVAL;
    span = std::max(span, h_displs[j] + n);
    set_geom(J, n, L, tpb);
    J.in = job_ptr((const uint8_t*)d_root + h_displs[j] * esize(dtype));
    J.out = job_ptr(d_out);
    J.out_bytes = job_ptr((unsigned long long*)(d_chunk_bytes + j));
    J.chunk_off = job_ptr((unsigned long long*)(d_chunk_offsets + j));
    J.fixed_off = fixed;
    J.strip0 = strip;
    J.chain0 = 0;
    J.job = j;
    fixed += fixed_of(n, L);
    need += bound_of(n, dtype, L);
    pay += n * esize(dtype) / 4;
    strip += J.nstrips;
    jobs[j] = J;
  }
  if (out_cap < need) return GZ_ENOSPC;
  if (pay > MAX_CHAIN_DW) return GZ_EINVAL;
  if (strip > c->max_strips) return GZ_ENOSPC;
  if (overlaps(d_root, span * esize(dtype), d_out, out_cap)) return GZ_EINVAL;
  std::vector<uint32_t> map;
  fill_map(jobs, false, map);  // one chain through all chunks
  hipStream_t st = (hipStream_t)stream;
  gz_status r = stage_upload(c, jobs, map, st);
  if (r != GZ_OK) return r;
  const uint32_t grid = pick_grid(c, 0, dtype, L, tpb, strip, p);
  return hip_status(gzk::launch_batch(0, c->d_jobs, c->d_map, 0, (uint32_t)strip, c->ctl(), tpb,
                                      grid, dtype == GZ_F64, st));
}

gz_status gz_scatter_decompress(gz_ctx* c, const void* d_packed, uint64_t packed_bytes,
                                const uint64_t* d_chunk_offsets, gz_dtype dtype,
                                const uint64_t* h_counts, const uint64_t* h_displs,
                                uint32_t nchunks, const gz_params* p, void* d_root,
                                gz_stream_t stream) {
  uint32_t L;
  if (!c || !d_packed || !d_chunk_offsets || !h_counts || !h_displs || !d_root ||
      (dtype != GZ_F32 && dtype != GZ_F64) || !params_ok(p, L) || tile_mode(p) || nchunks == 0)
    return GZ_EINVAL;
  if (nchunks > c->max_jobs) return GZ_ENOSPC;
  // waves when asked for, or by default for fp32 chunks where each chunk can
  // have waves of its own (else strips)
  const bool asked = p && p->threads == WAVE_TPB;
  const bool dflt = (!p || (p->threads == 0 && p->grid == 0)) && dtype == GZ_F32;
  const bool want_wave = (asked || dflt) && wave_fits(c, 1, dtype);
  gz_params q;  // the strips' shape when waves were asked for (geometry, fallback)
  const gz_params* ps = p;
  if (p && p->threads == WAVE_TPB) {
    q = *p;
    q.threads = q.grid = 0;
    ps = &q;
  }
  const uint32_t tpb = pick_tpb(c, 1, dtype, L, ps);
  std::vector<Job> jobs(nchunks);
  uint64_t strip = 0, span = 0;
  for (uint32_t j = 0; j < nchunks; ++j) {
    Job J;
    memset(&J, 0, sizeof J);
    J.dtype = dtype;
    const uint64_t n = h_counts[j];
    if (n * (uint64_t)esize(dtype) >= (1ull << 34)) return GZ_EINVAL;
    span = std::max(span, h_displs[j] + n);
    set_geom(J, n, L, tpb);
    J.in = job_ptr(d_packed);
    J.in_off = job_ptr((const unsigned long long*)d_chunk_offsets);
    J.in_bytes = packed_bytes;
    J.out = job_ptr((uint8_t*)d_root + h_displs[j] * esize(dtype));
    J.strip0 = J.chain0 = strip;
    J.job = j;
    strip += J.nstrips;
    jobs[j] = J;
  }
  if (strip > c->max_strips) return GZ_ENOSPC;
  if (overlaps(d_packed, packed_bytes, d_root, span * esize(dtype))) return GZ_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  if (want_wave) {
    std::vector<uint32_t> smap;
    const uint64_t total = wave_decode_map(jobs, smap);
    if (batch_decode_wave_ok(c, GZ_OP_DECOMPRESS, jobs, dtype == GZ_F64, total)) {
      const std::vector<uint32_t> jm =
          wave_job_shares(c, GZ_OP_DECOMPRESS, jobs, dtype == GZ_F64, total);
      if (asked || !jm.empty()) {
        gz_status r = stage_upload(c, jobs, jm.empty() ? smap : jm, st);
        if (r != GZ_OK) return r;
        return hip_status(gzk::launch_decode_wave_batch(
            1, c->d_jobs, (smap.empty() && jm.empty()) ? nullptr : c->d_map, nchunks,
            (uint32_t)total, dtype == GZ_F64, (uint32_t)(jm.size() / 3), (uint32_t)c->cus,
            c->ctl(), st));
      }
    }
    if (asked) return GZ_EUNSUPPORTED;
  }
  if (!tpb_fits(c, dtype == GZ_F64, false, tpb)) return GZ_EUNSUPPORTED;
  std::vector<uint32_t> map;
  fill_map(jobs, true, map);
  gz_status r = stage_upload(c, jobs, map, st);
  if (r != GZ_OK) return r;
  const uint32_t grid = pick_grid(c, 1, dtype, L, tpb, strip, ps);
  return hip_status(gzk::launch_batch(1, c->d_jobs, c->d_map, uniform_jobs(jobs), (uint32_t)strip,
                                      c->ctl(), tpb,
                                      grid, dtype == GZ_F64, st));
}

gz_status gz_batch(gz_ctx* c, gz_op op, const gz_request* h_reqs, uint32_t nreq,
                   const gz_params* p, gz_stream_t stream) {
  if (!c || op > GZ_OP_ACCUMULATE) return GZ_EINVAL;
  if (p && !tpb_ok(p->threads)) return GZ_EINVAL;
  if (!h_reqs || nreq == 0) return GZ_EINVAL;
  bool wide;
  const uint32_t tpb = batch_tpb(c, op, h_reqs, nreq, p, wide);
  if (!tpb_fits(c, wide, false, tpb)) return GZ_EUNSUPPORTED;
  std::vector<Job> jobs;
  std::vector<uint32_t> map;
  gz_status r = build_requests(c, op, h_reqs, nreq, tpb, jobs, map);
  if (r != GZ_OK) return r;
  hipStream_t st = (hipStream_t)stream;
  if ((op == GZ_OP_DECOMPRESS || op == GZ_OP_ACCUMULATE) && batch_wave_wanted(c, op, p, wide)) {
    std::vector<uint32_t> smap;
    const uint64_t total = wave_decode_map(jobs, smap);
    if (batch_decode_wave_ok(c, op, jobs, wide, total)) {
      const std::vector<uint32_t> jm = wave_job_shares(c, op, jobs, wide, total);
      r = stage_upload(c, jobs, jm.empty() ? smap : jm, st);
      if (r != GZ_OK) return r;
      return hip_status(gzk::launch_decode_wave_batch(
          (uint32_t)op, c->d_jobs, (smap.empty() && jm.empty()) ? nullptr : c->d_map,
          (uint32_t)jobs.size(), (uint32_t)total, wide, (uint32_t)(jm.size() / 3),
          (uint32_t)c->cus, c->ctl(), st));
    }
    if (p && p->threads == WAVE_TPB) return GZ_EUNSUPPORTED;
  }
  const bool wave = !wide && batch_wave_wanted(c, op, p) && batch_wave_ok(c, op, jobs);
  if (p && p->threads == WAVE_TPB && !wave) return GZ_EUNSUPPORTED;
  r = stage_upload(c, jobs, map, st);
  if (r != GZ_OK) return r;
  if (wave)
    return hip_status(gzk::launch_encode_wave(
        (uint32_t)op, c->d_jobs, Job(), (uint32_t)jobs.size(),
        (uint32_t)(jobs.size() * gzk::wave_rounds(jobs[0].NS)), jobs[0].log2L, c->ctl(),
        (uint32_t)c->cus, st));
  const uint64_t total = map.size() / 2;
  const uint32_t g = batch_grid(c, op, wide, tpb, total, p);
  return hip_status(gzk::launch_batch((uint32_t)op, c->d_jobs, c->d_map, uniform_jobs(jobs),
                                      (uint32_t)total, c->ctl(), tpb, g, wide, st));
}

gz_status gz_plan_create(gz_ctx* c, gz_op op, const gz_request* h_reqs, uint32_t nreq,
                         const gz_params* p, gz_plan** out) {
  if (!c || !out || op > GZ_OP_ACCUMULATE) return GZ_EINVAL;
  *out = nullptr;
  if (p && !tpb_ok(p->threads)) return GZ_EINVAL;
  if (!h_reqs || nreq == 0) return GZ_EINVAL;
  bool wide;
  const uint32_t tpb = batch_tpb(c, op, h_reqs, nreq, p, wide);
  if (!tpb_fits(c, wide, false, tpb)) return GZ_EUNSUPPORTED;
  std::vector<Job> jobs;
  std::vector<uint32_t> map;
  gz_status r = build_requests(c, op, h_reqs, nreq, tpb, jobs, map);
  if (r != GZ_OK) return r;
  bool wave_dec = false;
  uint64_t dec_total = 0;
  uint32_t jw = 0;
  if ((op == GZ_OP_DECOMPRESS || op == GZ_OP_ACCUMULATE) && batch_wave_wanted(c, op, p, wide)) {
    std::vector<uint32_t> smap;
    dec_total = wave_decode_map(jobs, smap);
    wave_dec = batch_decode_wave_ok(c, op, jobs, wide, dec_total);
    if (wave_dec) {
      std::vector<uint32_t> jm = wave_job_shares(c, op, jobs, wide, dec_total);
      jw = (uint32_t)(jm.size() / 3);
      map.swap(jm.empty() ? smap : jm);
    } else if (p && p->threads == WAVE_TPB) {
      return GZ_EUNSUPPORTED;
    }
  }
  const bool wave = !wave_dec && !wide && batch_wave_wanted(c, op, p) && batch_wave_ok(c, op, jobs);
  if (p && p->threads == WAVE_TPB && !wave && !wave_dec) return GZ_EUNSUPPORTED;
  // a range released by gz_plan_destroy may still be read by a launch in
  // flight: the device finishes its work before the arena is written
  if (hipDeviceSynchronize() != hipSuccess) return GZ_EHIP;
  uint64_t jo = 0, mo = 0;
  if (!c->plan_jobs_arena.take(jobs.size(), jo)) return GZ_ENOSPC;
  if (!c->plan_map_arena.take(std::max<size_t>(map.size(), 1), mo)) {
    c->plan_jobs_arena.give(jo);
    return GZ_ENOSPC;
  }
  gz_plan* pl = new (std::nothrow) gz_plan();
  if (!pl) {
    c->plan_jobs_arena.give(jo);
    c->plan_map_arena.give(mo);
    return GZ_ENOMEM;
  }
  pl->ctx = c;
  pl->op = op;
  pl->jobs_off = jo;
  pl->map_off = mo;
  pl->d_jobs = c->plan_jobs + jo;
  pl->d_map = c->plan_map + mo;
  pl->total = (uint32_t)(map.size() / 2);
  pl->njobs = uniform_jobs(jobs);
  pl->tpb = tpb;
  pl->wide = wide;
  pl->grid = batch_grid(c, op, wide, tpb, pl->total, p);
  if (wave) {
    pl->wave = true;
    pl->njobs = (uint32_t)jobs.size();
    pl->total = (uint32_t)(jobs.size() * gzk::wave_rounds(jobs[0].NS));
    pl->log2L = jobs[0].log2L;
  }
  if (wave_dec) {
    pl->wave_dec = true;
    pl->has_map = !map.empty();
    pl->jw = jw;
    pl->njobs = (uint32_t)jobs.size();
    pl->total = (uint32_t)dec_total;
  }
  c->live_plans.push_back(pl);
  if (hipMemcpy(pl->d_jobs, jobs.data(), jobs.size() * sizeof(Job), hipMemcpyHostToDevice) !=
          hipSuccess ||
      (!map.empty() &&
       hipMemcpy(pl->d_map, map.data(), map.size() * 4, hipMemcpyHostToDevice) != hipSuccess)) {
    gz_plan_destroy(pl);
    return GZ_EHIP;
  }
  *out = pl;
  return GZ_OK;
}

gz_status gz_plan_launch(gz_plan* pl, gz_stream_t stream) {
  if (!pl || !pl->ctx) return GZ_EINVAL;
  if (pl->wave)
    return hip_status(gzk::launch_encode_wave(pl->op, pl->d_jobs, Job(), pl->njobs, pl->total,
                                              pl->log2L, pl->ctx->ctl(),
                                              (uint32_t)pl->ctx->cus, (hipStream_t)stream));
  if (pl->wave_dec)
    return hip_status(gzk::launch_decode_wave_batch(
        pl->op, pl->d_jobs, pl->has_map ? pl->d_map : nullptr, pl->njobs, pl->total, pl->wide,
        pl->jw, (uint32_t)pl->ctx->cus, pl->ctx->ctl(), (hipStream_t)stream));
  return hip_status(gzk::launch_batch(pl->op, pl->d_jobs, pl->d_map, pl->njobs, pl->total,
                                      pl->ctx->ctl(),
                                      pl->tpb, pl->grid, pl->wide, (hipStream_t)stream));
}

void gz_plan_destroy(gz_plan* pl) {
  if (!pl) return;
  if (gz_ctx* c = pl->ctx) {
    c->plan_jobs_arena.give(pl->jobs_off);
    c->plan_map_arena.give(pl->map_off);
    c->live_plans.erase(std::remove(c->live_plans.begin(), c->live_plans.end(), pl),
                        c->live_plans.end());
  }
  delete pl;
}

gz_status gz_graph_create(gz_plan* const* plans, uint32_t nplans, gz_graph** out) {
  if (!plans || !nplans || !out) return GZ_EINVAL;
  *out = nullptr;
  for (uint32_t i = 0; i < nplans; ++i)
    if (!plans[i] || plans[i]->ctx != plans[0]->ctx) return GZ_EINVAL;
  hipStream_t st;
  if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) return GZ_EHIP;
  gz_graph* g = new (std::nothrow) gz_graph();
  if (!g) {
    (void)hipStreamDestroy(st);
    return GZ_ENOMEM;
  }
  gz_status r = GZ_OK;
  if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess) r = GZ_EHIP;
  for (uint32_t i = 0; r == GZ_OK && i < nplans; ++i) r = gz_plan_launch(plans[i], st);
  hipGraph_t graph = nullptr;
  if (hipStreamEndCapture(st, &graph) != hipSuccess && r == GZ_OK) r = GZ_EHIP;
  if (r == GZ_OK && hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0) != hipSuccess)
    r = GZ_EHIP;
  g->graph = graph;
  (void)hipStreamDestroy(st);
  if (r != GZ_OK) {
    gz_graph_destroy(g);
    return r;
  }
  *out = g;
  return GZ_OK;
}

gz_status gz_graph_launch(gz_graph* g, gz_stream_t stream) {
  if (!g || !g->exec) return GZ_EINVAL;
  return hip_status(hipGraphLaunch(g->exec, (hipStream_t)stream));
}

void gz_graph_destroy(gz_graph* g) {
  if (!g) return;
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  delete g;
}

}  // extern "C"


extern "C" {

// ---- autotuner: launch shapes (threads, grid) and optionally block length.
// Shapes never change the bytes; block length does (it is recorded in the
// stream), so tuning it is opt-in (block_len == 0).
static bool cache_lookup(const char* path, const std::string& key, uint32_t& tpb,
                         uint32_t& grid) {
  if (!path) return false;
  FILE* f = fopen(path, "r");
  if (!f) return false;
  char line[512];
  bool hit = false;
  while (fgets(line, sizeof line, f)) {
    char k[256];
    unsigned t, g;
    // entries with a workgroup size or grid the kernels do not take are ignored
    if (sscanf(line, " {\"key\": \"%255[^\"]\", \"tpb\": %u, \"grid\": %u", k, &t, &g) == 3 &&
        key == k && t != 0 && tpb_ok(t) && g >= 1 && g <= 65536) {
      tpb = t;
      grid = g;
      hit = true;
    }
  }
  fclose(f);
  return hit;
}

static void cache_store(const char* path, const std::string& key, uint32_t tpb, uint32_t grid,
                        float ms) {
  if (!path) return;
  FILE* f = fopen(path, "a");
  if (!f) return;
  fprintf(f, "{\"key\": \"%s\", \"tpb\": %u, \"grid\": %u, \"ms\": %.4f}\n", key.c_str(),
          tpb, grid, ms);
  fclose(f);
}

static gz_status time_op(gz_ctx* c, uint32_t op, const void* x, void* y, void* s,
                         uint64_t cap, unsigned long long* nb, uint64_t n, gz_dtype dt,
                         uint32_t L, uint32_t tpb, uint32_t grid, hipStream_t st,
                         hipEvent_t e0, hipEvent_t e1, float& ms) {
  gz_params p = {L, tpb, grid, 0, 0, 0};
  auto run = [&]() -> gz_status {
    return op == 0 ? gz_compress(c, x, n, dt, 1e-3, &p, s, cap, (uint64_t*)nb, st)
                   : gz_decompress(c, s, cap, n, dt, &p, y, st);
  };
  gz_status r = run();
  if (r != GZ_OK) return r;
  if (hipEventRecord(e0, st) != hipSuccess) return GZ_EHIP;
  for (int k = 0; k < 3 && r == GZ_OK; ++k) r = run();
  if (r != GZ_OK) return r;
  if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess)
    return GZ_EHIP;
  if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) return GZ_EHIP;
  ms /= 3;
  return GZ_OK;
}

static uint64_t round256(uint64_t a) { return (a + 255) & ~255ull; }

gz_status gz_tune(gz_ctx* c, gz_dtype dt, uint32_t block_len, const void* d_sample, uint64_t n,
                  void* d_work, uint64_t work_bytes, const char* cache_path, gz_params* best,
                  gz_stream_t stream) {
  if (!c || (dt != GZ_F32 && dt != GZ_F64) || n == 0 || n > c->max_elems) return GZ_EINVAL;
  if (block_len != 0 && !valid_L(block_len)) return GZ_EINVAL;
  if (!d_sample || !d_work) return GZ_EINVAL;
  // the caller's work buffer: decoded values | stream (the largest bound of
  // the three lengths) | size word
  const uint64_t cap = bound_of(n, dt, 32);
  const uint64_t dec_b = round256(n * esize(dt)), str_b = round256(cap);
  if (work_bytes < dec_b + str_b + 8) return GZ_ENOSPC;
  if (overlaps(d_sample, n * esize(dt), d_work, work_bytes)) return GZ_EINVAL;
  uint8_t* w = (uint8_t*)d_work;
  void* y = w;
  void* s = w + dec_b;
  unsigned long long* nb = (unsigned long long*)(w + dec_b + str_b);
  const uint32_t Ls[3] = {32, 64, 128};
  hipStream_t st = (hipStream_t)stream;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  gz_status r = GZ_OK;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) r = GZ_EHIP;
  float best_total = 1e30f;
  uint32_t best_L = block_len ? block_len : 32;
  for (int li = 0; r == GZ_OK && li < 3; ++li) {
    const uint32_t L = Ls[li];
    if (block_len && L != block_len) continue;
    float total = 0;
    for (uint32_t op = 0; r == GZ_OK && op < 2; ++op) {
      char keyb[128];
      snprintf(keyb, sizeof keyb, "gfx950/cus%d/op%u/dt%u/L%u/n%llu", c->cus, op, (unsigned)dt,
               L, (unsigned long long)n);
      uint32_t tpb = 0, grid = 0;
      float ms = 0;
      const bool wave_ok = wave_fits(c, op, dt);
      if (cache_lookup(cache_path, keyb, tpb, grid) &&
          (tpb_fits(c, dt == GZ_F64, false, tpb) || (tpb == WAVE_TPB && wave_ok))) {
        r = time_op(c, op, d_sample, y, s, cap, nb, n, dt, L, tpb, grid, st, e0, e1, ms);
      } else {
        float bms = 1e30f;
        if (wave_ok) {  // the per-wave kernel (its grid is its own)
          r = time_op(c, op, d_sample, y, s, cap, nb, n, dt, L, WAVE_TPB, (uint32_t)c->cus, st,
                      e0, e1, bms);
          tpb = WAVE_TPB;
          grid = (uint32_t)c->cus;
        }
        const uint32_t tpbs[4] = {128, 256, 512, 1024};
        for (uint32_t ti = 0; r == GZ_OK && ti < 4; ++ti) {
          if (!tpb_fits(c, dt == GZ_F64, false, tpbs[ti])) continue;
          const int occ = gzk::occupancy_blocks(op, dt, log2_of(L), tpbs[ti]);
          const uint32_t grids[4] = {(uint32_t)c->cus, 2u * c->cus, (uint32_t)(c->cus * occ),
                                     (uint32_t)(c->cus * occ * 2)};
          for (uint32_t gi = 0; r == GZ_OK && gi < 4; ++gi) {
            float t = 0;
            r = time_op(c, op, d_sample, y, s, cap, nb, n, dt, L, tpbs[ti], grids[gi], st, e0,
                        e1, t);
            if (r == GZ_OK && t < bms) {
              bms = t;
              tpb = tpbs[ti];
              grid = grids[gi];
            }
          }
        }
        ms = bms;
        if (r == GZ_OK) cache_store(cache_path, keyb, tpb, grid, ms);
      }
      if (r == GZ_OK) {
        c->tuned[op][dt][log2_of(L) - 5].tpb = tpb;
        c->tuned[op][dt][log2_of(L) - 5].grid = grid;
        total += ms;
      }
    }
    if (r == GZ_OK && total < best_total) {
      best_total = total;
      best_L = L;
    }
  }
  if (r == GZ_OK && hipStreamSynchronize(st) != hipSuccess) r = GZ_EHIP;
  if (r == GZ_OK && block_len == 0) c->best_L[dt] = best_L;  // for requests of length 0
  if (r == GZ_OK && best) {
    const Tuned& t = c->tuned[0][dt][log2_of(best_L) - 5];
    *best = gz_params{best_L, t.tpb, t.grid, 0, 0, 0};
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  return r;
}

gz_status gz_tune_batch(gz_ctx* c, gz_op op, const gz_request* h_reqs, uint32_t nreq,
                        const char* cache_path, gz_params* best, gz_stream_t stream) {
  if (!c || !h_reqs || nreq == 0 || op > GZ_OP_FUSED) return GZ_EINVAL;
  bool wide = false;
  uint64_t elems = 0;
  for (uint32_t j = 0; j < nreq; ++j) {
    wide = wide || h_reqs[j].dtype == GZ_F64;
    elems += h_reqs[j].n;
  }
  char keyb[160];
  snprintf(keyb, sizeof keyb, "gfx950/cus%d/batch/op%u/wide%u/nreq%u/elems%llu", c->cus,
           (unsigned)op, wide ? 1u : 0u, nreq, (unsigned long long)elems);
  uint32_t tpb = 0, grid = 0;
  gz_status r = GZ_OK;
  // the per-wave kernels are a candidate where the batch qualifies
  bool wave_ok = false;
  {
    std::vector<Job> jobs;
    std::vector<uint32_t> map;
    r = build_requests(c, op, h_reqs, nreq, gzk::MAX_TPB_WIDE, jobs, map);
    if (r != GZ_OK) return r;
    if (op == GZ_OP_DECOMPRESS) {
      std::vector<uint32_t> smap;
      wave_ok = batch_decode_wave_ok(c, op, jobs, wide, wave_decode_map(jobs, smap));
    } else if (!wide) {
      wave_ok = batch_wave_ok(c, op, jobs);
    }
  }
  if (!(cache_lookup(cache_path, keyb, tpb, grid) &&
        (tpb_fits(c, wide, false, tpb) || (tpb == WAVE_TPB && wave_ok)))) {
    hipStream_t st = (hipStream_t)stream;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) r = GZ_EHIP;
    float bms = 1e30f;
    const uint32_t tpbs[5] = {WAVE_TPB, 128, 256, 512, 1024};
    for (uint32_t ti = 0; r == GZ_OK && ti < 5; ++ti) {
      const bool wv = tpbs[ti] == WAVE_TPB;
      if (wv ? !wave_ok : !tpb_fits(c, wide, false, tpbs[ti])) continue;
      const int occ =
          wv ? 1 : gzk::occupancy_blocks(gzk::OCC_BATCH + (uint32_t)op, wide, 5, tpbs[ti]);
      const uint32_t grids[4] = {(uint32_t)c->cus, 2u * c->cus, (uint32_t)(c->cus * occ),
                                 (uint32_t)(c->cus * occ * 2)};
      for (uint32_t gi = 0; r == GZ_OK && gi < (wv ? 1u : 4u); ++gi) {
        const gz_params p = {0, tpbs[ti], grids[gi], 0, 0, 0};
        r = gz_batch(c, op, h_reqs, nreq, &p, st);  // warm-up
        if (r == GZ_OK && hipEventRecord(e0, st) != hipSuccess) r = GZ_EHIP;
        for (int k = 0; k < 3 && r == GZ_OK; ++k) r = gz_batch(c, op, h_reqs, nreq, &p, st);
        float ms = 0;
        if (r == GZ_OK && (hipEventRecord(e1, st) != hipSuccess ||
                           hipEventSynchronize(e1) != hipSuccess ||
                           hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
          r = GZ_EHIP;
        if (r == GZ_OK && ms < bms) {
          bms = ms;
          tpb = tpbs[ti];
          grid = grids[gi];
        }
      }
    }
    if (r == GZ_OK && hipStreamSynchronize(st) != hipSuccess) r = GZ_EHIP;
    if (r == GZ_OK) cache_store(cache_path, keyb, tpb, grid, bms / 3);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
  }
  if (r != GZ_OK) return r;
  c->batch_tuned[op][wide ? 1 : 0] = Tuned{tpb, grid};
  if (best) *best = gz_params{0, tpb, grid, 0, 0, 0};
  return GZ_OK;
}

gz_status gz_selector_load(gz_ctx* c, const void* h_blob, uint64_t bytes) {
  if (!c || !h_blob || bytes != 756) return GZ_EINVAL;
  const uint8_t* b = (const uint8_t*)h_blob;
  uint32_t magic, shift;
  memcpy(&magic, b, 4);
  memcpy(&shift, b + 4, 4);
  if (magic != 0x314D5A47u || shift > 24) return GZ_EINVAL;
  for (int k = 0; k < 35; ++k) {  // b1[32] at 520, b2[3] at 744
    int32_t v;
    memcpy(&v, b + (k < 32 ? 520 + 4 * k : 744 + 4 * (k - 32)), 4);
    if (v <= -(1 << 24) || v >= (1 << 24)) return GZ_EINVAL;
  }
  if (hipMemcpy(c->blob, h_blob, bytes, hipMemcpyHostToDevice) != hipSuccess) return GZ_EHIP;
  c->blob_loaded = true;
  return GZ_OK;
}

gz_status gz_tile_trial(gz_ctx* c, const float* d_in, uint64_t n, uint32_t nx, double eb,
                        int8_t* d_feat, uint32_t* d_sizes, uint8_t* d_label, gz_stream_t stream) {
  if (!c || nx == 0 || nx % 8 != 0 || n % (8ull * nx) != 0) return GZ_EINVAL;
  if (n && (!d_in || !d_feat || !d_sizes || !d_label)) return GZ_EINVAL;
  Job J;
  memset(&J, 0, sizeof J);
  J.dtype = GZ_F32;
  if (!set_bound(J, GZ_F32, eb)) return GZ_EINVAL;
  if (!n) return GZ_OK;
  J.in = job_ptr(d_in);
  J.n = n;
  J.B = n / 64;
  J.nx = nx;
  J.mode = 1;
  return hip_status(gzk::launch_tile_trial(J, d_feat, d_sizes, d_label, (hipStream_t)stream));
}

gz_status gz_mlp_grad(gz_ctx* c, const float* d_w, const int8_t* d_feat, const uint8_t* d_label,
                      uint64_t nsamp, float* d_grad, float* d_loss, gz_stream_t stream) {
  if (!c || !d_w || !d_grad || !d_loss || nsamp > gzs::MLP_MAX_BATCH) return GZ_EINVAL;
  if (nsamp && (!d_feat || !d_label)) return GZ_EINVAL;
  return hip_status(gzs::launch_mlp_grad(d_w, d_feat, d_label, (uint32_t)nsamp, c->train_ws,
                                         d_grad, d_loss, (hipStream_t)stream));
}

gz_status gz_mlp_adam(gz_ctx* c, float* d_w, const float* d_grad, float* d_m, float* d_v,
                      uint32_t step, float lr, gz_stream_t stream) {
  if (!c || !d_w || !d_grad || !d_m || !d_v || step == 0 || !(lr > 0.0f)) return GZ_EINVAL;
  const float bc1 = (float)(1.0 - pow(0.9, (double)step));
  const float bc2 = (float)(1.0 - pow(0.999, (double)step));
  return hip_status(gzs::launch_mlp_adam(d_w, d_grad, d_m, d_v, lr, bc1, bc2,
                                         (hipStream_t)stream));
}

}  // extern "C"

// ---- compression without allocation, for callers that cannot allocate
// device memory (code under HIP graph capture, serving loops).  Its
// workspace is the file-scope device array `scratch`: the control block,
// 1 KiB of selector weights (zero: the MLP selector is not available here)
// and one look-back word per strip.  Each device holds its own copy until
// the process ends.  The last workgroup of every launch leaves the ticket
// counters at zero and the look-back words are tagged with a launch epoch,
// so nothing needs clearing between calls; the finishing kernel reports and
// clears the sticky error word.  Calls that overlap on one device race on
// the array.
namespace {

constexpr uint64_t NA_MAX_STRIPS = 32768;
constexpr size_t NA_CTRL = 0, NA_BLOB = sizeof(Ctrl), NA_STATUS = NA_BLOB + 1024;
constexpr size_t NA_BYTES = NA_STATUS + NA_MAX_STRIPS * 8;
constexpr int NA_MAX_DEV = 64;

struct NoAllocDev {
  std::once_flag once;
  gz_status setup = GZ_EHIP;
  gz_ctx ctx;  // host description of the device-resident workspace
};
NoAllocDev g_noalloc[NA_MAX_DEV];

}  // namespace

static __device__ __align__(256) unsigned char scratch[NA_BYTES];

namespace {

// Once per device, with that device current: the array's device address
// (host code never uses the symbol itself as an address) and the launch
// limits of the device.
gz_status noalloc_setup(int device, gz_ctx& c) {
  void* ptr = nullptr;
  if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return GZ_EHIP;
  c.device = device;
  if (hipDeviceGetAttribute(&c.cus, hipDeviceAttributeMultiprocessorCount, device) !=
      hipSuccess)
    return GZ_EHIP;
  int wclk_khz = 0;
  if (hipDeviceGetAttribute(&wclk_khz, hipDeviceAttributeWallClockRate, device) != hipSuccess ||
      wclk_khz <= 0)
    wclk_khz = 100000;
  c.wait_ticks = (uint64_t)wclk_khz * 1000ull;
  int lds = 0;
  if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device) !=
          hipSuccess ||
      lds <= 0)
    lds = 65536;
  c.lds_max = (size_t)lds;
  uint8_t* base = (uint8_t*)ptr;
  c.ctrl = (Ctrl*)(base + NA_CTRL);
  c.blob = base + NA_BLOB;
  c.blob_loaded = false;
  c.status = (unsigned long long*)(base + NA_STATUS);
  c.jobbase = nullptr;  // single streams only (no packed chains)
  c.max_strips = NA_MAX_STRIPS;
  c.max_elems = 0;
  c.max_jobs = 0;
  return GZ_OK;
}

}  // namespace

extern "C" {

gz_status gz_compress_noalloc(const void* d_in, uint64_t n, gz_dtype dtype, double eb,
                              const gz_params* p, void* d_out, uint64_t out_cap,
                              uint64_t* d_out_bytes, uint32_t* d_status, gz_stream_t stream) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return GZ_EHIP;
  if (dev < 0 || dev >= NA_MAX_DEV) return GZ_EUNSUPPORTED;
  NoAllocDev& d = g_noalloc[dev];
  std::call_once(d.once, [&] { d.setup = noalloc_setup(dev, d.ctx); });
  if (d.setup != GZ_OK) return d.setup;
  gz_status r = compress_impl(&d.ctx, d_in, n, dtype, eb, p, d_out, out_cap, d_out_bytes, stream);
  if (r != GZ_OK) return r;
  return hip_status(gzk::launch_finish(d.ctx.ctl(), d_status, (hipStream_t)stream));
}

}  // extern "C"
