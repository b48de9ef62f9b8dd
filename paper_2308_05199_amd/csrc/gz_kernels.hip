// gz_kernels.hip -- gfx950 kernels of the GZ1 codec.
//
// Layout of the work: a lane owns a 32-element segment (L/32 consecutive
// lanes own one block), a workgroup of TPB lanes owns a strip of TPB*32
// elements (a whole number of 4096-element superblocks).  Workgroups are
// persistent: they take strips in ticket order, so every strip a strip waits
// for is already running.  Strip payload offsets come from one decoupled
// look-back pass over agent-scope status words (a single read of the input,
// a single write of the output), tagged with a launch epoch so they never
// need clearing.  No MFMA: the path is bound by HBM, not by arithmetic.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "gz_common.h"
#include "gz_kernels.h"

namespace gzk {

// ------------------------------------------------------------------ utils
typedef float f4u __attribute__((ext_vector_type(4), aligned(4)));
typedef double d2u __attribute__((ext_vector_type(2), aligned(8)));
typedef uint32_t u4u __attribute__((ext_vector_type(4), aligned(4)));

constexpr uint32_t SPIN_LIMIT = 1u << 22;
constexpr uint64_t VMASK = (1ull << 34) - 1;

__device__ __forceinline__ void st_agent(unsigned long long* p, unsigned long long v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned long long ld_agent(const unsigned long long* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t ld_agent32(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t sw_pack(uint64_t flag, uint32_t ep, uint64_t v) {
  return (flag << 62) | ((uint64_t)(ep & 0x0FFFFFFFu) << 34) | (v & VMASK);
}

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
  const int lane = __lane_id();
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    uint32_t t = __shfl_up(v, o);
    if (lane >= o) v += t;
  }
  return v;
}

__device__ __forceinline__ unsigned long long wave_sum64(unsigned long long v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// OR / carry over the LPB lanes that own one block.
template <int LPB>
__device__ __forceinline__ uint32_t grp_or(uint32_t v) {
  if (LPB >= 2) v |= __shfl_xor(v, 1);
  if (LPB >= 4) v |= __shfl_xor(v, 2);
  return v;
}

template <int LPB>
__device__ __forceinline__ uint32_t grp_excl_sum(uint32_t v, uint32_t w) {
  uint32_t incl = v;
  if (LPB >= 2) {
    uint32_t t = __shfl_up(incl, 1);
    if (w >= 1) incl += t;
  }
  if (LPB >= 4) {
    uint32_t t = __shfl_up(incl, 2);
    if (w >= 2) incl += t;
  }
  return incl - v;
}

// ----------------------------------------------------------- quantisation
// fp32: r = x/t is formed as fl32((double)x * (1/(double)t)).  The double
// product is within 2^-52 (relative) of x/t, while x/t never lies within
// 2^-49 of a float rounding boundary in the normal range (x, t have 24-bit
// significands and a boundary needs 25), so the rounding to float equals
// the IEEE quotient; below the normal range both give q = 0.  x - xh is
// exact (Sterbenz), so |x - xh| <= eb is tested in float against the largest
// float not above eb.
__device__ __forceinline__ int32_t quant(float x, double rinv, float t, float eblo,
                                         bool& bad) {
  float r = (float)((double)x * rinv);
  bool inr = fabsf(r) < 536870912.0f;  // false for NaN
  float rr = inr ? __builtin_rintf(r) : 0.0f;
  int32_t q = (int32_t)rr;
  float xh = (float)q * t;
  float d = x - xh;
  bad = !inr || !(fabsf(d) <= eblo);
  return q;
}

__device__ __forceinline__ int32_t quant(double x, double t, double eb, bool& bad) {
  double r = x / t;
  bool inr = fabs(r) <= 536870911.0;
  double rr = inr ? __builtin_rint(r) : 0.0;
  int32_t q = (int32_t)rr;
  double xh = (double)q * t;
  double d = x - xh;
  bad = !inr || !(fabs(d) <= eb);
  return q;
}

template <typename T>
__device__ __forceinline__ int32_t quant_t(T x, const Job& J, bool& bad);
template <>
__device__ __forceinline__ int32_t quant_t<float>(float x, const Job& J, bool& bad) {
  return quant(x, J.rinv, J.t32, J.eblo, bad);
}
template <>
__device__ __forceinline__ int32_t quant_t<double>(double x, const Job& J, bool& bad) {
  return quant(x, J.t64, J.eb, bad);
}

// ------------------------------------------------------------ load/store
template <typename T>
__device__ __forceinline__ void load_seg(const T* __restrict__ p, uint32_t vcnt, T (&v)[32]);
template <>
__device__ __forceinline__ void load_seg<float>(const float* __restrict__ p, uint32_t vcnt,
                                                float (&v)[32]) {
  if (vcnt == 32) {
#pragma unroll
    for (int k = 0; k < 32; k += 4) {
      f4u t = *(const f4u*)(p + k);
      v[k] = t.x; v[k + 1] = t.y; v[k + 2] = t.z; v[k + 3] = t.w;
    }
  } else {
#pragma unroll
    for (int k = 0; k < 32; ++k) v[k] = (k < (int)vcnt) ? p[k] : 0.0f;
  }
}
template <>
__device__ __forceinline__ void load_seg<double>(const double* __restrict__ p, uint32_t vcnt,
                                                 double (&v)[32]) {
  if (vcnt == 32) {
#pragma unroll
    for (int k = 0; k < 32; k += 2) {
      d2u t = *(const d2u*)(p + k);
      v[k] = t.x; v[k + 1] = t.y;
    }
  } else {
#pragma unroll
    for (int k = 0; k < 32; ++k) v[k] = (k < (int)vcnt) ? p[k] : 0.0;
  }
}

template <typename T>
__device__ __forceinline__ void store_seg(T* __restrict__ p, uint32_t vcnt, const T (&v)[32]);
template <>
__device__ __forceinline__ void store_seg<float>(float* __restrict__ p, uint32_t vcnt,
                                                 const float (&v)[32]) {
  if (vcnt == 32) {
#pragma unroll
    for (int k = 0; k < 32; k += 4) {
      f4u t;
      t.x = v[k]; t.y = v[k + 1]; t.z = v[k + 2]; t.w = v[k + 3];
      *(f4u*)(p + k) = t;
    }
  } else {
#pragma unroll
    for (int k = 0; k < 32; ++k)
      if (k < (int)vcnt) p[k] = v[k];
  }
}
template <>
__device__ __forceinline__ void store_seg<double>(double* __restrict__ p, uint32_t vcnt,
                                                  const double (&v)[32]) {
  if (vcnt == 32) {
#pragma unroll
    for (int k = 0; k < 32; k += 2) {
      d2u t;
      t.x = v[k]; t.y = v[k + 1];
      *(d2u*)(p + k) = t;
    }
  } else {
#pragma unroll
    for (int k = 0; k < 32; ++k)
      if (k < (int)vcnt) p[k] = v[k];
  }
}

// bits of element i as u32 words (1 for float, 2 for double)
__device__ __forceinline__ void raw_words(float v, uint32_t* dst) {
  dst[0] = __float_as_uint(v);
}
__device__ __forceinline__ void raw_words(double v, uint32_t* dst) {
  unsigned long long b = (unsigned long long)__double_as_longlong(v);
  dst[0] = (uint32_t)b;
  dst[1] = (uint32_t)(b >> 32);
}
__device__ __forceinline__ float from_raw(const uint32_t* src, float) {
  return __uint_as_float(src[0]);
}
__device__ __forceinline__ double from_raw(const uint32_t* src, double) {
  unsigned long long b = (unsigned long long)src[0] | ((unsigned long long)src[1] << 32);
  return __longlong_as_double((long long)b);
}

// ------------------------------------------------------------- LDS state
struct Smem {
  uint32_t ticket;
  uint32_t epoch;
  uint32_t flag;                 // strip error flags
  uint32_t hdr_ok;
  uint32_t wtot[MAX_TPB / 64];
  unsigned long long excl;       // strip exclusive prefix (dwords, chain-wide)
  unsigned long long pj;         // chain prefix at the job's first strip
  unsigned long long paydw;      // decode: payload size of the incoming stream (dwords)
  float t32;                     // decode: step of the incoming stream
  double t64;
  uint32_t hb[MAX_TPB / 4];      // header bytes of the strip's blocks
};

__device__ __forceinline__ void prologue(const Ctl& C, Smem& sm) {
  if (threadIdx.x == 0) sm.epoch = ld_agent32(&C.ctrl->epoch);
  __syncthreads();
}

__device__ __forceinline__ uint32_t next_ticket(const Ctl& C, Smem& sm) {
  __syncthreads();  // everyone is done with the previous strip's LDS
  if (threadIdx.x == 0) sm.ticket = atomicAdd(&C.ctrl->ticket, 1u);
  __syncthreads();
  return sm.ticket;
}

__device__ __forceinline__ void epilogue(const Ctl& C) {
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t d = atomicAdd(&C.ctrl->done, 1u);
    if (d == gridDim.x - 1) {  // last workgroup: reset for the next launch
      atomicExch(&C.ctrl->ticket, 0u);
      atomicExch(&C.ctrl->done, 0u);
      atomicAdd(&C.ctrl->epoch, 1u);
    }
  }
}

__device__ __forceinline__ bool aborted(const Ctl& C) {
  return (ld_agent32(&C.ctrl->err) & ERRF_TIMEOUT) != 0;
}

// Decoupled look-back run by wave 0: publishes the strip aggregate, returns
// the exclusive prefix (dwords) of strip gs within its chain.
__device__ uint64_t lookback(const Ctl& C, uint64_t gs, uint64_t chain0, uint32_t ep,
                             uint64_t agg, bool& timeout) {
  const int lane = __lane_id();
  unsigned long long* status = C.status;
  if (gs == chain0) {
    if (lane == 0) st_agent(status + gs, sw_pack(2, ep, agg));
    return 0;
  }
  if (lane == 0) st_agent(status + gs, sw_pack(1, ep, agg));
  uint64_t excl = 0;
  int64_t top = (int64_t)gs - 1;
  uint32_t spins = 0;
  for (;;) {
    int64_t idx = top - lane;
    uint32_t flag;
    uint64_t val;
    if (idx >= (int64_t)chain0) {
      uint64_t w = ld_agent(status + idx);
      bool cur = (uint32_t)((w >> 34) & 0x0FFFFFFFu) == (ep & 0x0FFFFFFFu);
      flag = cur ? (uint32_t)(w >> 62) : 0u;
      val = w & VMASK;
    } else {
      flag = 2;
      val = 0;
    }
    uint64_t pm = __ballot(flag == 2);
    uint64_t zm = __ballot(flag == 0);
    int p = pm ? (int)__builtin_ctzll(pm) : 64;
    uint64_t upto = p >= 63 ? ~0ull : ((2ull << p) - 1);
    if (zm & upto) {
      ++spins;
      if (spins > SPIN_LIMIT || ((spins & 255u) == 0 && aborted(C))) {
        timeout = true;
        break;
      }
      __builtin_amdgcn_s_sleep(2);
      continue;
    }
    excl += wave_sum64(lane <= p ? val : 0ull);
    if (p < 64) break;
    top -= 64;
  }
  if (lane == 0) st_agent(status + gs, sw_pack(2, ep, timeout ? 0 : excl + agg));
  return excl;
}

// Chain prefix at the first strip of job j (packed Scatter output).
__device__ uint64_t job_base_wait(const Ctl& C, uint32_t j, uint32_t ep, bool& timeout) {
  uint32_t spins = 0;
  for (;;) {
    uint64_t w = ld_agent(C.jobbase + j);
    if ((uint32_t)((w >> 34) & 0x0FFFFFFFu) == (ep & 0x0FFFFFFFu) && (w >> 62) == 2)
      return w & VMASK;
    ++spins;
    if (spins > SPIN_LIMIT || ((spins & 255u) == 0 && aborted(C))) {
      timeout = true;
      return 0;
    }
    __builtin_amdgcn_s_sleep(2);
  }
}

// Strip-level exclusive scan of per-lane sizes; returns the lane's exclusive
// prefix and the strip total.
__device__ __forceinline__ uint32_t strip_scan(uint32_t contrib, Smem& sm, uint32_t& total) {
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int nw = blockDim.x >> 6;
  uint32_t incl = wave_incl_scan(contrib);
  if (lane == 63) sm.wtot[wid] = incl;
  __syncthreads();
  uint32_t pre = 0, tot = 0;
  for (int k = 0; k < nw; ++k) {
    uint32_t t = sm.wtot[k];
    pre += (k < wid) ? t : 0u;
    tot += t;
  }
  total = tot;
  return pre + incl - contrib;
}

// Magnitude plane j of a segment: bit i = bit j of a[i].
__device__ __forceinline__ uint32_t plane_of(const uint32_t (&a)[32], uint32_t j) {
  uint32_t p = 0;
#pragma unroll
  for (int i = 0; i < 32; ++i) p |= ((a[i] >> j) & 1u) << i;
  return p;
}

// --------------------------------------------------------------- encode
// Encodes the strip whose lane values are v[0..vcnt) (mode 0), publishes
// its look-back word and writes its part of the stream.
template <typename T, int L>
__device__ void encode_strip(const Job& J, uint64_t s, uint64_t gs, const Ctl& C, Smem& sm,
                             const T (&v)[32], uint32_t vcnt, bool skip) {
  constexpr int LPB = L / 32;
  constexpr uint32_t ES = sizeof(T);
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const uint32_t TPB = blockDim.x;
  const uint64_t seg = s * TPB + tid;
  const uint32_t w = tid & (LPB - 1);
  const uint64_t b = seg / LPB;

  // quantise
  int32_t q[32];
  bool bad = false, nz = false;
#pragma unroll
  for (int i = 0; i < 32; ++i) {
    bool bi = false;
    int32_t qi = quant_t<T>(v[i], J, bi);
    bool valid = i < (int)vcnt;
    q[i] = valid ? qi : 0;
    bad |= valid && bi;
    nz |= valid && qi != 0;
  }
  // residuals against the previous element (previous lane for i == 0)
  int32_t prev = __shfl_up(q[31], 1);
  uint32_t a[32];
  uint32_t sg = 0, orv = 0;
#pragma unroll
  for (int i = 31; i >= 0; --i) {
    int32_t pq = i ? q[i - 1] : prev;
    int32_t d = (i < (int)vcnt) ? (int32_t)((uint32_t)q[i] - (uint32_t)pq) : 0;
    if (i == 0 && w == 0) d = 0;
    uint32_t ad = (uint32_t)(d < 0 ? -d : d);
    a[i] = ad;
    orv |= ad;
    sg |= (uint32_t)(d < 0) << i;
  }
  orv = grp_or<LPB>(orv);
  uint32_t badb = grp_or<LPB>((uint32_t)bad);
  uint32_t nzb = grp_or<LPB>((uint32_t)nz);

  const uint64_t bstart = b * (uint64_t)L;
  const bool exists = b < J.B;
  const uint32_t m = exists ? (uint32_t)min((uint64_t)L, J.n - bstart) : 0u;
  uint32_t F = orv ? 32u - (uint32_t)__clz(orv) : 0u;
  uint32_t kind, size_dw;
  const uint32_t raw_dw = m * (ES / 4);
  if (!exists) {
    kind = K_ZERO; size_dw = 0; F = 0;
  } else if (badb) {
    kind = K_RAW; size_dw = raw_dw; F = 0;
  } else if (!nzb) {
    kind = K_ZERO; size_dw = 0; F = 0;
  } else {
    kind = K_L1D;
    size_dw = 1u + (F ? (F + 1u) * LPB : 0u);
    if (size_dw > raw_dw) { kind = K_RAW; size_dw = raw_dw; F = 0; }
  }
  const uint32_t hbyte = (kind << 5) | F;

  uint32_t total;
  uint32_t excl_lane = strip_scan(w == 0 ? size_dw : 0u, sm, total);
  const uint32_t boff = (w == 0) ? excl_lane : excl_lane - size_dw;

  if (wid == 0) {
    bool to = false;
    uint64_t ex = lookback(C, gs, J.chain0, sm.epoch, total, to);
    uint64_t pj = 0;
    if (J.chain0 != J.strip0) {
      if (s == 0) {
        if (lane == 0 && !to) st_agent(C.jobbase + J.job, sw_pack(2, sm.epoch, ex));
        pj = ex;
      } else if (!to) {
        pj = job_base_wait(C, J.job, sm.epoch, to);
      }
    }
    if (lane == 0) {
      sm.excl = ex;
      sm.pj = pj;
      sm.flag = to ? ERRF_TIMEOUT : 0u;
      if (to) atomicOr(&C.ctrl->err, ERRF_TIMEOUT);
    }
  }
  // header bytes of this strip's blocks
  if (w == 0) ((uint8_t*)sm.hb)[tid / LPB] = (uint8_t)(exists ? hbyte : 0u);
  __syncthreads();
  if (sm.flag || skip) return;

  const uint64_t pj = sm.pj;
  const uint64_t erel = sm.excl - pj;  // strip offset inside this job's payload
  uint8_t* base8 = (uint8_t*)J.out + J.fixed_off + 4 * pj;
  uint32_t* pay = (uint32_t*)(base8 + J.pay_off) + erel + boff;

  if (exists && (seg & (SUPER / SEG - 1)) == 0)
    ((uint32_t*)(base8 + HDR))[seg / (SUPER / SEG)] = (uint32_t)(erel + boff);

  if (exists) {
    if (kind == K_L1D) {
      if (w == 0) pay[0] = (uint32_t)q[0];
      if (F) {
        pay[1 + w] = sg;
        for (uint32_t j = 0; j < F; ++j) pay[1 + (j + 1) * LPB + w] = plane_of(a, j);
      }
    } else if (kind == K_RAW) {
#pragma unroll
      for (int i = 0; i < 32; ++i) {
        if (i < (int)vcnt) {
          uint32_t wd[2];
          raw_words(v[i], wd);
          pay[(w * 32 + i) * (ES / 4)] = wd[0];
          if (ES == 8) pay[(w * 32 + i) * (ES / 4) + 1] = wd[1];
        }
      }
    }
  }
  // header bytes as whole words (the strip starts on a 4-block boundary)
  const uint32_t nblk = TPB / LPB;
  const uint64_t blk0 = s * (uint64_t)nblk;
  for (uint32_t i = tid; i < nblk / 4; i += TPB) {
    if (blk0 + 4 * i < J.B) *(uint32_t*)(base8 + J.hdr_off + blk0 + 4 * i) = sm.hb[i];
  }
  // the last strip completes the header and the size outputs
  if (s == J.nstrips - 1 && tid < 16) {
    const uint64_t payload = 4 * (sm.excl + total - pj);
    unsigned long long ebits = (unsigned long long)__double_as_longlong(J.eb);
    uint32_t wv = 0;
    switch (tid) {
      case 0: wv = 0x31435A47u; break;
      case 1: wv = 1u | (J.dtype << 16) | (J.log2L << 24); break;
      case 2: wv = (uint32_t)J.n; break;
      case 3: wv = (uint32_t)(J.n >> 32); break;
      case 4: wv = (uint32_t)ebits; break;
      case 5: wv = (uint32_t)(ebits >> 32); break;
      case 6: wv = (uint32_t)payload; break;
      case 7: wv = (uint32_t)(payload >> 32); break;
      case 8: wv = J.mode; break;
      case 9: wv = J.nx; break;
      case 10: wv = SUPER; break;
      default: wv = 0; break;
    }
    ((uint32_t*)base8)[tid] = wv;
    if (tid == 0) {
      if (J.out_bytes) *J.out_bytes = J.pay_off + payload;
      if (J.chunk_off) *J.chunk_off = J.fixed_off + 4 * pj;
    }
  }
}

// --------------------------------------------------------------- decode
// Checks the stream header against the job; sets sm.hdr_ok, sm.paydw, sm.t*.
__device__ void check_header(const Job& J, const uint8_t* in, uint64_t in_bytes, Smem& sm) {
  const int tid = threadIdx.x;
  if (tid < 64) {
    const bool readable = in_bytes >= HDR;
    uint32_t wv = (tid < 16 && readable) ? ((const uint32_t*)in)[tid] : 0u;
    uint32_t expect = 0;
    bool ok = true;
    switch (tid) {
      case 0: ok = wv == 0x31435A47u; break;
      case 1: ok = wv == (1u | (J.dtype << 16) | (J.log2L << 24)); break;
      case 2: ok = wv == (uint32_t)J.n; break;
      case 3: ok = wv == (uint32_t)(J.n >> 32); break;
      case 8: ok = wv == J.mode; break;
      case 9: ok = wv == J.nx; break;
      case 10: ok = wv == SUPER; break;
      case 4: case 5: case 6: case 7: ok = true; break;
      default: ok = wv == expect; break;
    }
    uint64_t okm = __ballot(ok);
    const uint32_t e0 = __shfl(wv, 4), e1 = __shfl(wv, 5);
    const uint32_t p0 = __shfl(wv, 6), p1 = __shfl(wv, 7);
    if (tid == 0) {
      double eb = __longlong_as_double((long long)(((uint64_t)e1 << 32) | e0));
      uint64_t payload = ((uint64_t)p1 << 32) | p0;
      bool good = readable && okm == ~0ull;
      good = good && (eb > 0.0) && isfinite(eb);
      float t32 = (float)(2.0 * eb);
      double t64 = 2.0 * eb;
      if (J.dtype == 0) good = good && isfinite(t32) && t32 != 0.0f;
      else good = good && isfinite(t64) && t64 != 0.0;
      good = good && (payload % 4 == 0) && payload <= in_bytes &&
             J.pay_off <= in_bytes - payload;
      sm.hdr_ok = good ? 1u : 0u;
      sm.t32 = t32;
      sm.t64 = t64;
      sm.paydw = payload / 4;
    }
  }
  __syncthreads();
}

template <typename T>
__device__ __forceinline__ T step_of(const Smem& sm);
template <>
__device__ __forceinline__ float step_of<float>(const Smem& sm) { return sm.t32; }
template <>
__device__ __forceinline__ double step_of<double>(const Smem& sm) { return sm.t64; }

// Decodes the lane's segment of strip s of the stream at `in` into v[];
// returns false (and flags the context) if the strip is malformed.
template <typename T, int L>
__device__ bool decode_strip(const Job& J, const uint8_t* in, uint64_t in_bytes, uint64_t s,
                             const Ctl& C, Smem& sm, T (&v)[32], uint32_t& vcnt) {
  constexpr int LPB = L / 32;
  constexpr uint32_t ES = sizeof(T);
  const int tid = threadIdx.x;
  const uint32_t TPB = blockDim.x;
  const uint64_t seg = s * TPB + tid;
  const uint32_t w = tid & (LPB - 1);
  const uint64_t b = seg / LPB;
  const uint64_t e0 = seg * SEG;
  vcnt = e0 >= J.n ? 0u : (uint32_t)min((uint64_t)SEG, J.n - e0);

  check_header(J, in, in_bytes, sm);
  const uint64_t pay_dw = sm.paydw;
  bool ok = sm.hdr_ok != 0;
  __syncthreads();

  const bool exists = b < J.B;
  const uint32_t m = exists ? (uint32_t)min((uint64_t)L, J.n - b * (uint64_t)L) : 0u;
  uint32_t hb = (ok && exists) ? (uint32_t)in[J.hdr_off + b] : 0u;
  uint32_t kind = hb >> 5, F = hb & 31u;
  uint32_t size_dw = 0;
  bool hv = true;
  if (kind == K_ZERO) hv = F == 0;
  else if (kind == K_RAW) { hv = F == 0; size_dw = m * (ES / 4); }
  else if (kind == K_L1D) size_dw = 1u + (F ? (F + 1u) * LPB : 0u);
  else hv = false;
  if (!hv) size_dw = 0;

  uint32_t total;
  uint32_t excl_lane = strip_scan(w == 0 ? size_dw : 0u, sm, total);
  const uint32_t boff = (w == 0) ? excl_lane : excl_lane - size_dw;
  const uint32_t* table = (const uint32_t*)(in + HDR);
  const uint64_t sb0 = s * (uint64_t)(TPB * SEG / SUPER);
  const uint64_t E = (ok && sb0 < J.NS) ? table[sb0] : 0u;
  bool good = hv;
  if (ok && exists && (seg & (SUPER / SEG - 1)) == 0)
    good = good && (uint64_t)table[seg / (SUPER / SEG)] == E + boff;
  if (ok && tid == 0) {
    const uint64_t sbn = sb0 + TPB * SEG / SUPER;
    const uint64_t end = E + total;
    good = good && end <= pay_dw && (sbn < J.NS ? (uint64_t)table[sbn] == end : end == pay_dw);
    if (s == 0) good = good && E == 0;
  }
  if (ok && s == J.nstrips - 1 && tid < 4) {
    const uint64_t pb = J.B + tid;
    if (pb < ((J.B + 3) & ~3ull)) good = good && in[J.hdr_off + pb] == 0;
  }
  good = __syncthreads_and(good ? 1 : 0) != 0;
  if (!ok || !good) {
    if (tid == 0) atomicOr(&C.ctrl->err, ERRF_CORRUPT);
#pragma unroll
    for (int i = 0; i < 32; ++i) v[i] = (T)0;
    return false;
  }

  const uint32_t* pay = (const uint32_t*)(in + J.pay_off) + E + boff;
  const T t = step_of<T>(sm);
  if (kind == K_RAW) {
#pragma unroll
    for (int i = 0; i < 32; ++i)
      v[i] = (i < (int)vcnt) ? from_raw(pay + (w * 32 + i) * (ES / 4), T()) : (T)0;
    return true;
  }
  if (kind == K_ZERO || !exists) {
#pragma unroll
    for (int i = 0; i < 32; ++i) v[i] = (T)0;
    return true;
  }
  // L1D
  const int32_t base = (int32_t)pay[0];
  uint32_t a[32];
#pragma unroll
  for (int i = 0; i < 32; ++i) a[i] = 0;
  uint32_t sg = 0;
  if (F) {
    sg = pay[1 + w];
    for (uint32_t j = 0; j < F; ++j) {
      uint32_t pw = pay[1 + (j + 1) * LPB + w];
#pragma unroll
      for (int i = 0; i < 32; ++i) a[i] |= ((pw >> i) & 1u) << j;
    }
  }
  uint32_t acc = 0;
#pragma unroll
  for (int i = 0; i < 32; ++i) {
    uint32_t neg = 0u - ((sg >> i) & 1u);
    uint32_t d = (a[i] ^ neg) - neg;
    if (i == 0 && w == 0) d = 0;
    acc += d;
    a[i] = acc;  // local prefix
  }
  const uint32_t carry = grp_excl_sum<LPB>(acc, w);
#pragma unroll
  for (int i = 0; i < 32; ++i) {
    int32_t qi = (int32_t)((uint32_t)base + carry + a[i]);
    v[i] = (T)qi * t;
  }
  return true;
}

// ---------------------------------------------------------------- kernels
template <typename T, int L>
__device__ __forceinline__ void compress_one(const Job& J, uint64_t s, uint64_t gs,
                                             const Ctl& C, Smem& sm) {
  const uint64_t seg = s * blockDim.x + threadIdx.x;
  const uint64_t e0 = seg * SEG;
  const uint32_t vcnt = e0 >= J.n ? 0u : (uint32_t)min((uint64_t)SEG, J.n - e0);
  T v[32];
  load_seg<T>((const T*)J.in + (vcnt ? e0 : 0), vcnt, v);
  encode_strip<T, L>(J, s, gs, C, sm, v, vcnt, false);
}

template <typename T, int L>
__device__ __forceinline__ void decompress_one(const Job& J, uint64_t s, const Ctl& C,
                                               Smem& sm) {
  const uint64_t off = J.in_off ? J.in_off[J.job] : 0ull;
  const uint8_t* in = (const uint8_t*)J.in + off;
  const uint64_t avail = off <= J.in_bytes ? J.in_bytes - off : 0ull;
  T v[32];
  uint32_t vcnt;
  if (decode_strip<T, L>(J, in, avail, s, C, sm, v, vcnt)) {
    const uint64_t e0 = (s * blockDim.x + threadIdx.x) * SEG;
    if (vcnt) store_seg<T>((T*)J.out + e0, vcnt, v);
  }
}

template <int L>
__device__ __forceinline__ void fused_one(const Job& J, uint64_t s, uint64_t gs,
                                          const Ctl& C, Smem& sm) {
  float v[32];
  uint32_t vcnt;
  bool ok = decode_strip<float, L>(J, (const uint8_t*)J.in, J.in_bytes, s, C, sm, v, vcnt);
  const uint64_t e0 = (s * blockDim.x + threadIdx.x) * SEG;
  float a[32];
  load_seg<float>(J.local + (vcnt ? e0 : 0), vcnt, a);
#pragma unroll
  for (int i = 0; i < 32; ++i) v[i] = v[i] + a[i];  // incoming + local, fp32
  encode_strip<float, L>(J, s, gs, C, sm, v, vcnt, !ok);
}

template <typename T, int L>
__global__ __launch_bounds__(MAX_TPB) void k_compress(Job J, Ctl C) {
  __shared__ Smem sm;
  prologue(C, sm);
  for (;;) {
    uint32_t t = next_ticket(C, sm);
    if (t >= J.nstrips) break;
    compress_one<T, L>(J, t, t, C, sm);
  }
  epilogue(C);
}

template <typename T, int L>
__global__ __launch_bounds__(MAX_TPB) void k_decompress(Job J, Ctl C) {
  __shared__ Smem sm;
  prologue(C, sm);
  for (;;) {
    uint32_t t = next_ticket(C, sm);
    if (t >= J.nstrips) break;
    decompress_one<T, L>(J, t, C, sm);
  }
  epilogue(C);
}

template <int L>
__global__ __launch_bounds__(MAX_TPB) void k_fused(Job J, Ctl C) {
  __shared__ Smem sm;
  prologue(C, sm);
  for (;;) {
    uint32_t t = next_ticket(C, sm);
    if (t >= J.nstrips) break;
    fused_one<L>(J, t, t, C, sm);
  }
  epilogue(C);
}

// Batched: strip_job maps a global strip to its job.
__global__ __launch_bounds__(MAX_TPB) void k_batch(const Job* __restrict__ jobs,
                                                  const uint32_t* __restrict__ strip_job,
                                                  uint32_t total, uint32_t op, Ctl C) {
  __shared__ Smem sm;
  prologue(C, sm);
  for (;;) {
    uint32_t t = next_ticket(C, sm);
    if (t >= total) break;
    const uint32_t j = strip_job[t];
    const Job J = jobs[j];
    const uint64_t s = t - J.strip0;
    const uint32_t key = (op << 4) | (J.dtype << 3) | J.log2L;
    switch (key) {
      case (0u << 4) | (0u << 3) | 5u: compress_one<float, 32>(J, s, t, C, sm); break;
      case (0u << 4) | (0u << 3) | 6u: compress_one<float, 64>(J, s, t, C, sm); break;
      case (0u << 4) | (0u << 3) | 7u: compress_one<float, 128>(J, s, t, C, sm); break;
      case (0u << 4) | (1u << 3) | 5u: compress_one<double, 32>(J, s, t, C, sm); break;
      case (0u << 4) | (1u << 3) | 6u: compress_one<double, 64>(J, s, t, C, sm); break;
      case (0u << 4) | (1u << 3) | 7u: compress_one<double, 128>(J, s, t, C, sm); break;
      case (1u << 4) | (0u << 3) | 5u: decompress_one<float, 32>(J, s, C, sm); break;
      case (1u << 4) | (0u << 3) | 6u: decompress_one<float, 64>(J, s, C, sm); break;
      case (1u << 4) | (0u << 3) | 7u: decompress_one<float, 128>(J, s, C, sm); break;
      case (1u << 4) | (1u << 3) | 5u: decompress_one<double, 32>(J, s, C, sm); break;
      case (1u << 4) | (1u << 3) | 6u: decompress_one<double, 64>(J, s, C, sm); break;
      case (1u << 4) | (1u << 3) | 7u: decompress_one<double, 128>(J, s, C, sm); break;
      case (2u << 4) | (0u << 3) | 5u: fused_one<32>(J, s, t, C, sm); break;
      case (2u << 4) | (0u << 3) | 6u: fused_one<64>(J, s, t, C, sm); break;
      case (2u << 4) | (0u << 3) | 7u: fused_one<128>(J, s, t, C, sm); break;
      default: break;
    }
  }
  epilogue(C);
}

// Elementwise quantisation (verification entry point).
template <typename T>
__global__ void k_quantize(const T* __restrict__ x, uint64_t n, Job J, int32_t* __restrict__ q,
                           uint8_t* __restrict__ fail) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x) {
    bool bad = false;
    int32_t qi = quant_t<T>(x[i], J, bad);
    q[i] = bad ? 0 : qi;
    fail[i] = bad ? 1 : 0;
  }
}

// Clears the control block (after a device error) without a memset node.
__global__ void k_reset(Ctl C) {
  if (threadIdx.x == 0) {
    C.ctrl->ticket = 0;
    C.ctrl->done = 0;
    C.ctrl->epoch = C.ctrl->epoch + 1;
  }
}

// ------------------------------------------------------------ launchers
template <typename T, int L>
static hipError_t launch_c(const Job& J, const Ctl& C, uint32_t tpb, uint32_t grid,
                           hipStream_t st) {
  hipLaunchKernelGGL((k_compress<T, L>), dim3(grid), dim3(tpb), 0, st, J, C);
  return hipGetLastError();
}
template <typename T, int L>
static hipError_t launch_d(const Job& J, const Ctl& C, uint32_t tpb, uint32_t grid,
                           hipStream_t st) {
  hipLaunchKernelGGL((k_decompress<T, L>), dim3(grid), dim3(tpb), 0, st, J, C);
  return hipGetLastError();
}
template <int L>
static hipError_t launch_f(const Job& J, const Ctl& C, uint32_t tpb, uint32_t grid,
                           hipStream_t st) {
  hipLaunchKernelGGL((k_fused<L>), dim3(grid), dim3(tpb), 0, st, J, C);
  return hipGetLastError();
}

hipError_t launch_single(uint32_t op, const Job& J, const Ctl& C, uint32_t tpb, uint32_t grid,
                         hipStream_t st) {
  const uint32_t key = (J.dtype << 3) | J.log2L;
  if (op == 0) {
    switch (key) {
      case 5: return launch_c<float, 32>(J, C, tpb, grid, st);
      case 6: return launch_c<float, 64>(J, C, tpb, grid, st);
      case 7: return launch_c<float, 128>(J, C, tpb, grid, st);
      case 13: return launch_c<double, 32>(J, C, tpb, grid, st);
      case 14: return launch_c<double, 64>(J, C, tpb, grid, st);
      case 15: return launch_c<double, 128>(J, C, tpb, grid, st);
    }
  } else if (op == 1) {
    switch (key) {
      case 5: return launch_d<float, 32>(J, C, tpb, grid, st);
      case 6: return launch_d<float, 64>(J, C, tpb, grid, st);
      case 7: return launch_d<float, 128>(J, C, tpb, grid, st);
      case 13: return launch_d<double, 32>(J, C, tpb, grid, st);
      case 14: return launch_d<double, 64>(J, C, tpb, grid, st);
      case 15: return launch_d<double, 128>(J, C, tpb, grid, st);
    }
  } else if (op == 2) {
    switch (key) {
      case 5: return launch_f<32>(J, C, tpb, grid, st);
      case 6: return launch_f<64>(J, C, tpb, grid, st);
      case 7: return launch_f<128>(J, C, tpb, grid, st);
    }
  }
  return hipErrorInvalidValue;
}

hipError_t launch_batch(uint32_t op, const Job* d_jobs, const uint32_t* d_strip_job,
                        uint32_t total, const Ctl& C, uint32_t tpb, uint32_t grid,
                        hipStream_t st) {
  hipLaunchKernelGGL(k_batch, dim3(grid), dim3(tpb), 0, st, d_jobs, d_strip_job, total, op, C);
  return hipGetLastError();
}

hipError_t launch_quantize(const void* x, uint64_t n, const Job& J, int32_t* q, uint8_t* fail,
                           hipStream_t st) {
  uint64_t blocks = (n + 255) / 256;
  uint32_t grid = (uint32_t)(blocks < 65536 ? (blocks ? blocks : 1) : 65536);
  if (J.dtype == 0)
    hipLaunchKernelGGL(k_quantize<float>, dim3(grid), dim3(256), 0, st, (const float*)x, n, J, q,
                       fail);
  else
    hipLaunchKernelGGL(k_quantize<double>, dim3(grid), dim3(256), 0, st, (const double*)x, n, J,
                       q, fail);
  return hipGetLastError();
}

hipError_t launch_reset(const Ctl& C, hipStream_t st) {
  hipLaunchKernelGGL(k_reset, dim3(1), dim3(64), 0, st, C);
  return hipGetLastError();
}

int occupancy_blocks(uint32_t op, uint32_t dtype, uint32_t log2L, uint32_t tpb) {
  int nb = 0;
  const void* f = nullptr;
  const uint32_t key = (dtype << 3) | log2L;
  if (op == 0) {
    switch (key) {
      case 5: f = (const void*)k_compress<float, 32>; break;
      case 6: f = (const void*)k_compress<float, 64>; break;
      case 7: f = (const void*)k_compress<float, 128>; break;
      case 13: f = (const void*)k_compress<double, 32>; break;
      case 14: f = (const void*)k_compress<double, 64>; break;
      case 15: f = (const void*)k_compress<double, 128>; break;
    }
  } else if (op == 1) {
    switch (key) {
      case 5: f = (const void*)k_decompress<float, 32>; break;
      case 6: f = (const void*)k_decompress<float, 64>; break;
      case 7: f = (const void*)k_decompress<float, 128>; break;
      case 13: f = (const void*)k_decompress<double, 32>; break;
      case 14: f = (const void*)k_decompress<double, 64>; break;
      case 15: f = (const void*)k_decompress<double, 128>; break;
    }
  } else if (op == 2) {
    switch (key) {
      case 5: f = (const void*)k_fused<32>; break;
      case 6: f = (const void*)k_fused<64>; break;
      case 7: f = (const void*)k_fused<128>; break;
    }
  } else {
    f = (const void*)k_batch;
  }
  if (!f) return 1;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, f, (int)tpb, 0) != hipSuccess || nb < 1)
    nb = 1;
  return nb;
}

}  // namespace gzk
