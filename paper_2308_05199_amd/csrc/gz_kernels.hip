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

// Look-back words and control counters are read and written at system
// scope (sc0 sc1): such accesses are not served from an XCD's own L2, so a
// word published by a workgroup on another XCD is seen on the next poll.
__device__ __forceinline__ void st_agent(unsigned long long* p, unsigned long long v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}
__device__ __forceinline__ unsigned long long ld_agent(const unsigned long long* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}
__device__ __forceinline__ uint32_t ld_agent32(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
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
// Saturating conversions (the hardware instructions are defined for every
// input; the C++ casts are not).
__device__ __forceinline__ int32_t cvt_sat(float f) {
  int32_t r;
  asm("v_cvt_i32_f32 %0, %1" : "=v"(r) : "v"(f));
  return r;
}
__device__ __forceinline__ int32_t cvt_sat(double f) {
  int32_t r;
  asm("v_cvt_i32_f64 %0, %1" : "=v"(r) : "v"(f));
  return r;
}

// When |r| < 2^29 the rounded value rr is an integer held exactly, so
// (T)q == rr and xh is formed from rr directly.
__device__ __forceinline__ int32_t quant(float x, double rinv, float t, float eblo,
                                         bool& bad) {
  float r = (float)((double)x * rinv);
  float rr = __builtin_rintf(r);
  // |rr| < 2^29 exactly when |r| < 2^29 (floats from 2^23 up are integers,
  // which rint leaves alone; below, both hold), so r dies here; NaN fails
  bool inr = fabsf(rr) < 536870912.0f;
  int32_t q = cvt_sat(rr);
  float d = x - rr * t;
  bad = !inr || !(fabsf(d) <= eblo);
  return q;
}

__device__ __forceinline__ int32_t quant(double x, double t, double eb, bool& bad) {
  double r = x / t;
  double rr = __builtin_rint(r);
  bool inr = fabs(r) <= 536870911.0;
  int32_t q = cvt_sat(rr);
  double d = x - rr * t;
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
  uint32_t cur;                  // strip being processed
  uint32_t epoch;
  uint32_t tp_key;               // decode: 1 + ticket whose table words follow
  uint32_t tp_t0, tp_t1;
  uint32_t flag;                 // strip error flags
  uint32_t hdr_ok;
  uint32_t hdr_job;              // 1 + job whose stream header was checked
  uint32_t wtot[MAX_TPB / 64];
  unsigned long long excl;       // strip exclusive prefix (dwords, chain-wide)
  unsigned long long pj;         // chain prefix at the job's first strip
  unsigned long long paydw;      // decode: payload size of the incoming stream (dwords)
  float t32;                     // decode: step of the incoming stream
  double t64;
  uint32_t hb[MAX_TPB / 4];      // header bytes of the strip's blocks
  uint32_t wts[192];             // selector weights (tile mode)
};

// Staging buffer for one strip's payload (dynamic LDS): 16 bytes of headroom
// for realigning the copy-in, TPB*32*sizeof(T) bytes, 16 bytes of tail.
extern __shared__ __attribute__((aligned(16))) uint32_t g_stage[];

__device__ __forceinline__ uint32_t first_ticket(const Ctl& C, Smem& sm) {
  if (threadIdx.x == 0) {
    sm.epoch = ld_agent32(&C.ctrl->epoch);
    sm.hdr_job = 0;
    sm.tp_key = 0;
    sm.cur = atomicAdd(&C.ctrl->ticket, 1u);
  }
  __syncthreads();
  return sm.cur;
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

// Bound of every inter-workgroup wait: C.wait_ticks of the constant-rate
// clock from the 64th unsuccessful poll (or SPIN_LIMIT polls), or another
// workgroup's timeout.  Checked every 64 polls; the clock (a scalar memory
// read) is not touched by waits that end within the first 63 polls.
__device__ __forceinline__ bool wait_over(const Ctl& C, uint32_t spins, uint64_t& t0) {
  if ((spins & 63u) != 0) return false;
  if (spins == 64) {
    t0 = (uint64_t)wall_clock64();
    return false;
  }
  return spins > SPIN_LIMIT || (uint64_t)wall_clock64() - t0 > C.wait_ticks || aborted(C);
}

// Publishes the strip aggregate (or, at the head of a chain, its prefix).
__device__ __forceinline__ void publish_agg(const Ctl& C, uint64_t gs, uint64_t chain0,
                                            uint32_t ep, uint64_t agg) {
  st_agent(C.status + gs, sw_pack(gs == chain0 ? 2 : 1, ep, agg));
}

// Decoupled look-back run by one wave after publish_agg: returns the
// exclusive prefix (dwords) of strip gs within its chain and publishes its
// inclusive prefix.  One probe reads SUB x 64 predecessors (SUB independent
// loads per lane); sub-windows resolved before a not-yet-published word are
// added in before the probe is retried from there.  Strips probe 256 words;
// the per-wave encoder, with eight times as many chain elements, probes 64
// (its status-word reads would otherwise rival its payload traffic).
constexpr int LB_SUB = 4;

template <int SUB = LB_SUB, bool PUBLISH = true>
__device__ uint64_t lookback(const Ctl& C, uint64_t gs, uint64_t chain0, uint32_t ep,
                             uint64_t agg, bool& timeout) {
  const int lane = __lane_id();
  if (gs == chain0) return 0;
  uint64_t excl = 0;
  int64_t top = (int64_t)gs - 1;
  uint32_t spins = 0;
  uint64_t t0 = 0;
  for (;;) {
    uint32_t flag[SUB];
    uint64_t val[SUB];
    // every load is issued before any is used: lanes before the chain's
    // start read its first word (a load under a divergent branch is merged
    // by register copies that wait for it at once, one round trip per load)
    uint64_t w[SUB];
#pragma unroll
    for (int m = 0; m < SUB; ++m) {
      const int64_t idx = top - 64 * m - lane;
      w[m] = ld_agent(C.status + (idx >= (int64_t)chain0 ? idx : (int64_t)chain0));
    }
#pragma unroll
    for (int m = 0; m < SUB; ++m) {
      const int64_t idx = top - 64 * m - lane;
      const bool cur = (uint32_t)((w[m] >> 34) & 0x0FFFFFFFu) == (ep & 0x0FFFFFFFu);
      const bool in_chain = idx >= (int64_t)chain0;
      flag[m] = in_chain ? (cur ? (uint32_t)(w[m] >> 62) : 0u) : 2u;
      val[m] = in_chain ? (w[m] & VMASK) : 0ull;
    }
    uint64_t part = 0;  // this lane's share of the resolved sub-windows
    int resolved = 0;   // sub-windows fully added in
    bool done = false, wait = false;
#pragma unroll
    for (int m = 0; m < SUB; ++m) {
      if (!done && !wait) {
        const uint64_t pm = __ballot(flag[m] == 2);
        const uint64_t zm = __ballot(flag[m] == 0);
        const int p = pm ? (int)__builtin_ctzll(pm) : 64;
        const uint64_t upto = p >= 63 ? ~0ull : ((2ull << p) - 1);
        if (zm & upto) {
          wait = true;
        } else {
          part += lane <= p ? val[m] : 0ull;
          ++resolved;
          done = p < 64;
        }
      }
    }
    excl += wave_sum64(part);
    if (done) break;
    top -= 64 * resolved;
    if (wait) {
      ++spins;
      if (wait_over(C, spins, t0)) {
        timeout = true;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
  }
  if (PUBLISH && lane == 0) st_agent(C.status + gs, sw_pack(2, ep, timeout ? 0 : excl + agg));
  return excl;
}

// Chain prefix at the first strip of job j (packed Scatter output).
__device__ uint64_t job_base_wait(const Ctl& C, uint32_t j, uint32_t ep, bool& timeout) {
  uint32_t spins = 0;
  uint64_t t0 = 0;
  for (;;) {
    uint64_t w = ld_agent(C.jobbase + j);
    if ((uint32_t)((w >> 34) & 0x0FFFFFFFu) == (ep & 0x0FFFFFFFu) && (w >> 62) == 2)
      return w & VMASK;
    ++spins;
    if (wait_over(C, spins, t0)) {
      timeout = true;
      return 0;
    }
    __builtin_amdgcn_s_sleep(1);
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
// ---- bit planes.  Plane j of a lane's 32 magnitudes a[i] is the word whose
// bit i is bit j of a[i].  Planes are moved 8 at a time: the bytes 8g..8g+7
// of eight magnitudes form an 8x8 bit matrix (one byte per element) that a
// three-stage delta swap transposes into one byte per plane.

// v_perm_b32: byte k of the result is byte sel.k of the 8-byte value
// (hi:lo); selector 0x0C yields a zero byte.
__device__ __forceinline__ uint32_t perm(uint32_t hi, uint32_t lo, uint32_t sel) {
  return __builtin_amdgcn_perm(hi, lo, sel);
}
// Selector taking byte b of x0..x3 (as lo, hi pairs (x0, x1), (x2, x3)).
__device__ __forceinline__ uint32_t sel_lo(uint32_t b) { return 0x0C0C0000u | ((4u + b) << 8) | b; }
__device__ __forceinline__ uint32_t sel_hi(uint32_t b) { return ((4u + b) << 24) | (b << 16) | 0x0C0Cu; }
// Byte b of four words, gathered into one word (x0's byte lowest).
__device__ __forceinline__ uint32_t gather4(uint32_t x0, uint32_t x1, uint32_t x2, uint32_t x3,
                                            uint32_t b) {
  return perm(x1, x0, sel_lo(b)) | perm(x3, x2, sel_hi(b));
}

// 8x8 bit transpose of the 64-bit value hi:lo (bit c of byte r <-> bit r of
// byte c).
__device__ __forceinline__ void tr8x8(uint32_t& lo, uint32_t& hi) {
  uint32_t t;
  t = ((lo >> 7) ^ lo) & 0x00AA00AAu;
  lo ^= t | (t << 7);
  t = ((hi >> 7) ^ hi) & 0x00AA00AAu;
  hi ^= t | (t << 7);
  t = ((lo >> 14) ^ lo) & 0x0000CCCCu;
  lo ^= t | (t << 14);
  t = ((hi >> 14) ^ hi) & 0x0000CCCCu;
  hi ^= t | (t << 14);
  const uint32_t nl = (lo & 0x0F0F0F0Fu) | ((hi << 4) & 0xF0F0F0F0u);
  const uint32_t nh = (hi & 0xF0F0F0F0u) | ((lo >> 4) & 0x0F0F0F0Fu);
  lo = nl;
  hi = nh;
}

// Writes planes 0..F-1 of a[] to dst[j * stride].
__device__ __forceinline__ void put_planes(const uint32_t (&a)[32], uint32_t F, uint32_t* dst,
                                           uint32_t stride) {
  for (uint32_t g = 0; 8 * g < F; ++g) {
    uint32_t lo[4], hi[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      lo[k] = gather4(a[8 * k], a[8 * k + 1], a[8 * k + 2], a[8 * k + 3], g);
      hi[k] = gather4(a[8 * k + 4], a[8 * k + 5], a[8 * k + 6], a[8 * k + 7], g);
      tr8x8(lo[k], hi[k]);
    }
    const uint32_t nj = min(F - 8 * g, 8u);
#pragma unroll
    for (uint32_t j = 0; j < 8; ++j) {
      if (j < nj) {
        const uint32_t b = j & 3;
        const uint32_t word = j < 4 ? gather4(lo[0], lo[1], lo[2], lo[3], b)
                                    : gather4(hi[0], hi[1], hi[2], hi[3], b);
        dst[(8 * g + j) * stride] = word;
      }
    }
  }
}

// Magnitudes a[] from planes src[j * stride], j < F (planes >= F are zero).
__device__ __forceinline__ void get_planes(const uint32_t* src, uint32_t stride, uint32_t F,
                                           uint32_t (&a)[32]) {
  if (F == 0) {
#pragma unroll
    for (int i = 0; i < 32; ++i) a[i] = 0;
    return;
  }
  {  // planes 0..7 set byte 0 and clear the rest (no separate clearing pass)
    const uint32_t nj = min(F, 8u);
    uint32_t P[8];
#pragma unroll
    for (uint32_t j = 0; j < 8; ++j) P[j] = j < nj ? src[j * stride] : 0u;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      uint32_t lo = gather4(P[0], P[1], P[2], P[3], (uint32_t)k);
      uint32_t hi = gather4(P[4], P[5], P[6], P[7], (uint32_t)k);
      tr8x8(lo, hi);
#pragma unroll
      for (int m = 0; m < 8; ++m) a[8 * k + m] = perm(m < 4 ? lo : hi, 0u, 0x0C0C0C04u + (m & 3));
    }
  }
  for (uint32_t g = 1; 8 * g < F; ++g) {
    const uint32_t nj = min(F - 8 * g, 8u);
    uint32_t P[8];
#pragma unroll
    for (uint32_t j = 0; j < 8; ++j) P[j] = j < nj ? src[(8 * g + j) * stride] : 0u;
    // a[8k+m] takes byte m of (lo, hi) of group k as its byte g
    uint32_t sel[4];
#pragma unroll
    for (uint32_t b = 0; b < 4; ++b)
      sel[b] = (0x03020100u & ~(0xFFu << (8 * g))) | ((4u + b) << (8 * g));
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      uint32_t lo = gather4(P[0], P[1], P[2], P[3], (uint32_t)k);
      uint32_t hi = gather4(P[4], P[5], P[6], P[7], (uint32_t)k);
      tr8x8(lo, hi);
#pragma unroll
      for (int m = 0; m < 8; ++m) {
        a[8 * k + m] = perm(m < 4 ? lo : hi, a[8 * k + m], sel[m & 3]);
      }
    }
  }
}

// ---- coalesced strip transfers through LDS.  A strip's raw values sit in
// LDS segment by segment with 4 dwords of padding after each 32-element
// segment, so 16-byte global accesses stay contiguous across lanes and the
// per-lane 16-byte LDS accesses hit distinct banks.
template <typename T>
__device__ __forceinline__ constexpr uint32_t seg_stride() {
  return 32 * (sizeof(T) / 4) + 4;
}

// Loads strip values src[0 .. TPB*32) (nvalid of them valid, the rest 0)
// into the LDS segment layout.
template <typename T>
__device__ __forceinline__ void strip_to_lds(const T* __restrict__ src, uint64_t nvalid) {
  constexpr uint32_t SEGW = 32 * (sizeof(T) / 4), STR = seg_stride<T>();
  const uint32_t tid = threadIdx.x, TPB = blockDim.x;
  const uint32_t nch = TPB * SEGW / 4;  // 16-byte chunks
  const uint32_t* s32 = (const uint32_t*)src;
  const uint64_t vdw = nvalid * (sizeof(T) / 4);
  uint32_t* buf = g_stage + 4;
  for (uint32_t k0 = 0; k0 < nch; k0 += 4 * TPB) {
    u4u r[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const uint32_t k = k0 + u * TPB + tid;
      const uint64_t dw = 4ull * k;
      if (k < nch && dw + 4 <= vdw) {
        r[u] = *(const u4u*)(s32 + dw);
      } else {
        r[u].x = (k < nch && dw + 0 < vdw) ? s32[dw + 0] : 0u;
        r[u].y = (k < nch && dw + 1 < vdw) ? s32[dw + 1] : 0u;
        r[u].z = (k < nch && dw + 2 < vdw) ? s32[dw + 2] : 0u;
        r[u].w = 0u;
      }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const uint32_t k = k0 + u * TPB + tid;
      if (k < nch) {
        const uint32_t dw = 4 * k;
        *(u4u*)(buf + (dw / SEGW) * STR + dw % SEGW) = r[u];
      }
    }
  }
}

// A whole input strip into the padded LDS layout with eight unconditional
// 16-byte loads in flight per lane, in straight-line code (the general copy
// above waits for every outstanding memory operation, the previous strip's
// stores included, at the top of each pass, and after each load of a
// branch that has a partial-chunk side).  Used by the fp32 encoder, whose
// registers are free at this point.
template <typename T>
__device__ __forceinline__ void strip_to_lds_whole(const T* __restrict__ src) {
  constexpr uint32_t SEGW = 32 * (sizeof(T) / 4), STR = seg_stride<T>();
  const uint32_t tid = threadIdx.x, TPB = blockDim.x;
  const uint32_t* s32 = (const uint32_t*)src;
  uint32_t* buf = g_stage + 4;
#pragma unroll
  for (uint32_t h = 0; h < SEGW / 4; h += 8) {
    u4u r[8];
#pragma unroll
    for (uint32_t u = 0; u < 8; ++u) r[u] = *(const u4u*)(s32 + 4 * ((h + u) * TPB + tid));
#pragma unroll
    for (uint32_t u = 0; u < 8; ++u) {
      const uint32_t dw = 4 * ((h + u) * TPB + tid);
      *(u4u*)(buf + (dw / SEGW) * STR + dw % SEGW) = r[u];
    }
  }
}

// The lane index as a value the compiler cannot see through: addresses
// derived from it are formed where they are used, not hoisted out of the
// persistent loop into registers held across a whole strip.
__device__ __forceinline__ uint32_t opaque_tid() {
  uint32_t t = threadIdx.x;
  asm volatile("" : "+v"(t));
  return t;
}

// Stores the LDS segment layout to dst[0 .. nvalid) with 16-byte stores.
template <typename T>
__device__ __forceinline__ void lds_to_strip(T* __restrict__ dst, uint64_t nvalid) {
  constexpr uint32_t SEGW = 32 * (sizeof(T) / 4), STR = seg_stride<T>();
  const uint32_t tid = threadIdx.x, TPB = blockDim.x;
  const uint64_t vdw = nvalid * (sizeof(T) / 4);
  const uint32_t nch = (uint32_t)min((uint64_t)TPB * SEGW / 4, (vdw + 3) / 4);
  uint32_t* d32 = (uint32_t*)dst;
  const uint32_t* buf = g_stage + 4;
  if (nvalid == (uint64_t)TPB * SEG) {  // a whole strip: 8 reads in flight, then 8 stores
    const uint32_t t = opaque_tid();
#pragma unroll
    for (uint32_t h = 0; h < SEGW / 4; h += 8) {
      u4u r[8];
#pragma unroll
      for (uint32_t u = 0; u < 8; ++u) {
        const uint32_t dw = 4 * ((h + u) * TPB + t);
        r[u] = *(const u4u*)(buf + (dw / SEGW) * STR + dw % SEGW);
      }
#pragma unroll
      for (uint32_t u = 0; u < 8; ++u) ((u4u*)(d32 + 4ull * (h + u) * TPB))[t] = r[u];
    }
    return;
  }
  for (uint32_t k = tid; k < nch; k += TPB) {
    const uint32_t dw = 4 * k;
    const u4u r = *(const u4u*)(buf + (dw / SEGW) * STR + dw % SEGW);
    if (dw + 4 <= vdw) {
      *(u4u*)(d32 + dw) = r;
    } else {
      if (dw + 0 < vdw) d32[dw + 0] = r.x;
      if (dw + 1 < vdw) d32[dw + 1] = r.y;
      if (dw + 2 < vdw) d32[dw + 2] = r.z;
    }
  }
}

// The lane's own segment in the LDS layout.
template <typename T>
__device__ __forceinline__ void lane_from_lds(T (&v)[32]);
template <>
__device__ __forceinline__ void lane_from_lds<float>(float (&v)[32]) {
  const f4u* p = (const f4u*)(g_stage + 4 + threadIdx.x * seg_stride<float>());
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const f4u r = p[k];
    v[4 * k] = r.x; v[4 * k + 1] = r.y; v[4 * k + 2] = r.z; v[4 * k + 3] = r.w;
  }
}
template <>
__device__ __forceinline__ void lane_from_lds<double>(double (&v)[32]) {
  const d2u* p = (const d2u*)(g_stage + 4 + threadIdx.x * seg_stride<double>());
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    const d2u r = p[k];
    v[2 * k] = r.x; v[2 * k + 1] = r.y;
  }
}
template <typename T>
__device__ __forceinline__ void lane_to_lds(const T (&v)[32]);
template <>
__device__ __forceinline__ void lane_to_lds<float>(const float (&v)[32]) {
  f4u* p = (f4u*)(g_stage + 4 + threadIdx.x * seg_stride<float>());
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    f4u r;
    r.x = v[4 * k]; r.y = v[4 * k + 1]; r.z = v[4 * k + 2]; r.w = v[4 * k + 3];
    p[k] = r;
  }
}
template <>
__device__ __forceinline__ void lane_to_lds<double>(const double (&v)[32]) {
  d2u* p = (d2u*)(g_stage + 4 + threadIdx.x * seg_stride<double>());
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    d2u r;
    r.x = v[2 * k]; r.y = v[2 * k + 1];
    p[k] = r;
  }
}

// Where the lane's block sits in the incoming payload (dwords from the
// payload start) and how it is coded; lets the fused step re-read a block.
struct DecInfo {
  uint32_t off_dw, kind, F;
};

// Rebuilds the lane's 32 values from its block's words at pw (LDS or global).
template <typename T, int LPB, bool FULL>
__device__ __forceinline__ void unpack_seg(const uint32_t* pw, uint32_t kind, uint32_t F,
                                           uint32_t w, uint32_t vcnt, bool exists, T t,
                                           T (&v)[32]) {
  constexpr uint32_t EW = sizeof(T) / 4;
  if (kind == K_RAW) {
#pragma unroll
    for (int i = 0; i < 32; ++i)
      v[i] = (FULL || i < (int)vcnt) ? from_raw(pw + (w * 32 + i) * EW, T()) : (T)0;
    return;
  }
  // L1D; a ZERO block (or a lane past the end) is an L1D block with base 0
  // and no planes, which decodes to +0 without a separate clearing pass
  const bool z = kind == K_ZERO || !exists;
  const int32_t base = z ? 0 : (int32_t)pw[0];
  const uint32_t Fz = z ? 0u : F;
  uint32_t a[32];
  get_planes(pw + 1 + LPB + w, LPB, Fz, a);
  const uint32_t sg = Fz ? pw[1 + w] : 0u;
  uint32_t acc = 0;
#pragma unroll
  for (int i = 0; i < 32; ++i) {
    const uint32_t neg = (uint32_t)__builtin_amdgcn_sbfe((int32_t)sg, i, 1);  // 0 or ~0
    uint32_t d = (a[i] ^ neg) - neg;
    if (i == 0 && w == 0) d = 0;
    acc += d;
    a[i] = acc;  // local prefix
  }
  const uint32_t carry = grp_excl_sum<LPB>(acc, w) + (uint32_t)base;
#pragma unroll
  for (int i = 0; i < 32; ++i) v[i] = (T)(int32_t)(carry + a[i]) * t;
}

// --------------------------------------------------------------- encode
// Per-lane result of analysing a segment: the block's kind, width and size
// (identical on the LPB lanes of a block) and this lane's share of the
// payload (base, sign word, residual magnitudes).
struct LaneCode {
  uint32_t a[32];   // |d| of the lane's 32 elements (rawregs: their fp32 bits)
  uint32_t rawregs; // RAW block whose fp32 values sit in a[]
  uint32_t sg;      // sign bits
  int32_t base;     // q of the block's first element (lane w == 0)
  uint32_t kind, F, size_dw;
  bool exists;
};

// Mode 0: 1D blocks of L consecutive elements, L1D prediction.  KEEP (fp32
// fused step): a block whose quantisation fails puts its values' bits in a[]
// for the RAW payload, from the lane's LDS segment, where the fused step
// stored them (they are not in global memory); keep_row: that segment, if
// not the strip layout's.
template <typename T, int L, bool FULL, bool KEEP = false>
__device__ __forceinline__ void analyze_1d(const Job& J, uint64_t seg, uint32_t w,
                                           const T (&v)[32], uint32_t vcnt, LaneCode& lc,
                                           const uint32_t* keep_row = nullptr) {
  constexpr int LPB = L / 32;
  constexpr uint32_t EW = sizeof(T) / 4;
  const uint64_t b = seg / LPB;
  uint32_t (&a)[32] = lc.a;
  bool bad = false;
#pragma unroll
  for (int i = 0; i < 32; ++i) {
    bool bi = false;
    int32_t qi = quant_t<T>(v[i], J, bi);
    if (FULL) {
      a[i] = (uint32_t)qi;
      bad |= bi;
    } else {
      const bool valid = i < (int)vcnt;
      a[i] = valid ? (uint32_t)qi : 0u;
      bad |= valid && bi;
    }
  }
  const int32_t base = (int32_t)a[0];
  const int32_t prev = __shfl_up((int32_t)a[31], 1);
  const uint32_t badb = grp_or<LPB>(bad ? 1u : 0u);
  const bool rawregs = KEEP && EW == 1 && badb;
  uint32_t sg = 0, orv = 0;
  if (rawregs) {
    // a RAW block stores the values themselves: the fused step left them in
    // the lane's own LDS segment (so v[] need not outlive the quantisation)
    float u[32];
    if (keep_row) {
      const f4u* p = (const f4u*)keep_row;
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const f4u r = p[k];
        u[4 * k] = r.x; u[4 * k + 1] = r.y; u[4 * k + 2] = r.z; u[4 * k + 3] = r.w;
      }
    } else {
      lane_from_lds<float>(u);
    }
#pragma unroll
    for (int i = 0; i < 32; ++i) a[i] = (FULL || i < (int)vcnt) ? __float_as_uint(u[i]) : 0u;
  } else {
    // residual magnitudes in place (downwards, so a[i-1] still holds q)
#pragma unroll
    for (int i = 31; i >= 0; --i) {
      const int32_t pq = i ? (int32_t)a[i - 1] : prev;
      int32_t d = (int32_t)(a[i] - (uint32_t)pq);
      if (i == 0 && w == 0) d = 0;
      if (!FULL && i >= (int)vcnt) d = 0;
      const uint32_t ad = (uint32_t)(d < 0 ? -d : d);
      a[i] = ad;
      orv |= ad;
      sg = __builtin_amdgcn_alignbit(sg, (uint32_t)d, 31);
    }
  }
  const uint32_t nzb = grp_or<LPB>((base != 0 ? 1u : 0u) | orv);
  orv = grp_or<LPB>(orv);

  const bool exists = FULL || b < J.B;
  const uint32_t m = FULL ? (uint32_t)L
                          : (exists ? (uint32_t)min((uint64_t)L, J.n - b * (uint64_t)L) : 0u);
  uint32_t F = orv ? 32u - (uint32_t)__clz(orv) : 0u;
  uint32_t kind, size_dw;
  const uint32_t raw_dw = m * EW;
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
  lc.rawregs = (exists && rawregs) ? 1u : 0u;
  lc.sg = sg;
  lc.base = base;
  lc.kind = kind;
  lc.F = F;
  lc.size_dw = size_dw;
  lc.exists = exists;
}

// ---- mode 1: 8x8 tiles, two lanes per tile (lane w owns rows 4w..4w+3).
__device__ __forceinline__ uint32_t bitlen(int32_t v) {
  const uint32_t a = (uint32_t)(v < 0 ? -v : v);
  return a ? 32u - (uint32_t)__clz(a) : 0u;
}

// Tile features (16 int8 bit lengths of sampled values and residuals) as
// four packed words, identical on both lanes of the tile.
__device__ __forceinline__ void tile_features(const int32_t (&q)[32], uint32_t w,
                                              uint32_t (&f)[4]) {
  // each lane computes 8 features in pairs (g0: f0 f1 | f2 f3, g1: f4 f5 |
  // f6 f7, g2: f8 f9 | f10 f11, g3: f12 f13 | f14 f15)
  uint32_t p0, p1, p2, p3;
  if (w == 0) {  // rows 0..3
    p0 = bitlen(q[0]) | bitlen(q[21]) << 8;
    p1 = bitlen(q[9] - q[8]) | bitlen(q[30] - q[29]) << 8;
    p2 = bitlen(q[11] - q[3]) | bitlen(q[25] - q[17]) << 8;
    p3 = bitlen(q[13] - q[12] - q[5] + q[4]) | bitlen(q[18] - q[17] - q[10] + q[9]) << 8;
  } else {       // rows 4..7
    p0 = bitlen(q[10]) | bitlen(q[31]) << 8;
    p1 = bitlen(q[3] - q[2]) | bitlen(q[23] - q[22]) << 8;
    p2 = bitlen(q[14] - q[6]) | bitlen(q[28] - q[20]) << 8;
    p3 = bitlen(q[13] - q[12] - q[5] + q[4]) | bitlen(q[17] - q[16] - q[9] + q[8]) << 8;
  }
  const uint32_t x0 = p0 | p1 << 16, x1 = p2 | p3 << 16;
  const uint32_t y0 = __shfl_xor(x0, 1), y1 = __shfl_xor(x1, 1);
  const uint32_t l0 = w ? y0 : x0, l1 = w ? y1 : x1;  // lane 0's pairs
  const uint32_t h0 = w ? x0 : y0, h1 = w ? x1 : y1;  // lane 1's pairs
  f[0] = (l0 & 0xFFFFu) | (h0 << 16);
  f[1] = (l0 >> 16) | (h0 & 0xFFFF0000u);
  f[2] = (l1 & 0xFFFFu) | (h1 << 16);
  f[3] = (l1 >> 16) | (h1 & 0xFFFF0000u);
}

// int8 MLP 16 -> 32 -> 3 on the tile's features; the two lanes of a tile
// each evaluate 16 hidden units.  Weights come from LDS (blob layout).
// Returns 0 NONE, 1 L1D, 2 L2D (argmax, lowest index on ties).
__device__ __forceinline__ uint32_t mlp_choose(const uint32_t (&f)[4], uint32_t w,
                                               const uint32_t* wts) {
  const int s = (int)wts[1];
  const int32_t rnd = s ? (1 << (s - 1)) : 0;
  const uint32_t* W1 = wts + 2;           // 32 rows x 4 words
  const int32_t* b1 = (const int32_t*)(wts + 2 + 128);
  const uint32_t* W2 = wts + 2 + 128 + 32;  // 3 rows x 8 words
  const int32_t* b2 = (const int32_t*)(wts + 2 + 128 + 32 + 24);
  uint32_t hp[4];
#pragma unroll
  for (int g = 0; g < 4; ++g) {
    uint32_t packed = 0;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int k = 16 * (int)w + 4 * g + u;
      int32_t acc = b1[k];
      acc = __builtin_amdgcn_sdot4((int)W1[4 * k + 0], (int)f[0], acc, false);
      acc = __builtin_amdgcn_sdot4((int)W1[4 * k + 1], (int)f[1], acc, false);
      acc = __builtin_amdgcn_sdot4((int)W1[4 * k + 2], (int)f[2], acc, false);
      acc = __builtin_amdgcn_sdot4((int)W1[4 * k + 3], (int)f[3], acc, false);
      int32_t h = (acc + rnd) >> s;
      h = h < 0 ? 0 : (h > 127 ? 127 : h);
      packed |= (uint32_t)h << (8 * u);
    }
    hp[g] = packed;
  }
  int32_t lg[3];
#pragma unroll
  for (int o = 0; o < 3; ++o) {
    int32_t acc = 0;
#pragma unroll
    for (int g = 0; g < 4; ++g)
      acc = __builtin_amdgcn_sdot4((int)W2[8 * o + 4 * w + g], (int)hp[g], acc, false);
    lg[o] = acc + __shfl_xor(acc, 1) + b2[o];
  }
  uint32_t best = 0;
  int32_t bv = lg[0];
  if (lg[1] > bv) { best = 1; bv = lg[1]; }
  if (lg[2] > bv) { best = 2; }
  return best;
}

// Residual of element i of the lane for predictor k (0 NONE, 1 L1D, 2 L2D).
// up[c] is q of the row above the lane's first row (lane 1 only).
template <int K>
__device__ __forceinline__ int32_t tile_res(const int32_t (&q)[32], const int32_t (&up)[8],
                                            uint32_t w, int i) {
  const int r = i / 8, c = i % 8;
  const int32_t x = q[i];
  if (K == 0) return x;
  const bool top = (r == 0 && w == 0);  // first row of the tile
  const int32_t left = c ? q[i - 1] : 0;
  const int32_t above = r ? q[i - 8] : up[c];
  if (K == 1) {
    if (c) return (int32_t)((uint32_t)x - (uint32_t)left);
    return top ? 0 : (int32_t)((uint32_t)x - (uint32_t)above);
  }
  if (top) return c ? (int32_t)((uint32_t)x - (uint32_t)left) : 0;
  if (!c) return (int32_t)((uint32_t)x - (uint32_t)above);
  const int32_t diag = r ? q[i - 9] : up[c - 1];
  return (int32_t)((uint32_t)x - (uint32_t)left - (uint32_t)above + (uint32_t)diag);
}

template <int K>
__device__ __forceinline__ uint32_t tile_or(const int32_t (&q)[32], const int32_t (&up)[8],
                                            uint32_t w) {
  uint32_t o = 0;
#pragma unroll
  for (int i = 0; i < 32; ++i) {
    const int32_t d = tile_res<K>(q, up, w, i);
    o |= (uint32_t)(d < 0 ? -d : d);
  }
  return grp_or<2>(o);
}

template <int K>
__device__ __forceinline__ void tile_mag(int32_t (&q)[32], const int32_t (&up)[8], uint32_t w,
                                         uint32_t& sg) {
  sg = 0;
#pragma unroll
  for (int i = 31; i >= 0; --i) {  // in place, downwards
    const int32_t d = tile_res<K>(q, up, w, i);
    q[i] = d < 0 ? -d : d;
    sg = __builtin_amdgcn_alignbit(sg, (uint32_t)d, 31);
  }
}

__device__ __forceinline__ uint32_t size_of(uint32_t kind, uint32_t F) {
  const uint32_t planes = F ? (F + 1u) * 2u : 0u;  // L = 64: two words per plane
  return kind == K_NONE ? planes : 1u + planes;
}

// Quantised tile values of the lane (used by the trial kernel and mode 1).
__device__ __forceinline__ void tile_quant(const Job& J, const float (&v)[32], int32_t (&q)[32],
                                           bool& bad) {
  bad = false;
#pragma unroll
  for (int i = 0; i < 32; ++i) {
    bool bi = false;
    q[i] = quant_t<float>(v[i], J, bi);
    bad |= bi;
  }
  bad = grp_or<2>(bad ? 1u : 0u) != 0;
}

// Mode 1 analysis: exhaustive trial (select 1), MLP (select 0) or L1D only.
__device__ __forceinline__ void analyze_tile(const Job& J, uint32_t w, const float (&v)[32],
                                             bool exists, const uint32_t* wts, LaneCode& lc) {
  int32_t (&q)[32] = *reinterpret_cast<int32_t(*)[32]>(lc.a);
  bool bad;
  tile_quant(J, v, q, bad);
  int32_t up[8];
#pragma unroll
  for (int c = 0; c < 8; ++c) up[c] = __shfl_up(q[24 + c], 1);
  const int32_t base = q[0];
  uint32_t pk;  // 0 NONE, 1 L1D, 2 L2D
  uint32_t orv;
  if (J.select == 1) {
    const uint32_t o0 = tile_or<0>(q, up, w), o1 = tile_or<1>(q, up, w), o2 = tile_or<2>(q, up, w);
    const uint32_t F0 = o0 ? 32u - __clz(o0) : 0u, F1 = o1 ? 32u - __clz(o1) : 0u,
                   F2 = o2 ? 32u - __clz(o2) : 0u;
    const uint32_t s0 = size_of(K_NONE, F0), s1 = size_of(K_L1D, F1), s2 = size_of(K_L2D, F2);
    pk = 0; orv = o0;
    uint32_t bs = s0;
    if (s1 < bs) { pk = 1; bs = s1; orv = o1; }
    if (s2 < bs) { pk = 2; orv = o2; }
  } else if (J.select == 0) {
    uint32_t f[4];
    tile_features(q, w, f);
    pk = mlp_choose(f, w, wts);
    orv = pk == 0 ? tile_or<0>(q, up, w) : pk == 1 ? tile_or<1>(q, up, w) : tile_or<2>(q, up, w);
  } else {
    pk = 1;
    orv = tile_or<1>(q, up, w);
  }
  uint32_t sg;
  if (pk == 0) tile_mag<0>(q, up, w, sg);
  else if (pk == 1) tile_mag<1>(q, up, w, sg);
  else tile_mag<2>(q, up, w, sg);
  const uint32_t nzb = grp_or<2>(base != 0 ? 1u : 0u) | orv;
  uint32_t F = orv ? 32u - (uint32_t)__clz(orv) : 0u;
  uint32_t kind = pk == 0 ? K_NONE : pk == 1 ? K_L1D : K_L2D;
  uint32_t size_dw = size_of(kind, F);
  if (!exists) {
    kind = K_ZERO; F = 0; size_dw = 0;
  } else if (bad) {
    kind = K_RAW; F = 0; size_dw = 64;
  } else if (!nzb) {
    kind = K_ZERO; F = 0; size_dw = 0;
  } else if (size_dw > 64) {
    kind = K_RAW; F = 0; size_dw = 64;
  }
  lc.rawregs = 0;  // RAW tiles re-read their values from the input
  lc.sg = sg;
  lc.base = base;
  lc.kind = kind;
  lc.F = F;
  lc.size_dw = size_dw;
  lc.exists = exists;
}

// Element i of a lane segment: its offset from the segment's first element.
template <int MODE>
__device__ __forceinline__ uint64_t seg_off(const Job& J, int i) {
  return MODE == 0 ? (uint64_t)i : (uint64_t)(i / 8) * J.nx + (i % 8);
}
// First element of segment seg (mode 1: row 4w of tile seg/2).
template <int MODE>
__device__ __forceinline__ uint64_t seg_first(const Job& J, uint64_t seg) {
  if (MODE == 0) return seg * SEG;
  const uint64_t b = seg >> 1, tpr = J.nx / 8;
  const uint64_t R = b / tpr, Cc = b - R * tpr;
  return (8 * R + 4 * (seg & 1)) * J.nx + 8 * Cc;
}

// Scan, publish, stage, look back and write one strip (any mode).  KEEPV:
// v stays valid for RAW blocks; otherwise RAW blocks re-read J.in.
// Recomputes the fused step's sums y = x' + local of a lane (RAW blocks).
struct FusedSrc {
  const uint32_t* pay;  // incoming payload (global)
  DecInfo di;
  float t;
  bool exists;
};

// Residual i of a lane read straight from its block's planes.
template <int LPB>
__device__ __forceinline__ uint32_t plane_res(const uint32_t* pw, uint32_t F, uint32_t sg,
                                              uint32_t w, int i) {
  uint32_t a = 0;
  for (uint32_t j = 0; j < F; ++j) a |= ((pw[1 + (j + 1) * LPB + w] >> i) & 1u) << j;
  const uint32_t neg = (uint32_t)__builtin_amdgcn_sbfe((int32_t)sg, i, 1);
  return (i == 0 && w == 0) ? 0u : (a ^ neg) - neg;
}

// Stages the fused step's sums y = x' + local of a RAW block bit for bit,
// re-deriving x' from the incoming block one element at a time (rare path,
// kept rolled so it adds no register pressure).
template <int LPB>
__device__ __forceinline__ void fused_raw_stage(const Job& J, const FusedSrc& fs, uint64_t seg,
                                             uint32_t w, uint32_t vcnt, uint32_t* st) {
  const uint32_t* pw = fs.pay + fs.di.off_dw;
  const uint32_t kind = fs.di.kind, F = fs.di.F;
  uint32_t carry = 0, sg = 0;
  if (kind == K_L1D) {
    sg = F ? pw[1 + w] : 0u;
    uint32_t tot = 0;
    for (int i = 0; i < 32; ++i) tot += plane_res<LPB>(pw, F, sg, w, i);
    carry = grp_excl_sum<LPB>(tot, w) + pw[0];
  }
  const float* loc = J.local + seg * SEG;
  uint32_t acc = 0;
  for (int i = 0; i < (int)vcnt; ++i) {
    float xp = 0.0f;
    if (kind == K_L1D) {
      acc += plane_res<LPB>(pw, F, sg, w, i);
      xp = (float)(int32_t)(carry + acc) * fs.t;
    } else if (kind == K_RAW) {
      xp = __uint_as_float(pw[w * 32 + i]);
    }
    st[w * 32 + i] = __float_as_uint(xp + loc[i]);
  }
}

// Word i (0..15) of the stream header for a payload of `payload` bytes.
__device__ __forceinline__ uint32_t hdr_word(const Job& J, uint32_t i, uint64_t payload) {
  const unsigned long long ebits = (unsigned long long)__double_as_longlong(J.eb);
  switch (i) {
    case 0: return 0x31435A47u;
    case 1: return 1u | (J.dtype << 16) | (J.log2L << 24);
    case 2: return (uint32_t)J.n;
    case 3: return (uint32_t)(J.n >> 32);
    case 4: return (uint32_t)ebits;
    case 5: return (uint32_t)(ebits >> 32);
    case 6: return (uint32_t)payload;
    case 7: return (uint32_t)(payload >> 32);
    case 8: return J.mode;
    case 9: return J.nx;
    case 10: return SUPER;
    default: return 0u;
  }
}

template <typename T, int L, int MODE, bool FUSED, bool FULL>
__device__ void emit_strip(const Job& J, uint64_t s, uint64_t gs, const Ctl& C, Smem& sm,
                           uint32_t vcnt, const LaneCode& lc, const FusedSrc* fs, bool skip,
                           uint32_t& tk) {
  constexpr int LPB = L / 32;
  constexpr uint32_t EW = sizeof(T) / 4;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const uint32_t TPB = blockDim.x;
  const uint64_t seg = s * TPB + tid;
  const uint32_t w = tid & (LPB - 1);
  uint32_t* stage = g_stage + 4;
  const uint32_t kind = lc.kind, F = lc.F, size_dw = lc.size_dw;

  uint32_t total;
  const uint32_t excl_lane = strip_scan(w == 0 ? size_dw : 0u, sm, total);
  const uint32_t boff = (w == 0) ? excl_lane : excl_lane - size_dw;
  if (tid == 0) publish_agg(C, gs, J.chain0, sm.epoch, total);
  if (w == 0) ((uint8_t*)sm.hb)[tid / LPB] = (uint8_t)(lc.exists ? ((kind << 5) | F) : 0u);

  // pack the payload into LDS while the predecessors resolve
  uint32_t* st = stage + boff;
  if (kind == K_L1D || kind == K_L2D || kind == K_NONE) {
    uint32_t o = 0;
    if (kind != K_NONE) {
      if (w == 0) st[0] = (uint32_t)lc.base;
      o = 1;
    }
    if (F) {
      st[o + w] = lc.sg;
      put_planes(lc.a, F, st + o + LPB + w, LPB);
    }
  }
  // a separate (not else) branch: the magnitudes are dead before it runs
  if (FUSED && kind == K_RAW && lc.rawregs) {
#pragma unroll
    for (int i = 0; i < 32; ++i)  // unrolled: a[] stays in registers
      if ((FULL && MODE == 0) || i < (int)vcnt) st[w * 32 + i] = lc.a[i];
  } else if (kind == K_RAW) {  // blocks too wide to code (rare): re-derive
    if (FUSED) {
      fused_raw_stage<L / 32>(J, *fs, seg, w, vcnt, st);
    } else {
      const T* src = (const T*)J.in + seg_first<MODE>(J, seg);
      for (int i = 0; i < (int)vcnt; ++i) {  // rolled: a rare path, kept small
        uint32_t wd[2];
        raw_words(src[seg_off<MODE>(J, i)], wd);
        st[(w * 32 + i) * EW] = wd[0];
        if (EW == 2) st[(w * 32 + i) * EW + 1] = wd[1];
      }
    }
  }

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
  __syncthreads();
  // The workgroup's next strip is ticketed only now, once this strip's
  // offset is known: a ticket held by a workgroup that has not started it
  // would stall the look-back of every later strip.
  if (tid == 0) tk = atomicAdd(&C.ctrl->ticket, 1u);
  if (sm.flag || skip) return;

  const uint64_t pj = sm.pj;
  const uint64_t erel = sm.excl - pj;  // strip offset inside this job's payload
  uint8_t* base8 = (uint8_t*)J.out + J.fixed_off + 4 * pj;
  uint32_t* dst = (uint32_t*)(base8 + J.pay_off) + erel;
  for (uint32_t k = tid; k < total; k += TPB) dst[k] = stage[k];

  if (lc.exists && (seg & (SUPER / SEG - 1)) == 0)
    ((uint32_t*)(base8 + HDR))[seg / (SUPER / SEG)] = (uint32_t)(erel + boff);
  // header bytes as whole words (the strip starts on a 4-block boundary)
  const uint32_t nblk = TPB / LPB;
  const uint64_t blk0 = s * (uint64_t)nblk;
  for (uint32_t i = tid; i < nblk / 4; i += TPB) {
    if (blk0 + 4 * i < J.B) *(uint32_t*)(base8 + J.hdr_off + blk0 + 4 * i) = sm.hb[i];
  }
  // the last strip completes the header and the size outputs
  if (s == J.nstrips - 1 && tid < 16) {
    const uint64_t payload = 4 * (sm.excl + total - pj);
    ((uint32_t*)base8)[tid] = hdr_word(J, tid, payload);
    if (tid == 0) {
      if (J.out_bytes) *J.out_bytes = J.pay_off + payload;
      if (J.chunk_off) *J.chunk_off = J.fixed_off + 4 * pj;
    }
  }
}

// Mode 0 strip encode (FULL: the strip lies entirely inside n).  fs: the
// fused step's incoming stream, to re-derive the sums of RAW blocks.
template <typename T, int L, bool FULL, bool FUSED>
__device__ __forceinline__ void encode_strip(const Job& J, uint64_t s, uint64_t gs, const Ctl& C,
                                             Smem& sm, const T (&v)[32], uint32_t vcnt,
                                             const FusedSrc* fs, bool skip, uint32_t& tk) {
  const uint64_t seg = s * blockDim.x + threadIdx.x;
  LaneCode lc;
  analyze_1d<T, L, FULL, FUSED>(J, seg, threadIdx.x & (L / 32 - 1), v, vcnt, lc);
  emit_strip<T, L, 0, FUSED, FULL>(J, s, gs, C, sm, vcnt, lc, fs, skip, tk);
}

// --------------------------------------------------------------- decode
// Checks the stream header against the job; sets sm.hdr_ok, sm.paydw, sm.t*.
__device__ void check_header(const Job& J, const uint8_t* in, uint64_t in_bytes, Smem& sm) {
  const int tid = threadIdx.x;
  if (tid < 64) {
    const bool readable = in_bytes >= HDR;
    uint32_t wv = (tid < 16 && readable) ? ((const uint32_t*)in)[tid] : 0u;
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
      default: ok = wv == 0u; break;
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
  // Marked checked only after the barrier: every wave has then read the old
  // mark and entered this function, so all of them take the same barriers.
  if (tid == 0) sm.hdr_job = J.job + 1;
}

template <typename T>
__device__ __forceinline__ T step_of(const Smem& sm);
template <>
__device__ __forceinline__ float step_of<float>(const Smem& sm) { return sm.t32; }
template <>
__device__ __forceinline__ double step_of<double>(const Smem& sm) { return sm.t64; }

// Copies payload dwords [src, src + P) into LDS with 16-byte loads; returns
// the LDS address of src[0].  Only bytes inside [lo, src + 4P) are read,
// where lo <= src is readable stream memory.
__device__ __forceinline__ const uint32_t* copy_in(const uint32_t* src, uint32_t P) {
  const uint32_t tid = threadIdx.x, TPB = blockDim.x;
  // realigned by pointer arithmetic (an integer round trip would lose the
  // pointer's global address space)
  const uint32_t delta = (uint32_t)(((uintptr_t)src & 15u) >> 2);
  const u4u* al = (const u4u*)(src - delta);
  const uint32_t nch = (delta + P + 3) / 4;  // 16-byte chunks touched
  const uint32_t full = (delta + P) / 4;     // chunks entirely inside
  u4u* dstc = (u4u*)g_stage;
  // whole chunks, four independent loads in flight per lane.  The first
  // 8 TPB chunks (all of an fp32 strip: a payload never exceeds the raw
  // size) are straight-line code: in a loop, the next pass's loads into the
  // same registers make the compiler wait for every outstanding memory
  // operation before each load.  fp64 strips may need the loop after it.
  // Lanes past the end re-read the last whole chunk instead of branching
  // around the load (a conditional load leaves a merge of registers that the
  // compiler resolves with copies, which wait for the load at once).
#pragma unroll
  for (uint32_t h = 0; h < 2; ++h) {
    const uint32_t k0 = h * 4 * TPB;
    if (full <= k0) break;
    u4u r[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) r[u] = al[min(k0 + u * TPB + tid, full - 1)];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const uint32_t k = k0 + u * TPB + tid;
      if (k < full) dstc[k] = r[u];
    }
  }
  for (uint32_t k = 8 * TPB + tid; k < full; k += TPB) dstc[k] = al[k];
  // the range ends inside the last chunk: dword loads, so that nothing past
  // it is read
  if (full < nch && tid == 0) {
    const uint32_t* p = (const uint32_t*)(al + full);
    const uint32_t lim = delta + P - 4 * full;  // 1..3 valid dwords
    u4u r;
    r.x = p[0];
    r.y = lim > 1 ? p[1] : 0u;
    r.z = lim > 2 ? p[2] : 0u;
    r.w = 0u;
    dstc[full] = r;
  }
  return g_stage + delta;
}

// Rebuilds the lane's 4 tile rows (mode 1) from its block's words at pw.
// Each lane first sums its own rows as if the row above were zero; lane 1
// then adds lane 0's last row (L2D) or its first-column value (L1D).
template <typename T>
__device__ __forceinline__ void unpack_tile(const uint32_t* pw, uint32_t kind, uint32_t F,
                                            uint32_t w, bool exists, T t, T (&v)[32]) {
  if (kind == K_RAW) {
#pragma unroll
    for (int i = 0; i < 32; ++i) v[i] = from_raw(pw + (w * 32 + i) * (sizeof(T) / 4), T());
    return;
  }
  if (kind == K_ZERO || !exists) {
#pragma unroll
    for (int i = 0; i < 32; ++i) v[i] = (T)0;
    return;
  }
  const uint32_t o = kind == K_NONE ? 0u : 1u;
  const uint32_t base = o ? pw[0] : 0u;
  uint32_t q[32];
  get_planes(pw + o + 2 + w, 2, F, q);
  const uint32_t sg = F ? pw[o + w] : 0u;
#pragma unroll
  for (int i = 0; i < 32; ++i) {  // signed residuals
    const uint32_t neg = (uint32_t)__builtin_amdgcn_sbfe((int32_t)sg, i, 1);
    q[i] = (q[i] ^ neg) - neg;
  }
  if (kind == K_L1D) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        const int i = 8 * r + c;
        if (c) q[i] = q[i - 1] + q[i];
        else if (r) q[i] = q[i - 8] + q[i];
        else q[i] = w == 0 ? base : q[i];  // (0,0) holds the base
      }
    }
    const uint32_t carry = __shfl_up(q[24], 1);  // lane 0's q(3,0)
    if (w) {
#pragma unroll
      for (int i = 0; i < 32; ++i) q[i] += carry;
    }
  } else if (kind == K_L2D) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      uint32_t acc = 0;  // v(r,c): the row prefix of d
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        const int i = 8 * r + c;
        if (r == 0 && w == 0) {
          q[i] = c ? q[i - 1] + q[i] : base;  // first row: L1D along the row
        } else {
          acc += q[i];
          q[i] = (r ? q[i - 8] : 0u) + acc;
        }
      }
    }
    uint32_t up[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) up[c] = __shfl_up(q[24 + c], 1);  // lane 0's row 3
    if (w) {
#pragma unroll
      for (int i = 0; i < 32; ++i) q[i] += up[i % 8];
    }
  }
#pragma unroll
  for (int i = 0; i < 32; ++i) v[i] = (T)(int32_t)q[i] * t;
}

// Decodes the lane's segment of strip s of the stream at `in` into v[];
// returns false (and flags the context) if the strip is malformed.
// Superblock-table words bounding strip s's payload (0 where the table is
// absent or the superblock lies past the end).
__device__ __forceinline__ void table_words(const Job& J, const uint8_t* in, uint64_t in_bytes,
                                            uint64_t s, uint32_t& T0, uint32_t& T1) {
  const uint32_t* table = (const uint32_t*)(in + HDR);
  const uint64_t sb0 = s * (uint64_t)(blockDim.x * SEG / SUPER);
  const uint64_t sbn = sb0 + blockDim.x * SEG / SUPER;
  T0 = 0;
  T1 = 0;
  if (in_bytes >= J.pay_off && J.NS) {
    // both loads issued before either is used (clamped indices, not
    // conditional loads, which the compiler waits for one at a time)
    const uint32_t a = table[min(sb0, J.NS - 1)];
    const uint32_t b = table[min(sbn, J.NS - 1)];
    T0 = sb0 < J.NS ? a : 0u;
    T1 = sbn < J.NS ? b : 0u;
  }
}

// pkey (nonzero): the strip's table words may already sit in sm.tp_t0/t1,
// fetched by thread 0 during the previous strip (when sm.tp_key == pkey).
template <typename T, int L, bool FULL, int MODE = 0>
__device__ bool decode_strip(const Job& J, const uint8_t* in, uint64_t in_bytes, uint64_t s,
                             const Ctl& C, Smem& sm, T (&v)[32], uint32_t vcnt, DecInfo& di,
                             uint32_t pkey = 0) {
  constexpr int LPB = L / 32;
  constexpr uint32_t EW = sizeof(T) / 4;
  const int tid = threadIdx.x;
  const uint32_t TPB = blockDim.x;
  const uint64_t seg = s * TPB + tid;
  const uint32_t w = tid & (LPB - 1);
  const uint64_t b = seg / LPB;

  // strip payload range from the superblock table; the table words are
  // read together with the header (both lie in the stream's fixed part,
  // readable when in_bytes reaches the payload)
  const uint32_t* table = (const uint32_t*)(in + HDR);
  const uint64_t sb0 = s * (uint64_t)(TPB * SEG / SUPER);
  const uint64_t sbn = sb0 + TPB * SEG / SUPER;
  uint32_t T0, T1;
  if (pkey && sm.tp_key == pkey) {
    T0 = sm.tp_t0;
    T1 = sm.tp_t1;
  } else {
    table_words(J, in, in_bytes, s, T0, T1);
  }
  // a lane that starts a superblock checks its table entry below; the word
  // is read now, with the others, not after the scan
  const bool exists = FULL || b < J.B;
  const bool sb_lane = exists && (seg & (SUPER / SEG - 1)) == 0;
  uint32_t Tsb = 0;
  if (in_bytes >= J.pay_off && J.NS) {  // every lane loads (clamped): no wait per load
    const uint32_t x = table[min(seg / (SUPER / SEG), J.NS - 1)];
    Tsb = sb_lane ? x : 0u;
  }
  if (sm.hdr_job != J.job + 1) check_header(J, in, in_bytes, sm);
  const bool ok = sm.hdr_ok != 0;  // implies in_bytes >= J.pay_off
  const uint64_t pay_dw = sm.paydw;
  uint64_t E = 0, En = 0;
  if (ok) {
    E = sb0 < J.NS ? T0 : pay_dw;
    En = sbn < J.NS ? T1 : pay_dw;
  }
  const bool rng = ok && E <= En && En <= pay_dw && En - E <= (uint64_t)TPB * SEG * EW;
  const uint32_t P = rng ? (uint32_t)(En - E) : 0u;
  // the header byte is loaded before the payload copy, in the same round
  // trip (after it, it would cost a second one)
  const uint32_t hb = (rng && exists) ? (uint32_t)in[J.hdr_off + b] : 0u;
  const uint32_t* S = g_stage + 4;
  if (rng) S = copy_in((const uint32_t*)(in + J.pay_off) + E, P);

  const uint32_t m = FULL ? (uint32_t)L
                          : (exists ? (uint32_t)min((uint64_t)L, J.n - b * (uint64_t)L) : 0u);
  const uint32_t kind = hb >> 5, F = hb & 31u;
  uint32_t size_dw = 0;
  bool hv = true;
  if (kind == K_ZERO) hv = F == 0;
  else if (kind == K_RAW) { hv = F == 0; size_dw = m * EW; }
  else if (kind == K_L1D || (MODE == 1 && kind == K_L2D)) size_dw = 1u + (F ? (F + 1u) * LPB : 0u);
  else if (MODE == 1 && kind == K_NONE) { hv = F > 0; size_dw = (F + 1u) * LPB; }
  else hv = false;
  if (!hv) size_dw = 0;

  uint32_t total;
  const uint32_t excl_lane = strip_scan(w == 0 ? size_dw : 0u, sm, total);
  const uint32_t boff = (w == 0) ? excl_lane : excl_lane - size_dw;
  bool good = rng && hv && total == P;
  if (good && sb_lane) good = (uint64_t)Tsb == E + boff;
  if (s == 0) good = good && E == 0;
  if (rng && s == J.nstrips - 1 && tid < 4) {
    const uint64_t pb = J.B + tid;
    if (pb < ((J.B + 3) & ~3ull)) good = good && in[J.hdr_off + pb] == 0;
  }
  good = __syncthreads_and(good ? 1 : 0) != 0;  // also completes the copy-in
  if (!good) {
    if (tid == 0) atomicOr(&C.ctrl->err, ERRF_CORRUPT);
#pragma unroll
    for (int i = 0; i < 32; ++i) v[i] = (T)0;
    return false;
  }

  di.off_dw = (uint32_t)E + boff;
  di.kind = kind;
  di.F = F;
  if (MODE == 0) unpack_seg<T, LPB, FULL>(S + boff, kind, F, w, vcnt, exists, step_of<T>(sm), v);
  else unpack_tile<T>(S + boff, kind, F, w, exists, step_of<T>(sm), v);
  return true;
}

// ---------------------------------------------------------------- kernels
template <typename T, int L, bool FULL>
__device__ __forceinline__ void compress_body(const Job& J, uint64_t s, uint64_t gs,
                                              const Ctl& C, Smem& sm, uint32_t& tk) {
  const uint64_t seg = s * blockDim.x + threadIdx.x;
  const uint64_t e0 = seg * SEG;
  const uint32_t vcnt = FULL ? 32u : (e0 >= J.n ? 0u : (uint32_t)min((uint64_t)SEG, J.n - e0));
  const uint64_t s0 = s * blockDim.x * (uint64_t)SEG;
  if (FULL && sizeof(T) == 4) strip_to_lds_whole<T>((const T*)J.in + s0);
  else strip_to_lds<T>((const T*)J.in + s0, FULL ? (uint64_t)blockDim.x * SEG : J.n - s0);
  __syncthreads();
  T v[32];
  lane_from_lds<T>(v);
  encode_strip<T, L, FULL, false>(J, s, gs, C, sm, v, vcnt, nullptr, false, tk);
}

template <typename T, int L>
__device__ __forceinline__ void compress_one(const Job& J, uint64_t s, uint64_t gs,
                                             const Ctl& C, Smem& sm, uint32_t& tk) {
  if ((s + 1) * blockDim.x * SEG <= J.n) compress_body<T, L, true>(J, s, gs, C, sm, tk);
  else compress_body<T, L, false>(J, s, gs, C, sm, tk);
}

template <typename T, int L, bool FULL>
__device__ __forceinline__ void decompress_body(const Job& J, uint64_t s, const Ctl& C,
                                                Smem& sm) {
  const uint64_t off = J.in_off ? J.in_off[J.job] : 0ull;
  const uint8_t* in = (const uint8_t*)J.in + off;
  const uint64_t avail = off <= J.in_bytes ? J.in_bytes - off : 0ull;
  const uint64_t e0 = (s * blockDim.x + threadIdx.x) * SEG;
  const uint32_t vcnt = FULL ? 32u : (e0 >= J.n ? 0u : (uint32_t)min((uint64_t)SEG, J.n - e0));
  T v[32];
  DecInfo di;
  if (decode_strip<T, L, FULL>(J, in, avail, s, C, sm, v, vcnt, di)) {
    __syncthreads();  // every lane has read its payload words
    lane_to_lds<T>(v);
    __syncthreads();
    const uint64_t s0 = s * blockDim.x * (uint64_t)SEG;
    lds_to_strip<T>((T*)J.out + s0, FULL ? (uint64_t)blockDim.x * SEG : J.n - s0);
  }
}

template <typename T, int L>
__device__ __forceinline__ void decompress_one(const Job& J, uint64_t s, const Ctl& C,
                                               Smem& sm) {
  if ((s + 1) * blockDim.x * SEG <= J.n) decompress_body<T, L, true>(J, s, C, sm);
  else decompress_body<T, L, false>(J, s, C, sm);
}

// Decode-and-accumulate (fp32): acc[i] = fl32(decoded[i] + acc[i]), the
// reduction that follows each receive in recursive-doubling Allreduce
// (Sec. 3.3.4), without writing the decoded values to memory.  A whole
// strip's accumulator is read with coalesced loads issued before the decode,
// so they are in flight while it runs.  A malformed stream leaves acc as it
// was (and flags the context).
template <int L, bool FULL>
__device__ __forceinline__ void accum_body(const Job& J, uint64_t s, const Ctl& C, Smem& sm) {
  constexpr uint32_t STR = seg_stride<float>();
  const uint32_t TPB = blockDim.x;
  const uint64_t e0 = (s * TPB + threadIdx.x) * SEG;
  const uint32_t vcnt = FULL ? 32u : (e0 >= J.n ? 0u : (uint32_t)min((uint64_t)SEG, J.n - e0));
  const uint64_t s0 = s * TPB * (uint64_t)SEG;
  uint32_t* acc = (uint32_t*)((float*)J.out + s0);
  u4u old[8];
  if (FULL) {  // chunk u*TPB + tid of the strip
    const uint32_t tid = opaque_tid();
#pragma unroll
    for (int u = 0; u < 8; ++u) old[u] = ((const u4u*)(acc + 4ull * u * TPB))[tid];
  }
  float v[32];
  DecInfo di;
  if (!decode_strip<float, L, FULL>(J, (const uint8_t*)J.in, J.in_bytes, s, C, sm, v, vcnt, di))
    return;
  __syncthreads();  // every lane has read its payload words
  lane_to_lds<float>(v);
  __syncthreads();
  const uint32_t* buf = g_stage + 4;
  if (FULL) {
    const uint32_t tid = opaque_tid();
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const uint32_t k = u * TPB + tid;  // chunk k = segment k/8, words 4*(k%8)..
      const u4u d = *(const u4u*)(buf + (k / 8) * STR + 4 * (k % 8));
      u4u y;
      y.x = __float_as_uint(__uint_as_float(d.x) + __uint_as_float(old[u].x));
      y.y = __float_as_uint(__uint_as_float(d.y) + __uint_as_float(old[u].y));
      y.z = __float_as_uint(__uint_as_float(d.z) + __uint_as_float(old[u].z));
      y.w = __float_as_uint(__uint_as_float(d.w) + __uint_as_float(old[u].w));
      ((u4u*)(acc + 4ull * u * TPB))[tid] = y;
    }
  } else {  // the tail strip: element by element
    const uint64_t nv = J.n - s0;
    for (uint32_t i = threadIdx.x; i < nv; i += TPB) {
      const float d = __uint_as_float(buf[(i / 32) * STR + i % 32]);
      acc[i] = __float_as_uint(d + __uint_as_float(acc[i]));
    }
  }
}

template <int L>
__device__ __forceinline__ void accum_one(const Job& J, uint64_t s, const Ctl& C, Smem& sm) {
  if ((s + 1) * blockDim.x * SEG <= J.n) accum_body<L, true>(J, s, C, sm);
  else accum_body<L, false>(J, s, C, sm);
}

// Single-stream decoding that fetches the next strip's table words (thread 0
// holds the next ticket, nxt) while this strip unpacks and stores, so that
// the next strip's payload copy starts at once: one dependent memory round
// trip per strip instead of two.
template <typename T, int L, bool FULL>
__device__ __forceinline__ void decompress_tp_body(const Job& J, uint64_t s, const Ctl& C,
                                                   Smem& sm, uint32_t nxt) {
  const uint8_t* in = (const uint8_t*)J.in;
  const uint64_t e0 = (s * blockDim.x + threadIdx.x) * SEG;
  const uint32_t vcnt = FULL ? 32u : (e0 >= J.n ? 0u : (uint32_t)min((uint64_t)SEG, J.n - e0));
  T v[32];
  DecInfo di;
  if (decode_strip<T, L, FULL>(J, in, J.in_bytes, s, C, sm, v, vcnt, di, (uint32_t)s + 1u)) {
    uint32_t p0 = 0, p1 = 0;
    if (threadIdx.x == 0 && nxt < J.nstrips) table_words(J, in, J.in_bytes, nxt, p0, p1);
    __syncthreads();  // every lane has read its payload words
    lane_to_lds<T>(v);
    __syncthreads();
    // read by the next strip after the loop's barrier; written before the
    // stores are issued, so that waiting for the table words does not also
    // wait for this strip's stores (the wait counter is in order)
    if (threadIdx.x == 0) {
      sm.tp_t0 = p0;
      sm.tp_t1 = p1;
      sm.tp_key = nxt + 1u;
    }
    const uint64_t s0 = s * blockDim.x * (uint64_t)SEG;
    lds_to_strip<T>((T*)J.out + s0, FULL ? (uint64_t)blockDim.x * SEG : J.n - s0);
  }
}

template <typename T, int L>
__device__ __forceinline__ void decompress_tp_one(const Job& J, uint64_t s, const Ctl& C,
                                                  Smem& sm, uint32_t nxt) {
  if ((s + 1) * blockDim.x * SEG <= J.n) decompress_tp_body<T, L, true>(J, s, C, sm, nxt);
  else decompress_tp_body<T, L, false>(J, s, C, sm, nxt);
}

// ---------------------------------------------------------- per-wave decode
// A wave decodes whole 4096-element superblocks on its own: a superblock's
// payload offset is its table entry, so waves need no scan across each
// other, no ticket and no workgroup barrier, and the phases of different
// waves (loads, unpacking, stores) overlap freely.  Superblock i goes to
// wave i mod W (W waves in the grid): decoding has no dependency between
// superblocks, so this static assignment needs no co-residency.  A wave's
// LDS region holds the superblock's payload, then its decoded values in the
// padded segment layout for coalesced stores.  Lane l decodes segments l and
// 64 + l of the superblock.
template <typename T>
struct WaveDec {
  static constexpr uint32_t WAVES = sizeof(T) == 4 ? 8 : 4;               // per workgroup
  static_assert(sizeof(T) != 4 || WAVES == DEC_WAVES_F32, "host's job shares assume this");
  static constexpr uint32_t REGION = 2 * 64 * seg_stride<T>() + 8;         // dwords per wave
};

// LDS written by some lanes of the wave is read by others: the wave's LDS
// operations complete in order, and the compiler may not move memory
// accesses across this point.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0)
  __builtin_amdgcn_wave_barrier();
  asm volatile("" ::: "memory");
}

// The lane's word of the stream header (lanes 0..15; 0 if unreadable).
__device__ __forceinline__ uint32_t wave_header_load(const Job& J, const uint8_t* in) {
  const uint32_t lane = __lane_id();
  return (lane < 16 && J.in_bytes >= HDR) ? ((const uint32_t*)in)[lane] : 0u;
}

// The stream header (the lanes' words wv) against the job, by one wave: ok,
// payload dwords and step.
template <typename T>
__device__ __forceinline__ bool wave_header_eval(const Job& J, uint32_t wv, uint64_t& paydw,
                                                 T& t) {
  const uint32_t lane = __lane_id();
  const bool readable = J.in_bytes >= HDR;
  bool ok = true;
  switch (lane) {
    case 0: ok = wv == 0x31435A47u; break;
    case 1: ok = wv == (1u | (J.dtype << 16) | (J.log2L << 24)); break;
    case 2: ok = wv == (uint32_t)J.n; break;
    case 3: ok = wv == (uint32_t)(J.n >> 32); break;
    case 8: ok = wv == J.mode; break;
    case 9: ok = wv == J.nx; break;
    case 10: ok = wv == SUPER; break;
    case 4: case 5: case 6: case 7: ok = true; break;
    default: ok = lane < 16 ? wv == 0u : true; break;
  }
  const bool allok = __ballot(ok) == ~0ull;
  const uint32_t e0 = __shfl(wv, 4), e1 = __shfl(wv, 5), p0 = __shfl(wv, 6), p1 = __shfl(wv, 7);
  const double eb = __longlong_as_double((long long)(((uint64_t)e1 << 32) | e0));
  const uint64_t payload = ((uint64_t)p1 << 32) | p0;
  bool good = readable && allok && (eb > 0.0) && isfinite(eb);
  const float t32 = (float)(2.0 * eb);
  const double t64 = 2.0 * eb;
  if (sizeof(T) == 4) good = good && isfinite(t32) && t32 != 0.0f;
  else good = good && isfinite(t64) && t64 != 0.0;
  good = good && (payload % 4 == 0) && payload <= J.in_bytes && J.pay_off <= J.in_bytes - payload;
  paydw = payload / 4;
  t = sizeof(T) == 4 ? (T)t32 : (T)t64;
  return good;
}

template <typename T>
__device__ __forceinline__ bool wave_header(const Job& J, const uint8_t* in, uint64_t& paydw,
                                            T& t) {
  return wave_header_eval<T>(J, wave_header_load(J, in), paydw, t);
}

// Block layout of superblock sb of an incoming stream, read by one wave:
// its payload range [E, En) in dwords from the payload start and, for
// segment 64h + lane (h = 0, 1), its block's kind, width, existence and
// payload offset from E; half0 = the payload dwords of the first 64
// segments' blocks.
struct WaveBlocks {
  uint64_t E, En;
  uint32_t kind[2], F[2], boff[2], half0;
  bool ex[2];
};

// The words wave_blocks_eval needs (table entries of sb and sb + 1, the
// lane's word of header bytes), read together.  SPEC: the stream header
// has not been checked yet, so offsets are clamped to the readable bytes
// (a stream that fails the check never has these words used); otherwise
// the checked header puts them inside the stream.
template <int L, bool SPEC>
__device__ __forceinline__ void wave_blocks_load(const Job& J, const uint8_t* in, uint64_t sb,
                                                 uint32_t (&raw)[3]) {
  constexpr uint32_t BPS = SUPER / L;
  const uint32_t lane = __lane_id();
  const uint64_t hb_end = (J.B + 3) & ~3ull;
  const uint64_t hidx = min(sb * BPS + 4ull * (lane & (BPS / 4 - 1)), hb_end - 4);
  const uint64_t o[3] = {HDR + 4 * sb, HDR + 4 * min(sb + 1, J.NS - 1), J.hdr_off + hidx};
  if (!SPEC) {
#pragma unroll
    for (int i = 0; i < 3; ++i) raw[i] = *(const uint32_t*)(in + o[i]);
    return;
  }
  if (J.in_bytes < 4) {  // nothing readable (the header check fails too)
    raw[0] = raw[1] = raw[2] = 0u;
    return;
  }
  const uint64_t lim = (J.in_bytes - 4) & ~3ull;
#pragma unroll
  for (int i = 0; i < 3; ++i) raw[i] = *(const uint32_t*)(in + min(o[i], lim));
}

// False if the table entries, header bytes or block sizes are inconsistent
// (the same checks as the strip decoder's); raw from wave_blocks_load, of a
// stream whose header passed.
template <typename T, int L>
__device__ bool wave_blocks_eval(const Job& J, uint64_t sb, uint64_t paydw, uint32_t nval,
                                 const uint32_t (&raw)[3], WaveBlocks& wb) {
  constexpr uint32_t EW = sizeof(T) / 4, LPB = L / 32, BPS = SUPER / L;
  const uint32_t lane = __lane_id();
  const uint32_t ta = raw[0], tb = raw[1], hraw = raw[2];
  const uint64_t b0 = sb * BPS;
  const uint64_t hb_end = (J.B + 3) & ~3ull;
  const uint32_t hw = (lane < BPS / 4 && b0 + 4ull * lane < hb_end) ? hraw : 0u;
  const uint64_t E = ta;
  const uint64_t En = sb + 1 < J.NS ? (uint64_t)tb : paydw;
  bool good = (sb != 0 || E == 0) && E <= En && En <= paydw && En - E <= (uint64_t)SUPER * EW;
  // header bytes past the last block (zero padding of the last word)
  if (lane < BPS / 4) {
#pragma unroll
    for (uint32_t k = 0; k < 4; ++k) {
      const uint64_t bb = b0 + 4ull * lane + k;
      if (bb >= J.B && bb < hb_end && ((hw >> (8 * k)) & 0xFFu)) good = false;
    }
  }
  // kinds, widths and sizes of the lane's two blocks; exclusive offsets
  uint32_t tot = 0;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const uint32_t seg = 64 * h + lane, lb = seg / LPB, w = seg % LPB;
    const uint32_t hb = (__shfl(hw, (int)(lb / 4)) >> (8 * (lb % 4))) & 0xFFu;
    const bool ex = lb * (uint32_t)L < nval;
    const uint32_t m = ex ? min((uint32_t)L, nval - lb * (uint32_t)L) : 0u;
    const uint32_t kd = ex ? hb >> 5 : 0u, f = ex ? hb & 31u : 0u;
    uint32_t size_dw = 0;
    bool hv = true;
    if (kd == K_ZERO) hv = f == 0;
    else if (kd == K_RAW) { hv = f == 0; size_dw = m * EW; }
    else if (kd == K_L1D) size_dw = 1u + (f ? (f + 1u) * LPB : 0u);
    else hv = false;
    if (!hv) size_dw = 0;
    good = good && hv;
    const uint32_t contrib = w == 0 ? size_dw : 0u;
    const uint32_t incl = wave_incl_scan(contrib);
    const uint32_t excl = tot + incl - contrib;
    wb.boff[h] = w == 0 ? excl : excl - size_dw;  // later lanes of a block contribute 0
    tot += __shfl(incl, 63);
    if (h == 0) wb.half0 = tot;
    wb.kind[h] = kd;
    wb.F[h] = f;
    wb.ex[h] = ex;
  }
  good = good && (uint64_t)tot == En - E;
  wb.E = E;
  wb.En = En;
  return __ballot(good) == ~0ull;
}


// Copies P payload dwords from src (global) into dst (LDS, 16-byte aligned),
// realigned so that every load is a whole 16-byte chunk: only bytes inside
// [16-byte floor of src, src + P) are read, and src lies past the stream's
// fixed part.  Returns where src[0] landed (dst + 0..3).  MAXW bounds P.
// UNROLL: straight-line code with uniform guards (a loop makes the compiler
// wait for every outstanding memory operation at its head, the previous
// stores included; the decoder gains, the fused step, short of registers,
// does not).
template <uint32_t MAXW, bool UNROLL>
__device__ __forceinline__ const uint32_t* wave_stage_payload(const uint32_t* src, uint32_t P,
                                                              uint32_t* dst) {
  const uint32_t lane = __lane_id();
  const uint32_t delta = (uint32_t)(((uintptr_t)src & 15u) >> 2);
  const u4u* al = (const u4u*)(src - delta);
  const uint32_t full = (delta + P) / 4, nch = (delta + P + 3) / 4;
  u4u* d4 = (u4u*)dst;
  constexpr uint32_t MAXCH = (MAXW + 3) / 4 + 1;
  if (UNROLL) {
#pragma unroll
    for (uint32_t k0 = 0; k0 < MAXCH; k0 += 8 * 64) {
      if (k0 < full) {
        u4u r[8];
#pragma unroll
        for (uint32_t u = 0; u < 8; ++u) r[u] = al[min(k0 + u * 64 + lane, full - 1)];
#pragma unroll
        for (uint32_t u = 0; u < 8; ++u)
          if (k0 + u * 64 + lane < full) d4[k0 + u * 64 + lane] = r[u];
      }
    }
  } else {
    for (uint32_t k0 = 0; k0 < MAXCH && k0 < full; k0 += 8 * 64) {
      u4u r[8];
#pragma unroll
      for (uint32_t u = 0; u < 8; ++u) r[u] = al[min(k0 + u * 64 + lane, full - 1)];
#pragma unroll
      for (uint32_t u = 0; u < 8; ++u)
        if (k0 + u * 64 + lane < full) d4[k0 + u * 64 + lane] = r[u];
    }
  }
  if (full < nch && lane == 0) {
    const uint32_t* q = (const uint32_t*)(al + full);
    const uint32_t lim = delta + P - 4 * full;  // 1..3 valid dwords
    u4u r;
    r.x = q[0];
    r.y = lim > 1 ? q[1] : 0u;
    r.z = lim > 2 ? q[2] : 0u;
    r.w = 0u;
    d4[full] = r;
  }
  return dst + delta;
}

// The stream header's first 16-byte aligned chunk (always readable once the
// header has been checked).
__device__ __forceinline__ const uint32_t* hdr_chunk(const uint8_t* in) {
  return (const uint32_t*)(in + ((0u - (uint32_t)(uintptr_t)in) & 15u));  // keeps in's address space
}

// wave_stage_payload in two parts, so that a superblock's payload is in
// flight while the wave decodes the previous one.  Issue: the first
// PAY_CPL * 64 chunks (PAY_CPL per lane: payloads up to 2048 dwords, ratio
// 2 and up; 12 per lane measured no faster on ratio-1.7 data) and the
// partial last chunk's dwords into registers, every
// load issued whatever the size (clamped to the readable bytes [16-byte
// floor of src, src + P), or to the stream header's first aligned chunk if
// that range is empty), so that each path issues the same memory
// operations.  Commit: those into dst, and any chunks past them copied
// there and then.
constexpr uint32_t PAY_CPL = 8;
struct PayRegs {
  u4u r[PAY_CPL];
  uint32_t t[3];
  const u4u* al;
  uint32_t delta, full, nch, P;
};

__device__ __forceinline__ void wave_pay_issue(const uint32_t* src, uint32_t P, const uint8_t* in,
                                               PayRegs& pr) {
  const uint32_t lane = __lane_id();
  pr.delta = (uint32_t)(((uintptr_t)src & 15u) >> 2);
  pr.al = (const u4u*)(src - pr.delta);
  pr.P = P;
  pr.full = (pr.delta + P) / 4;
  pr.nch = (pr.delta + P + 3) / 4;
  const u4u* safe = (const u4u*)hdr_chunk(in);
  const u4u* base = pr.full ? pr.al : safe;
  const uint32_t last = pr.full ? pr.full - 1 : 0u;
#pragma unroll
  for (uint32_t u = 0; u < PAY_CPL; ++u) pr.r[u] = base[min(u * 64 + lane, last)];
  const uint32_t nd = pr.delta + P;  // readable dwords from al
  const uint32_t* b32 = nd ? (const uint32_t*)pr.al : (const uint32_t*)safe;
  const uint32_t lastd = nd ? nd - 1 : 0u;
#pragma unroll
  for (uint32_t j = 0; j < 3; ++j) pr.t[j] = b32[min(4 * pr.full + j, lastd)];
}

// Returns where src[0] landed in dst (16-byte aligned LDS).
__device__ __forceinline__ const uint32_t* wave_pay_commit(const PayRegs& pr, uint32_t* dst) {
  const uint32_t lane = __lane_id();
  u4u* d4 = (u4u*)dst;
#pragma unroll
  for (uint32_t u = 0; u < PAY_CPL; ++u)
    if (u * 64 + lane < pr.full) d4[u * 64 + lane] = pr.r[u];
  if (pr.full < pr.nch && lane == 0) {
    const uint32_t lim = pr.delta + pr.P - 4 * pr.full;  // 1..3 valid dwords
    u4u r;
    r.x = pr.t[0];
    r.y = lim > 1 ? pr.t[1] : 0u;
    r.z = lim > 2 ? pr.t[2] : 0u;
    r.w = 0u;
    d4[pr.full] = r;
  }
  for (uint32_t k0 = PAY_CPL * 64; k0 < pr.full; k0 += 8 * 64) {
    u4u r[8];
#pragma unroll
    for (uint32_t u = 0; u < 8; ++u) r[u] = pr.al[min(k0 + u * 64 + lane, pr.full - 1)];
#pragma unroll
    for (uint32_t u = 0; u < 8; ++u)
      if (k0 + u * 64 + lane < pr.full) d4[k0 + u * 64 + lane] = r[u];
  }
  return dst + pr.delta;
}

template <typename T, int L, uint32_t OP, uint32_t NOLD>
__device__ __forceinline__ void wave_unpack_store(const Job& J, uint64_t sb, uint32_t nval, T t,
                                                  uint32_t* R, const uint32_t* S,
                                                  const WaveBlocks& wb, const u4u (&old)[NOLD]);

// Decodes superblock sb into J.out (OP 1), or adds it to the fp32 values
// there (OP 3, decode-and-accumulate); false (nothing written) if it is
// malformed.  raw: sb's table and header-byte words (wave_blocks_load), on
// return those of the wave's next superblock nsb (if it exists), whose
// loads go out with this superblock's payload copy.
template <typename T, int L, uint32_t OP = 1>
__device__ bool wave_decode_super(const Job& J, const uint8_t* in, uint64_t sb, uint64_t paydw,
                                  T t, uint32_t* R, uint32_t (&raw)[3], uint64_t nsb) {
  static_assert(OP == 1 || (OP == 3 && sizeof(T) == 4), "accumulation is fp32");
  constexpr uint32_t EW = sizeof(T) / 4;
  constexpr uint32_t CPL = SUPER * EW / 4 / 64;  // 16-byte chunks per lane of a superblock
  const uint32_t lane = __lane_id();
  const uint64_t e0 = sb * SUPER;
  const uint32_t nval = (uint32_t)min((uint64_t)SUPER, J.n - e0);
  uint32_t* d32 = (uint32_t*)((T*)J.out + e0);
  // OP 3: the accumulator of a whole superblock is in flight during the decode
  u4u old[OP == 3 ? CPL : 1];
  if (OP == 3 && nval == SUPER) {
#pragma unroll
    for (uint32_t u = 0; u < CPL; ++u) old[u] = ((const u4u*)d32)[u * 64 + lane];
  }
  WaveBlocks wb;
  const bool ok = wave_blocks_eval<T, L>(J, sb, paydw, nval, raw, wb);
  const uint32_t* S = R;
  if (ok)
    S = wave_stage_payload<SUPER * EW, true>((const uint32_t*)(in + J.pay_off) + wb.E,
                                             (uint32_t)(wb.En - wb.E), R);
  // the next superblock's words are in flight during this one's unpacking
  if (nsb < J.NS) wave_blocks_load<L, false>(J, in, nsb, raw);
  if (!ok) return false;
  wave_unpack_store<T, L, OP>(J, sb, nval, t, R, S, wb, old);
  return true;
}

// Decodes superblock sb (layout wb, payload staged at S in the wave's
// region R) into J.out (OP 1), or adds it to the fp32 values there (OP 3,
// old: the accumulator's superblock if whole).
template <typename T, int L, uint32_t OP, uint32_t NOLD>
__device__ __forceinline__ void wave_unpack_store(const Job& J, uint64_t sb, uint32_t nval, T t,
                                                  uint32_t* R, const uint32_t* S,
                                                  const WaveBlocks& wb, const u4u (&old)[NOLD]) {
  constexpr uint32_t EW = sizeof(T) / 4, LPB = L / 32;
  constexpr uint32_t SEGW = 32 * EW, STR = seg_stride<T>();
  constexpr uint32_t CPL = SUPER * EW / 4 / 64;  // 16-byte chunks per lane of a superblock
  const uint32_t lane = __lane_id();
  const uint64_t e0 = sb * SUPER;
  uint32_t* d32 = (uint32_t*)((T*)J.out + e0);
  wave_lds_sync();
  const uint32_t* boff = wb.boff;
  const uint32_t* kind = wb.kind;
  const uint32_t* F = wb.F;
  const bool* ex = wb.ex;
  T v0[32], v1[32];
  {
    const uint32_t seg = lane, w = seg % LPB;
    const uint32_t vc = (uint32_t)min(32, max(0, (int)nval - (int)(seg * 32)));
    if (nval == SUPER) unpack_seg<T, LPB, true>(S + boff[0], kind[0], F[0], w, vc, ex[0], t, v0);
    else unpack_seg<T, LPB, false>(S + boff[0], kind[0], F[0], w, vc, ex[0], t, v0);
  }
  {
    const uint32_t seg = 64 + lane, w = seg % LPB;
    const uint32_t vc = (uint32_t)min(32, max(0, (int)nval - (int)(seg * 32)));
    if (nval == SUPER) unpack_seg<T, LPB, true>(S + boff[1], kind[1], F[1], w, vc, ex[1], t, v1);
    else unpack_seg<T, LPB, false>(S + boff[1], kind[1], F[1], w, vc, ex[1], t, v1);
  }
  wave_lds_sync();  // every lane has read its payload words
  // values into the padded segment layout, then coalesced 16-byte stores
  {
    uint32_t* p0 = R + lane * STR;
    uint32_t* p1 = R + (64 + lane) * STR;
#pragma unroll
    for (int i = 0; i < 32; ++i) {
      uint32_t wd[2];
      raw_words(v0[i], wd);
      p0[i * EW] = wd[0];
      if (EW == 2) p0[i * EW + 1] = wd[1];
      raw_words(v1[i], wd);
      p1[i * EW] = wd[0];
      if (EW == 2) p1[i * EW + 1] = wd[1];
    }
  }
  wave_lds_sync();
  const uint32_t vdw = nval * EW;
  // decoded + old, in fp32 (OP 3)
  auto addf = [](uint32_t a, uint32_t b) { return __float_as_uint(__uint_as_float(a) + __uint_as_float(b)); };
  if (nval == SUPER) {
#pragma unroll
    for (uint32_t u = 0; u < CPL; ++u) {  // 16 (fp32) or 32 (fp64) chunks per lane
      const uint32_t k = u * 64 + lane, dw = 4 * k;
      u4u r = *(const u4u*)(R + (dw / SEGW) * STR + dw % SEGW);
      if (OP == 3) {
        r.x = addf(r.x, old[u].x);
        r.y = addf(r.y, old[u].y);
        r.z = addf(r.z, old[u].z);
        r.w = addf(r.w, old[u].w);
      }
      ((u4u*)d32)[k] = r;
    }
  } else {
    for (uint32_t k = lane; 4 * k < vdw; k += 64) {
      const uint32_t dw = 4 * k;
      u4u r = *(const u4u*)(R + (dw / SEGW) * STR + dw % SEGW);
      if (dw + 4 <= vdw) {
        if (OP == 3) {
          const u4u a = ((const u4u*)d32)[k];
          r.x = addf(r.x, a.x);
          r.y = addf(r.y, a.y);
          r.z = addf(r.z, a.z);
          r.w = addf(r.w, a.w);
        }
        ((u4u*)d32)[k] = r;
      } else {
        if (dw + 0 < vdw) d32[dw + 0] = OP == 3 ? addf(r.x, d32[dw + 0]) : r.x;
        if (dw + 1 < vdw) d32[dw + 1] = OP == 3 ? addf(r.y, d32[dw + 1]) : r.y;
        if (dw + 2 < vdw) d32[dw + 2] = OP == 3 ? addf(r.z, d32[dw + 2]) : r.z;
      }
    }
  }
  wave_lds_sync();  // the region is read before the next superblock's copy-in
}

// One step of wave_decode_whole: commits superblock sb's payload (issued a
// step earlier), evaluates the layout of the next one (its words loaded a
// step earlier), issues that payload and the words after it, then decodes
// and stores sb.
template <int L>
__device__ __forceinline__ void wave_whole_step(const Job& J, const uint8_t* in, uint64_t paydw,
                                                float t, uint32_t* R, uint64_t W, uint64_t NF,
                                                uint64_t sb, const WaveBlocks& wb, PayRegs& pr,
                                                uint32_t (&raw)[3], WaveBlocks& wbn, bool& okn) {
  const uint32_t* pay = (const uint32_t*)(in + J.pay_off);
  const uint32_t* S = wave_pay_commit(pr, R);
  const uint64_t nx = min(sb + W, NF - 1);  // past the end: a whole superblock again, unused
  okn = wave_blocks_eval<float, L>(J, nx, paydw, SUPER, raw, wbn);
  wave_pay_issue(okn ? pay + wbn.E : hdr_chunk(in), okn ? (uint32_t)(wbn.En - wbn.E) : 0u, in, pr);
  wave_blocks_load<L, false>(J, in, min(nx + W, NF - 1), raw);
  const u4u none[1] = {};
  wave_unpack_store<float, L, 1>(J, sb, SUPER, t, R, S, wb, none);
}

// The whole superblocks sb, sb + W, ... of an fp32 stream, each one's
// payload in flight while the wave decodes the one before (the first step
// is written out once, so that at the loop's head the same memory
// operations are outstanding on every path: the compiler then waits only
// for the payload, not for the previous superblock's stores).  On return sb
// is the wave's first superblock not decoded; bad is set (and decoding
// stops) at a malformed one.
template <int L>
__device__ __forceinline__ void wave_decode_whole(const Job& J, const uint8_t* in, uint64_t paydw,
                                                  float t, uint32_t* R, uint64_t W, uint64_t& sb,
                                                  bool& bad) {
  const uint64_t NF = J.n / SUPER;
  if (sb >= NF) return;
  const uint32_t* pay = (const uint32_t*)(in + J.pay_off);
  uint32_t raw[3];
  wave_blocks_load<L, false>(J, in, sb, raw);
  WaveBlocks wb, wbn;
  bool ok = wave_blocks_eval<float, L>(J, sb, paydw, SUPER, raw, wb), okn;
  PayRegs pr;
  wave_pay_issue(ok ? pay + wb.E : hdr_chunk(in), ok ? (uint32_t)(wb.En - wb.E) : 0u, in, pr);
  wave_blocks_load<L, false>(J, in, min(sb + W, NF - 1), raw);
  if (!ok) {
    bad = true;
    return;
  }
  wave_whole_step<L>(J, in, paydw, t, R, W, NF, sb, wb, pr, raw, wbn, okn);
  for (sb += W; sb < NF; sb += W) {
    if (!okn) {
      bad = true;
      return;
    }
    wb = wbn;
    wave_whole_step<L>(J, in, paydw, t, R, W, NF, sb, wb, pr, raw, wbn, okn);
  }
}

template <typename T, int L>
__global__ __launch_bounds__(WaveDec<T>::WAVES * 64)
__attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 2 : 1, 2))) void k_decompress_w(Job J, Ctl C) {
  const uint32_t wid = threadIdx.x >> 6;
  uint32_t* R = g_stage + wid * WaveDec<T>::REGION;
  const uint8_t* in = (const uint8_t*)J.in;
  uint64_t paydw = 0;
  T t = 0;
  bool bad = !wave_header<T>(J, in, paydw, t);
  if (!bad) {
    const uint64_t W = (uint64_t)gridDim.x * (blockDim.x >> 6);
    uint64_t sb = (uint64_t)blockIdx.x * (blockDim.x >> 6) + wid;
    if constexpr (sizeof(T) == 4) wave_decode_whole<L>(J, in, paydw, t, R, W, sb, bad);
    if (!bad) {  // the rest (fp64: all), one superblock at a time
      uint32_t raw[3] = {0u, 0u, 0u};
      if (sb < J.NS) wave_blocks_load<L, false>(J, in, sb, raw);
      for (; sb < J.NS; sb += W)
        if (!wave_decode_super<T, L>(J, in, sb, paydw, t, R, raw, sb + W)) bad = true;
    }
  }
  if (bad && __lane_id() == 0) atomicOr(&C.ctrl->err, ERRF_CORRUPT);
}

// Single-stream decode-and-accumulate by waves (fp32): as k_decompress_w,
// each superblock added to the accumulator J.out.
template <int L>
__global__ __launch_bounds__(WaveDec<float>::WAVES * 64)
__attribute__((amdgpu_waves_per_eu(2, 2))) void k_accum_w(Job J, Ctl C) {
  const uint32_t wid = threadIdx.x >> 6;
  uint32_t* R = g_stage + wid * WaveDec<float>::REGION;
  const uint8_t* in = (const uint8_t*)J.in;
  uint64_t paydw = 0;
  float t = 0;
  bool bad = !wave_header<float>(J, in, paydw, t);
  if (!bad) {
    const uint64_t W = (uint64_t)gridDim.x * (blockDim.x >> 6);
    const uint64_t sb0 = (uint64_t)blockIdx.x * (blockDim.x >> 6) + wid;
    uint32_t raw[3] = {0u, 0u, 0u};
    if (sb0 < J.NS) wave_blocks_load<L, false>(J, in, sb0, raw);
    for (uint64_t sb = sb0; sb < J.NS; sb += W)
      if (!wave_decode_super<float, L, 3>(J, in, sb, paydw, t, R, raw, sb + W)) bad = true;
  }
  if (bad && __lane_id() == 0) atomicOr(&C.ctrl->err, ERRF_CORRUPT);
}

// One superblock of a batch job: the job's stream (at its scatter offset,
// if any) is checked and the superblock decoded (OP 1) or accumulated (OP 3).
template <typename T, int L, uint32_t OP>
__device__ __forceinline__ bool wave_batch_super(const Job& J, uint64_t sb, uint32_t* R) {
  const uint64_t off = J.in_off ? J.in_off[J.job] : 0ull;
  Job Jl = J;
  Jl.in_bytes = off <= J.in_bytes ? J.in_bytes - off : 0ull;
  const uint8_t* in = (const uint8_t*)J.in + off;
  uint32_t raw[3];
  wave_blocks_load<L, true>(Jl, in, sb, raw);  // in flight with the header's words
  uint64_t paydw = 0;
  T t = 0;
  if (!wave_header<T>(Jl, in, paydw, t)) return false;
  return wave_decode_super<T, L, OP>(Jl, in, sb, paydw, t, R, raw, ~0ull);
}

// Superblocks first, first + stride, ... of one fp32 stream (job J, its
// stream at in) by one wave, whole ones pipelined as in k_decompress_w.
template <int L>
__device__ __forceinline__ void wave_job_decode(const Job& J, const uint8_t* in, uint64_t first,
                                                uint64_t stride, uint32_t* R, bool& bad) {
  uint64_t paydw = 0;
  float t = 0;
  if (!wave_header<float>(J, in, paydw, t)) {
    bad = true;
    return;
  }
  uint64_t sb = first;
  wave_decode_whole<L>(J, in, paydw, t, R, stride, sb, bad);
  if (bad) return;
  uint32_t raw[3] = {0u, 0u, 0u};
  if (sb < J.NS) wave_blocks_load<L, false>(J, in, sb, raw);
  for (; sb < J.NS; sb += stride)
    if (!wave_decode_super<float, L>(J, in, sb, paydw, t, R, raw, sb + stride)) bad = true;
}

// Batched decoding (OP 1) or decode-and-accumulate (OP 3) by waves: batch
// superblock i is superblock map[2i + 1] of job map[2i], or, without a map
// (jobs of equal superblock counts), superblock i / njobs of job i % njobs;
// waves take them statically.  WIDE: the batch holds fp64 jobs (fp64-sized
// regions, four waves per workgroup).  jw (decoding an fp32 1D batch): the
// map holds jw (job, first superblock, stride) triples instead, one per
// wave's share (waves take them statically): each decodes superblocks
// first, first + stride, ... of its job with the pipelined single-stream
// decoder.
template <bool WIDE, uint32_t OP>
__global__ __launch_bounds__((WIDE ? WaveDec<double>::WAVES : WaveDec<float>::WAVES) * 64)
__attribute__((amdgpu_waves_per_eu(WIDE ? 1 : 2, 2))) void k_batch_decode_w(
    const Job* __restrict__ jobs, const uint32_t* __restrict__ map, uint32_t njobs,
    uint32_t total, uint32_t jw, Ctl C) {
  constexpr uint32_t WAVES = WIDE ? WaveDec<double>::WAVES : WaveDec<float>::WAVES;
  constexpr uint32_t REGION = WIDE ? WaveDec<double>::REGION : WaveDec<float>::REGION;
  const uint32_t wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  uint32_t* R = g_stage + wid * REGION;
  bool bad = false;
  const uint32_t W = gridDim.x * WAVES;
  if constexpr (!WIDE && OP == 1) {
    if (jw) {
      for (uint32_t w = blockIdx.x * WAVES + wid; w < jw; w += W) {
        Job J = jobs[map[3 * (uint64_t)w]];
        const uint64_t first = map[3 * (uint64_t)w + 1], stride = map[3 * (uint64_t)w + 2];
        const uint64_t off = J.in_off ? J.in_off[J.job] : 0ull;
        J.in_bytes = off <= J.in_bytes ? J.in_bytes - off : 0ull;
        const uint8_t* in = (const uint8_t*)J.in + off;
        bool jb = false;  // this share's job only
        switch (J.log2L) {
          case 5: wave_job_decode<32>(J, in, first, stride, R, jb); break;
          case 6: wave_job_decode<64>(J, in, first, stride, R, jb); break;
          case 7: wave_job_decode<128>(J, in, first, stride, R, jb); break;
          default: jb = true; break;
        }
        bad = bad || jb;
      }
      if (bad && __lane_id() == 0) atomicOr(&C.ctrl->err, ERRF_CORRUPT);
      return;
    }
  }
  for (uint32_t i = blockIdx.x * WAVES + wid; i < total; i += W) {
    const uint32_t j = map ? map[2 * (uint64_t)i] : i % njobs;
    const uint64_t sb = map ? map[2 * (uint64_t)i + 1] : i / njobs;
    const Job J = jobs[j];
    bool ok = false;
    switch ((J.dtype << 3) | J.log2L) {
      case 5: ok = wave_batch_super<float, 32, OP>(J, sb, R); break;
      case 6: ok = wave_batch_super<float, 64, OP>(J, sb, R); break;
      case 7: ok = wave_batch_super<float, 128, OP>(J, sb, R); break;
      case 13: if constexpr (WIDE && OP == 1) ok = wave_batch_super<double, 32, 1>(J, sb, R); break;
      case 14: if constexpr (WIDE && OP == 1) ok = wave_batch_super<double, 64, 1>(J, sb, R); break;
      case 15: if constexpr (WIDE && OP == 1) ok = wave_batch_super<double, 128, 1>(J, sb, R); break;
      default: break;
    }
    if (!ok) bad = true;
  }
  if (bad && __lane_id() == 0) atomicOr(&C.ctrl->err, ERRF_CORRUPT);
}

// ---------------------------------------------------------- per-wave encode
// fp32 1D encoding (compression and the fused step) by single waves.  A wave
// claims a superblock, builds its payload in LDS in two halves of 64
// segments (lane l codes segment 64h + l), learns its offset and writes
// payload, table word and header bytes.  There is no workgroup barrier, so
// the waves of a CU are in different phases (loads, arithmetic, waits,
// stores) at once.  Offsets come from a two-level scan: a workgroup claims
// rounds of WAVES consecutive superblocks with one global ticket; inside a
// round the waves combine their sizes through LDS, and the round is one
// element of the decoupled look-back (a look-back per superblock measured
// slower than strips: eight times as many chain elements published eight
// times as fast outrun a 64-word probe within one memory round trip).
// Wave region (dwords): X and A, each 64 padded segments, and HB, the
// superblock's header bytes.  Compression: input values through X, first
// half's payload in A, second half's in X.  Fused step: the incoming payload
// staged in X (whole, or half by half if it does not fit); each lane loads
// its own addend row; the first half's sums (kept for RAW blocks) and then
// payload in A, the second half's sums and payload in X.
struct WaveEnc {
  static constexpr uint32_t WAVES = 8;  // per workgroup
  static constexpr uint32_t STR = 36;   // seg_stride<float>()
  static constexpr uint32_t XW = 64 * STR, AW = 64 * STR, HBW = SUPER / 32 / 4;
  static constexpr uint32_t REGION = XW + AW + HBW + 4;
};

// One half's 2048 values src[0 .. hval) into registers, 16-byte loads, eight
// per lane in flight (positions past hval read as 0).
__device__ __forceinline__ void wave_half_load(const uint32_t* src, uint32_t hval, u4u (&r)[8]) {
  const uint32_t lane = __lane_id();
  if (hval == 64 * SEG) {
#pragma unroll
    for (uint32_t u = 0; u < 8; ++u) r[u] = ((const u4u*)src)[u * 64 + lane];
    return;
  }
#pragma unroll
  for (uint32_t u = 0; u < 8; ++u) {
    const uint32_t dw = 4 * (u * 64 + lane);
    if (dw + 4 <= hval) {
      r[u] = *(const u4u*)(src + dw);
    } else {
      r[u].x = dw + 0 < hval ? src[dw + 0] : 0u;
      r[u].y = dw + 1 < hval ? src[dw + 1] : 0u;
      r[u].z = dw + 2 < hval ? src[dw + 2] : 0u;
      r[u].w = 0u;
    }
  }
}

// The lane's own row of 32 values at src (vcnt valid, the rest 0): eight
// 16-byte loads, each instruction touching a line per lane, nearly all L1
// hits after the first.
template <bool FULL>
__device__ __forceinline__ void wave_row_load(const uint32_t* src, uint32_t vcnt, u4u (&r)[8]) {
#pragma unroll
  for (uint32_t k = 0; k < 8; ++k) {
    if (FULL) {
      r[k] = ((const u4u*)src)[k];
    } else {
      const uint32_t dw = 4 * k;
      if (dw + 4 <= vcnt) {
        r[k] = *(const u4u*)(src + dw);
      } else {
        r[k].x = dw + 0 < vcnt ? src[dw + 0] : 0u;
        r[k].y = dw + 1 < vcnt ? src[dw + 1] : 0u;
        r[k].z = dw + 2 < vcnt ? src[dw + 2] : 0u;
        r[k].w = 0u;
      }
    }
  }
}

// Registers of wave_half_load into X's padded segment layout.
__device__ __forceinline__ void wave_regs_to_x(const u4u (&r)[8], uint32_t* X) {
  const uint32_t lane = __lane_id();
#pragma unroll
  for (uint32_t u = 0; u < 8; ++u) {
    const uint32_t dw = 4 * (u * 64 + lane);
    *(u4u*)(X + (dw / SEG) * WaveEnc::STR + dw % SEG) = r[u];
  }
}

__device__ __forceinline__ void wave_row_get(const uint32_t* X, float (&v)[32]) {
  const f4u* p = (const f4u*)(X + __lane_id() * WaveEnc::STR);
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const f4u r = p[k];
    v[4 * k] = r.x; v[4 * k + 1] = r.y; v[4 * k + 2] = r.z; v[4 * k + 3] = r.w;
  }
}

__device__ __forceinline__ void wave_row_put(uint32_t* X, const float (&v)[32]) {
  f4u* p = (f4u*)(X + __lane_id() * WaveEnc::STR);
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    f4u r;
    r.x = v[4 * k]; r.y = v[4 * k + 1]; r.z = v[4 * k + 2]; r.w = v[4 * k + 3];
    p[k] = r;
  }
}

// The lane's share of its block's payload at st (the block's first word):
// base, sign word and planes of an L1D block, or the values of a RAW block
// (from registers, re-derived by the fused step, or re-read from J.in).
template <int L, bool FUSED, bool FULL>
__device__ __forceinline__ void wave_pack(const Job& J, uint64_t seg, uint32_t w, uint32_t vcnt,
                                          const LaneCode& lc, const FusedSrc& fs, uint32_t* st) {
  constexpr uint32_t LPB = L / 32;
  if (lc.kind == K_L1D) {
    if (w == 0) st[0] = (uint32_t)lc.base;
    if (lc.F) {
      st[1 + w] = lc.sg;
      put_planes(lc.a, lc.F, st + 1 + LPB + w, LPB);
    }
  }
  if (FUSED && lc.kind == K_RAW && lc.rawregs) {
#pragma unroll
    for (int i = 0; i < 32; ++i)  // unrolled: a[] stays in registers
      if (FULL || i < (int)vcnt) st[w * 32 + i] = lc.a[i];
  } else if (lc.kind == K_RAW) {  // blocks too wide to code (rare)
    if (FUSED) {
      fused_raw_stage<LPB>(J, fs, seg, w, vcnt, st);
    } else {
      const float* src = (const float*)J.in + seg * SEG;
      for (int i = 0; i < (int)vcnt; ++i) st[w * 32 + i] = __float_as_uint(src[i]);
    }
  }
}

// The fused step's first words of a superblock (the incoming stream's
// header word of the lane, table and header-byte words), loaded ahead.
struct UnitPre {
  uint32_t wv, raw[3];
  bool valid;
};

template <int L>
__device__ __forceinline__ void wave_unit_preload(const Job& J, uint64_t u, UnitPre& p) {
  const uint8_t* in = (const uint8_t*)J.in;
  wave_blocks_load<L, true>(J, in, u, p.raw);
  p.wv = wave_header_load(J, in);
  p.valid = true;
}

// Encodes superblock u of job J into the wave's region (fused: incoming
// stream J.in plus addend J.local; ahead: its first words if loaded ahead):
// tot[0] payload dwords in A, tot[1] in X, header bytes in HB; good is false
// for a malformed incoming superblock.  pub(size) is called with the whole
// size as soon as it is known, before the second half is packed.
template <int L, bool FUSED, bool FULL, class Pub>
__device__ __forceinline__ void wave_encode_unit(const Job& J, uint64_t u, uint32_t* R,
                                                 uint32_t (&tot)[2], bool& good,
                                                 const UnitPre& ahead, const Pub& pub) {
  constexpr uint32_t LPB = L / 32, BPS = SUPER / L, HALF = 64 * SEG;
  const uint32_t lane = __lane_id();
  const uint32_t w = lane & (LPB - 1);
  uint32_t* X = R;
  uint32_t* A = R + WaveEnc::XW;
  uint32_t* HB = A + WaveEnc::AW;
  const uint64_t e0 = u * SUPER;
  const uint32_t nval = FULL ? SUPER : (uint32_t)min((uint64_t)SUPER, J.n - e0);
  const uint8_t* in = (const uint8_t*)J.in;
  u4u pre[8];  // compression: the input half in flight
  if (!FUSED)
    wave_half_load((const uint32_t*)((const float*)J.in + e0),
                   FULL ? HALF : (uint32_t)min((uint32_t)HALF, nval), pre);

  // the incoming superblock's layout (fused step)
  good = true;
  WaveBlocks wb = {};
  FusedSrc fs;
  fs.pay = (const uint32_t*)(in + J.pay_off);
  fs.t = 0.0f;
  if (FUSED) {
    uint64_t paydw = 0;
    UnitPre p = ahead;
    if (!p.valid) wave_unit_preload<L>(J, u, p);  // table words with the header's
    good = wave_header_eval<float>(J, p.wv, paydw, fs.t);
    if (good) good = wave_blocks_eval<float, L>(J, u, paydw, nval, p.raw, wb);
  }
  // the whole incoming payload is staged at once when its realigned copy
  // fits X (always, at any ratio above about 1.8)
  const uint32_t Ptot = good ? (uint32_t)(wb.En - wb.E) : 0u;
  const bool whole = FUSED && Ptot + 8 <= WaveEnc::XW;
  const uint32_t* S = X;

#pragma unroll
  for (uint32_t h = 0; h < 2; ++h) {
    const uint32_t hval =
        FULL ? HALF : (uint32_t)min((int)HALF, max(0, (int)nval - (int)(h * HALF)));
    const uint64_t seg = e0 / SEG + 64 * h + lane;
    const uint32_t vcnt = FULL ? 32u : (uint32_t)min(32, max(0, (int)hval - 32 * (int)lane));
    float v[32];
    if (FUSED) {
      uint32_t* AD = h ? X : A;  // the sums' rows
      const uint32_t hoff = (h && !whole) ? wb.half0 : 0u;
      if (good && (h == 0 || !whole)) {
        const uint32_t P = whole ? Ptot : (h ? Ptot - wb.half0 : wb.half0);
        S = wave_stage_payload<SUPER, false>(fs.pay + wb.E + hoff, P, X);
      }
      // the lane's own 32 addend values, in flight during the decode (a
      // coalesced load transposed through LDS measured slower here)
      u4u lr[8];
      wave_row_load<FULL>((const uint32_t*)(J.local + e0 + h * HALF) + 32 * lane, vcnt, lr);
      if (good) {
        wave_lds_sync();
        unpack_seg<float, LPB, FULL>(S + (wb.boff[h] - hoff), wb.kind[h], wb.F[h], w, vcnt,
                                     wb.ex[h], fs.t, v);
        fs.di.off_dw = (uint32_t)wb.E + wb.boff[h];
        fs.di.kind = wb.kind[h];
        fs.di.F = wb.F[h];
      } else {
#pragma unroll
        for (int i = 0; i < 32; ++i) v[i] = 0.0f;
        fs.di.off_dw = 0;
        fs.di.kind = K_ZERO;
        fs.di.F = 0;
      }
      wave_lds_sync();  // payload words read before X takes the sums
#pragma unroll
      for (int k = 0; k < 8; ++k) {  // incoming + local, fp32
        v[4 * k] = v[4 * k] + __uint_as_float(lr[k].x);
        v[4 * k + 1] = v[4 * k + 1] + __uint_as_float(lr[k].y);
        v[4 * k + 2] = v[4 * k + 2] + __uint_as_float(lr[k].z);
        v[4 * k + 3] = v[4 * k + 3] + __uint_as_float(lr[k].w);
      }
      wave_row_put(AD, v);  // the sums, for a RAW block (own row)
    } else {
      // the first half's loads were issued by the caller (pre); the second
      // half's go out as soon as the first half's registers are free
      wave_regs_to_x(pre, X);
      wave_lds_sync();
      wave_row_get(X, v);
      if (h == 0) {
        const uint32_t h1 =
            FULL ? HALF : (uint32_t)min((int)HALF, max(0, (int)nval - (int)HALF));
        wave_half_load((const uint32_t*)((const float*)J.in + e0 + HALF), h1, pre);
      }
    }
    LaneCode lc;
    analyze_1d<float, L, FULL, FUSED>(J, seg, w, v, vcnt, lc,
                                      FUSED ? (h ? X : A) + lane * WaveEnc::STR : nullptr);
    const uint32_t contrib = w == 0 ? lc.size_dw : 0u;
    const uint32_t incl = wave_incl_scan(contrib);
    const uint32_t boff = w == 0 ? incl - contrib : incl - lc.size_dw;
    tot[h] = __shfl(incl, 63);
    if (h == 1) pub(tot[0] + tot[1]);
    if (w == 0)
      ((uint8_t*)HB)[(64 * h + lane) / LPB] =
          (uint8_t)(lc.exists ? ((lc.kind << 5) | lc.F) : 0u);
    wave_lds_sync();  // every row of X is read before the second half's payload goes there
    wave_pack<L, FUSED, FULL>(J, seg, w, vcnt, lc, fs, (h ? X : A) + boff);
  }
  wave_lds_sync();  // A, X and HB are complete
}

// Writes superblock u's payload (tot[0] dwords from A, tot[1] from X) at
// dword offset ex of the job's payload, its table word and header bytes;
// the job's last superblock also writes the stream header and size.
template <int L>
__device__ __forceinline__ void wave_write_unit(const Job& J, uint64_t u, uint64_t ex,
                                                const uint32_t (&tot)[2], const uint32_t* R) {
  constexpr uint32_t BPS = SUPER / L;
  const uint32_t lane = __lane_id();
  const uint32_t* X = R;
  const uint32_t* A = R + WaveEnc::XW;
  const uint32_t* HB = A + WaveEnc::AW;
  uint8_t* base8 = (uint8_t*)J.out;
  uint32_t* dst = (uint32_t*)(base8 + J.pay_off) + ex;
  for (uint32_t k = lane; k < tot[0]; k += 64) dst[k] = A[k];
  for (uint32_t k = lane; k < tot[1]; k += 64) dst[tot[0] + k] = X[k];
  if (lane == 0) ((uint32_t*)(base8 + HDR))[u] = (uint32_t)ex;
  const uint64_t b0 = u * BPS;
  if (lane < BPS / 4 && b0 + 4 * lane < J.B)
    *(uint32_t*)(base8 + J.hdr_off + b0 + 4 * lane) = HB[lane];
  if (u == J.NS - 1 && lane < 16) {
    const uint64_t payload = 4 * (ex + tot[0] + tot[1]);
    ((uint32_t*)base8)[lane] = hdr_word(J, lane, payload);
    if (lane == 0 && J.out_bytes) *J.out_bytes = J.pay_off + payload;
  }
  wave_lds_sync();  // the region is read before the next superblock reuses it
}

// ---- rounds.  A workgroup's waves claim slots of rounds through an LDS
// counter (claim k: round k / WAVES, slot k % WAVES).  A round's global
// ticket T is taken by the wave that fetched the previous round's prefix,
// right after: the previous round's waves are then about to write and
// claim again, so the ticket is held for about one write-out and the
// round's first claimer need not wait for the atomic (a round past the end
// hands on a ticket past the end; round 0's first claimer takes its own).
// Slot s of the round is superblock WAVES * (T's round within its job) + s.  Per round (a ring of RING
// entries in LDS): the slots' sizes, a count of them, and the round's
// exclusive prefix, fetched by one elected wave with the look-back over
// rounds.  The wave that completes the count publishes the round's
// aggregate (or its inclusive prefix, if the prefix is known); the fetcher
// publishes the inclusive prefix if the count is complete.  Either way the
// round's status word is published, and an inclusive word is not left
// overwritten by an aggregate (the completer re-checks for the prefix once
// its aggregate store has completed).
// Deadlock freedom: every wait is on earlier rounds (tickets handed to
// running workgroups) or on earlier slots of the same round (claimed
// before, by waves of the same workgroup); the first claimer of a round
// waits for the round RING earlier in the same entry to be released by all
// its claimers, each of which releases it once.  Nothing assumes that the
// grid's workgroups are resident together, and every wait is bounded.
constexpr uint32_t RING = 4;
constexpr uint32_t SIZE_NONE = 0xFFFFFFFFu;

struct RoundState {
  unsigned long long prefix;  // exclusive prefix of the round (dwords)
  uint32_t pticket;   // this entry's next round's ticket, taken ahead ...
  uint32_t pflag;     // ... by the previous round: 1 + the round it is for
  uint32_t ticket;
  uint32_t ready;     // 1 + round number once ticket (and the reset) is done
  uint32_t cnt;       // sizes written
  uint32_t fetch;     // 1 once a wave has been elected to fetch the prefix
  uint32_t pready;    // 1 + round number once prefix is set
  uint32_t released;  // claimers done with this entry
  uint32_t size[WaveEnc::WAVES];
};
struct WaveSched {
  uint32_t claim;
  RoundState rs[RING];
};

// Clears the schedule (before the workgroup's first barrier).
__device__ __forceinline__ void wave_sched_init(WaveSched& ws) {
  if (threadIdx.x == 0) {
    ws.claim = 0;
#pragma unroll
    for (uint32_t i = 0; i < RING; ++i) {
      ws.rs[i].ready = 0;
      ws.rs[i].pflag = 0;
      ws.rs[i].released = WaveEnc::WAVES;
    }
  }
  __syncthreads();
}

__device__ __forceinline__ uint32_t lds_load_acq(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void lds_store_rel(uint32_t* p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Bounded wait until *p >= want (lane 0 polls); false on timeout.
__device__ __forceinline__ bool lds_wait_ge(const Ctl& C, const uint32_t* p, uint32_t want) {
  uint32_t ok = 1;
  if (__lane_id() == 0) {
    uint32_t spins = 0;
    uint64_t t0 = 0;
    while (lds_load_acq(p) < want) {
      if (wait_over(C, ++spins, t0)) {
        atomicOr(&C.ctrl->err, ERRF_TIMEOUT);
        ok = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
  }
  return __shfl(ok, 0) != 0;
}

struct Claim {
  uint32_t round, slot, ticket;  // ticket 0xFFFFFFFF: timed out
  bool done;                     // ticket known
};

// A round's first claimer opens it: resets the entry, takes the round's
// ticket (handed on, or, for round 0, from the counter) and marks it ready.
__device__ __forceinline__ uint32_t wave_round_open(const Ctl& C, RoundState& rs,
                                                    uint32_t round) {
  uint32_t t = 0;
  if (__lane_id() == 0) {
    rs.cnt = 0;
    rs.fetch = 0;
    rs.pready = 0;
    rs.released = 0;
#pragma unroll
    for (uint32_t i = 0; i < WaveEnc::WAVES; ++i) rs.size[i] = SIZE_NONE;
    t = round > 0 ? rs.pticket : atomicAdd(&C.ctrl->ticket, 1u);
    rs.ticket = t;
    lds_store_rel(&rs.ready, round + 1);
  }
  return __builtin_amdgcn_readfirstlane(__shfl(t, 0));
}

// Takes the wave's next slot and, if that needs no wait, its round's ticket
// (done); wave_claim_finish completes it otherwise.  A wave may try this
// before releasing its current slot (it waits for nothing), but finishes
// only after the release, so the claim protocol's waits are unchanged.
__device__ __forceinline__ Claim wave_claim_try(const Ctl& C, WaveSched& ws) {
  const uint32_t lane = __lane_id();
  uint32_t k = 0;
  if (lane == 0) k = atomicAdd(&ws.claim, 1u);
  k = __builtin_amdgcn_readfirstlane(__shfl(k, 0));
  Claim c;
  c.round = k / WaveEnc::WAVES;
  c.slot = k % WaveEnc::WAVES;
  c.ticket = 0xFFFFFFFFu;
  c.done = false;
  RoundState& rs = ws.rs[c.round % RING];
  uint32_t ok = 0;
  if (lane == 0)
    ok = c.slot == 0
             ? (lds_load_acq(&rs.released) >= WaveEnc::WAVES &&
                (c.round == 0 || lds_load_acq(&rs.pflag) >= c.round + 1))
             : lds_load_acq(&rs.ready) >= c.round + 1;
  if (__shfl(ok, 0)) {
    c.ticket = c.slot == 0 ? wave_round_open(C, rs, c.round)
                           : __builtin_amdgcn_readfirstlane(rs.ticket);
    c.done = true;
  }
  return c;
}

__device__ __forceinline__ void wave_claim_finish(const Ctl& C, WaveSched& ws, Claim& c) {
  if (c.done) return;
  c.done = true;
  RoundState& rs = ws.rs[c.round % RING];
  if (c.slot == 0) {
    // the entry's previous round has been released by all its claimers, and
    // the round's ticket has been handed on by the previous round
    if (!lds_wait_ge(C, &rs.released, WaveEnc::WAVES) ||
        (c.round > 0 && !lds_wait_ge(C, &rs.pflag, c.round + 1)))
      return;  // timed out: ticket stays past the end
    c.ticket = wave_round_open(C, rs, c.round);
    return;
  }
  if (!lds_wait_ge(C, &rs.ready, c.round + 1)) return;
  c.ticket = __builtin_amdgcn_readfirstlane(rs.ticket);
}

__device__ __forceinline__ Claim wave_claim(const Ctl& C, WaveSched& ws) {
  Claim c = wave_claim_try(C, ws);
  wave_claim_finish(C, ws, c);
  return c;
}

// Hands round r + 1 its ticket (lane 0): a fresh one, or t past the end.
__device__ __forceinline__ void wave_hand_on(const Ctl& C, WaveSched& ws, uint32_t r,
                                             uint32_t t, bool fresh) {
  RoundState& nx = ws.rs[(r + 1) % RING];
  nx.pticket = fresh ? atomicAdd(&C.ctrl->ticket, 1u) : t;
  lds_store_rel(&nx.pflag, r + 2);
}

// The claimer is done with its round's entry.
__device__ __forceinline__ void wave_release(RoundState& rs) {
  if (__lane_id() == 0)
    __hip_atomic_fetch_add(&rs.released, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ __forceinline__ uint32_t round_sum(const RoundState& rs) {
  uint32_t a = 0;
#pragma unroll
  for (uint32_t i = 0; i < WaveEnc::WAVES; ++i) a += rs.size[i];
  return a;
}

// Superblock u (slot cl.slot of round entry rs; u >= J.NS: an empty slot
// past the job's end) of round gs of the chain that starts at chain0:
// encodes it into the wave's region and finds its offset (off, dwords).
// True if the unit is to be written out (wave_write_unit); the caller then
// releases the slot.
template <int L, bool FUSED>
__device__ __forceinline__ bool wave_round_begin(const Job& J, uint64_t u, const Claim& cl,
                                                 WaveSched& ws, uint64_t gs, uint64_t chain0,
                                                 const Ctl& C, uint32_t ep, uint32_t* R,
                                                 const UnitPre& pre, uint32_t (&tot)[2],
                                                 uint64_t& off) {
  RoundState& rs = ws.rs[cl.round % RING];
  const uint32_t lane = __lane_id();
  const bool live = u < J.NS;
  tot[0] = tot[1] = 0u;
  bool good = true;
  // the size into the round; the wave completing the count publishes
  auto pub = [&](uint32_t size) {
    if (lane != 0) return;
    __hip_atomic_store(&rs.size[cl.slot], size, __ATOMIC_RELEASE,
                       __HIP_MEMORY_SCOPE_WORKGROUP);
    const uint32_t c =
        __hip_atomic_fetch_add(&rs.cnt, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_WORKGROUP) + 1;
    if (c == WaveEnc::WAVES) {
      const uint32_t agg = round_sum(rs);
      if (lds_load_acq(&rs.pready) >= cl.round + 1) {
        st_agent(C.status + gs, sw_pack(2, ep, rs.prefix + agg));
      } else {
        publish_agg(C, gs, chain0, ep, agg);
        __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): that store has completed
        if (lds_load_acq(&rs.pready) >= cl.round + 1)
          st_agent(C.status + gs, sw_pack(2, ep, rs.prefix + agg));
      }
    }
  };
  if (live) {
    if ((u + 1) * SUPER <= J.n) wave_encode_unit<L, FUSED, true>(J, u, R, tot, good, pre, pub);
    else wave_encode_unit<L, FUSED, false>(J, u, R, tot, good, pre, pub);
  } else {
    pub(0u);
    return false;
  }
  // the round's prefix: fetched by one wave, read by the others
  uint32_t fetcher = 0;
  if (lane == 0) fetcher = atomicCAS(&rs.fetch, 0u, 1u) == 0u ? 1u : 0u;
  fetcher = __shfl(fetcher, 0);
  bool to = false;
  uint64_t prefix = 0;
  if (fetcher) {
    prefix = lookback<1, false>(C, gs, chain0, ep, 0, to);
    if (lane == 0) {
      rs.prefix = prefix;
      lds_store_rel(&rs.pready, cl.round + 1);
      if (lds_load_acq(&rs.cnt) == WaveEnc::WAVES && !to)
        st_agent(C.status + gs, sw_pack(2, ep, prefix + round_sum(rs)));
      wave_hand_on(C, ws, cl.round, 0, true);
    }
  } else {
    to = !lds_wait_ge(C, &rs.pready, cl.round + 1);
    prefix = rs.prefix;
  }
  // plus the sizes of the round's earlier slots
  uint32_t below = 0;
  if (lane < cl.slot) {
    uint32_t spins = 0;
    uint64_t t0 = 0;
    uint32_t v;
    while ((v = lds_load_acq(&rs.size[lane])) == SIZE_NONE) {
      if (wait_over(C, ++spins, t0)) {
        to = true;
        v = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    below = v;
  }
  to = __ballot(to) != 0;
  below = (uint32_t)wave_sum64(below);
  if (lane == 0) {
    if (to) atomicOr(&C.ctrl->err, ERRF_TIMEOUT);
    if (!good) atomicOr(&C.ctrl->err, ERRF_CORRUPT);
  }
  off = prefix + below;
  return !to && good;
}

#define GZ_WAVE_ATTR __launch_bounds__(WaveEnc::WAVES * 64) __attribute__((amdgpu_waves_per_eu(2, 2)))
// Rounds of a job of NS superblocks.
__device__ __forceinline__ uint64_t rounds_of(uint64_t NS) {
  return (NS + WaveEnc::WAVES - 1) / WaveEnc::WAVES;
}

// One stream: round ticket T covers superblocks WAVES * T + slot, look-back
// word T.
template <int L, bool FUSED>
__global__ GZ_WAVE_ATTR void k_encode_w(Job J, Ctl C) {
  __shared__ WaveSched ws;
  wave_sched_init(ws);
  uint32_t* R = g_stage + (threadIdx.x >> 6) * WaveEnc::REGION;
  const uint32_t ep = ld_agent32(&C.ctrl->epoch);
  const uint64_t NR = rounds_of(J.NS);
  Claim cl = wave_claim(C, ws);
  UnitPre pre;
  pre.valid = false;
  for (;;) {
    RoundState& rs = ws.rs[cl.round % RING];
    if (cl.ticket >= NR) {  // past the end (or timed out)
      if (cl.slot == 0 && __lane_id() == 0) wave_hand_on(C, ws, cl.round, cl.ticket, false);
      wave_release(rs);
      break;
    }
    const uint64_t u = (uint64_t)cl.ticket * WaveEnc::WAVES + cl.slot;
    uint32_t tot[2];
    uint64_t off = 0;
    const bool wr = wave_round_begin<L, FUSED>(J, u, cl, ws, cl.ticket, 0, C, ep, R, pre, tot, off);
    // the next slot, and its first words ahead of this unit's stores
    Claim nx = wave_claim_try(C, ws);
    pre.valid = false;
    if (FUSED && nx.done && nx.ticket < NR) {
      const uint64_t v = (uint64_t)nx.ticket * WaveEnc::WAVES + nx.slot;
      if (v < J.NS) wave_unit_preload<L>(J, v, pre);
    }
    if (wr) wave_write_unit<L>(J, u, off, tot, R);
    wave_release(rs);
    wave_claim_finish(C, ws, nx);
    cl = nx;
  }
  epilogue(C);
}
// njobs streams of NS superblocks each (total = njobs x rounds per job),
// every one its own chain: round ticket T is round T / njobs of job
// T % njobs, look-back word j x rounds + round.
template <int L, bool FUSED>
__global__ GZ_WAVE_ATTR void k_batch_encode_w(const Job* __restrict__ jobs, uint32_t njobs,
                                              uint32_t total, Ctl C) {
  __shared__ WaveSched ws;
  wave_sched_init(ws);
  uint32_t* R = g_stage + (threadIdx.x >> 6) * WaveEnc::REGION;
  const uint32_t ep = ld_agent32(&C.ctrl->epoch);
  Claim cl = wave_claim(C, ws);
  UnitPre pre;
  pre.valid = false;
  for (;;) {
    RoundState& rs = ws.rs[cl.round % RING];
    if (cl.ticket >= total) {  // past the end (or timed out)
      if (cl.slot == 0 && __lane_id() == 0) wave_hand_on(C, ws, cl.round, cl.ticket, false);
      wave_release(rs);
      break;
    }
    const uint32_t j = cl.ticket % njobs;
    const Job J = jobs[j];
    const uint64_t NR = rounds_of(J.NS), r = cl.ticket / njobs;
    const uint64_t u = r * WaveEnc::WAVES + cl.slot;
    uint32_t tot[2];
    uint64_t off = 0;
    const bool wr =
        wave_round_begin<L, FUSED>(J, u, cl, ws, j * NR + r, j * NR, C, ep, R, pre, tot, off);
    // the next slot, and its first words ahead of this unit's stores
    Claim nx = wave_claim_try(C, ws);
    pre.valid = false;
    if (FUSED && nx.done && nx.ticket < total) {
      const Job& K = jobs[nx.ticket % njobs];
      const uint64_t v = (uint64_t)(nx.ticket / njobs) * WaveEnc::WAVES + nx.slot;
      if (v < K.NS) wave_unit_preload<L>(K, v, pre);
    }
    if (wr) wave_write_unit<L>(J, u, off, tot, R);
    wave_release(rs);
    wave_claim_finish(C, ws, nx);
    cl = nx;
  }
  epilogue(C);
}

template <int L, bool FULL>
__device__ __forceinline__ void fused_body(const Job& J, uint64_t s, uint64_t gs, const Ctl& C,
                                           Smem& sm, uint32_t& tk) {
  const uint64_t e0 = (s * blockDim.x + threadIdx.x) * SEG;
  const uint32_t vcnt = FULL ? 32u : (e0 >= J.n ? 0u : (uint32_t)min((uint64_t)SEG, J.n - e0));
  const uint64_t s0 = s * blockDim.x * (uint64_t)SEG;
  float v[32];
  FusedSrc fs;
  const bool ok = decode_strip<float, L, FULL>(J, (const uint8_t*)J.in, J.in_bytes, s, C, sm,
                                               v, vcnt, fs.di);
  fs.pay = (const uint32_t*)((const uint8_t*)J.in + J.pay_off);
  fs.t = sm.t32;
  fs.exists = FULL || (s * blockDim.x + threadIdx.x) / (L / 32) < J.B;
  // The local addend moves through LDS with coalesced loads once the decode
  // is done with the LDS.  (Each lane reading its own 32 values would touch
  // a different 128-byte line in every lane of every load; loading it before
  // the decode holds 32 more registers across it: both measured slower.)
  __syncthreads();  // every lane has read its payload words from LDS
  strip_to_lds<float>(J.local + s0, FULL ? (uint64_t)blockDim.x * SEG : J.n - s0);
  __syncthreads();
  float a[32];
  lane_from_lds<float>(a);
#pragma unroll
  for (int i = 0; i < 32; ++i) v[i] = v[i] + a[i];  // incoming + local, fp32
  lane_to_lds<float>(v);  // the sums, for a RAW block (own segment: no barrier)
  encode_strip<float, L, FULL, true>(J, s, gs, C, sm, v, vcnt, &fs, !ok, tk);
}

template <int L>
__device__ __forceinline__ void fused_one(const Job& J, uint64_t s, uint64_t gs, const Ctl& C,
                                          Smem& sm, uint32_t& tk) {
  if ((s + 1) * blockDim.x * SEG <= J.n) fused_body<L, true>(J, s, gs, C, sm, tk);
  else fused_body<L, false>(J, s, gs, C, sm, tk);
}

// Persistent loop: the next ticket is requested while the current strip is
// processed, so the atomic's latency is hidden.
#define GZ_STRIP_LOOP(TOTAL, BODY)                                      \
  __shared__ Smem sm;                                                   \
  uint32_t t = first_ticket(C, sm);                                     \
  while (t < (TOTAL)) {                                                 \
    uint32_t nxt = 0;                                                   \
    if (threadIdx.x == 0) nxt = atomicAdd(&C.ctrl->ticket, 1u);         \
    BODY;                                                               \
    __syncthreads();                                                    \
    if (threadIdx.x == 0) sm.cur = nxt;                                 \
    __syncthreads();                                                    \
    t = sm.cur;                                                         \
  }                                                                     \
  epilogue(C);

// Persistent loop of the chained (encoding) operations: BODY sets `nxt`
// (in thread 0) to the next ticket right after its strip's look-back; a
// body that never reaches it leaves the exit value.
#define GZ_CHAIN_LOOP(TOTAL, BODY)                                      \
  __shared__ Smem sm;                                                   \
  uint32_t t = first_ticket(C, sm);                                     \
  while (t < (TOTAL)) {                                                 \
    uint32_t nxt = 0xFFFFFFFFu;                                         \
    BODY;                                                               \
    __syncthreads();                                                    \
    if (threadIdx.x == 0) sm.cur = nxt;                                 \
    __syncthreads();                                                    \
    t = sm.cur;                                                         \
  }                                                                     \
  epilogue(C);

// The fused step is built for four waves per SIMD (a few registers spill):
// that fits one 1024-thread workgroup per CU, which measured faster than
// two of 512 or three 256-thread ones without spills.
#define GZ_FUSED_ATTR __launch_bounds__(MAX_TPB) __attribute__((amdgpu_waves_per_eu(4, 8)))
// tile encoding (selector and three predictors) needs more registers
#define GZ_TILE_ATTR __launch_bounds__(MAX_TPB_WIDE) __attribute__((amdgpu_waves_per_eu(3, 8)))

template <typename T, int L>
__global__ __launch_bounds__(sizeof(T) == 4 ? MAX_TPB : MAX_TPB_WIDE)
__attribute__((amdgpu_waves_per_eu(sizeof(T) == 8 ? 3 : 4, 8))) void k_compress(Job J, Ctl C) {
  GZ_CHAIN_LOOP(J.nstrips, (compress_one<T, L>(J, t, t, C, sm, nxt)))
}

template <typename T, int L>
__global__ __launch_bounds__(sizeof(T) == 4 ? MAX_TPB : MAX_TPB_WIDE)
__attribute__((amdgpu_waves_per_eu(4, 8))) void k_decompress(Job J, Ctl C) {
  GZ_STRIP_LOOP(J.nstrips, (decompress_tp_one<T, L>(J, t, C, sm, nxt)))
}

template <int L>
__global__ __launch_bounds__(MAX_TPB) __attribute__((amdgpu_waves_per_eu(4, 8)))
void k_accum(Job J, Ctl C) {
  GZ_STRIP_LOOP(J.nstrips, (accum_one<L>(J, t, C, sm)))
}

template <int L>
__global__ GZ_FUSED_ATTR void k_fused(Job J, Ctl C) {
  GZ_CHAIN_LOOP(J.nstrips, (fused_one<L>(J, t, t, C, sm, nxt)))
}

// Batched: ticket t processes strip strip_job[2t + 1] of job strip_job[2t]
// or, when every job has the same strip count (njobs > 0, jobs interleaved
// round-robin), strip t / njobs of job t % njobs; its look-back word is
// J.strip0 + that strip.  One kernel per operation; WIDE admits fp64 jobs
// (fp32-only batches avoid the register pressure of the fp64 paths).
template <uint32_t OP, bool WIDE>
__device__ __forceinline__ void batch_body(const Job* __restrict__ jobs,
                                           const uint32_t* __restrict__ strip_job, uint32_t njobs,
                                           uint32_t t, const Ctl& C, Smem& sm, uint32_t& tk) {
  const uint32_t j = njobs ? t % njobs : strip_job[2 * (uint64_t)t];
  const uint64_t s = njobs ? t / njobs : strip_job[2 * (uint64_t)t + 1];
  const Job J = jobs[j];
  const uint64_t gs = J.strip0 + s;
  const uint32_t key = (J.dtype << 3) | J.log2L;
  if (OP == 0) {
    switch (key) {
      case 5: compress_one<float, 32>(J, s, gs, C, sm, tk); break;
      case 6: compress_one<float, 64>(J, s, gs, C, sm, tk); break;
      case 7: compress_one<float, 128>(J, s, gs, C, sm, tk); break;
      case 13: if (WIDE) compress_one<double, 32>(J, s, gs, C, sm, tk); break;
      case 14: if (WIDE) compress_one<double, 64>(J, s, gs, C, sm, tk); break;
      case 15: if (WIDE) compress_one<double, 128>(J, s, gs, C, sm, tk); break;
      default: break;
    }
  } else if (OP == 1) {
    switch (key) {
      case 5: decompress_one<float, 32>(J, s, C, sm); break;
      case 6: decompress_one<float, 64>(J, s, C, sm); break;
      case 7: decompress_one<float, 128>(J, s, C, sm); break;
      case 13: if (WIDE) decompress_one<double, 32>(J, s, C, sm); break;
      case 14: if (WIDE) decompress_one<double, 64>(J, s, C, sm); break;
      case 15: if (WIDE) decompress_one<double, 128>(J, s, C, sm); break;
      default: break;
    }
  } else if (OP == 2) {
    switch (key) {
      case 5: fused_one<32>(J, s, gs, C, sm, tk); break;
      case 6: fused_one<64>(J, s, gs, C, sm, tk); break;
      case 7: fused_one<128>(J, s, gs, C, sm, tk); break;
      default: break;
    }
  } else {
    switch (key) {
      case 5: accum_one<32>(J, s, C, sm); break;
      case 6: accum_one<64>(J, s, C, sm); break;
      case 7: accum_one<128>(J, s, C, sm); break;
      default: break;
    }
  }
}

template <uint32_t OP, bool WIDE>
__global__ __launch_bounds__(WIDE ? MAX_TPB_WIDE : MAX_TPB)
__attribute__((amdgpu_waves_per_eu((OP == 0 && WIDE) ? 3 : 4, 8))) void k_batch(const Job* __restrict__ jobs,
                                       const uint32_t* __restrict__ strip_job, uint32_t njobs,
                                       uint32_t total, Ctl C) {
  if constexpr (OP == 1 || OP == 3) {
    GZ_STRIP_LOOP(total, (batch_body<OP, WIDE>(jobs, strip_job, njobs, t, C, sm, nxt)))
  } else {
    GZ_CHAIN_LOOP(total, (batch_body<OP, WIDE>(jobs, strip_job, njobs, t, C, sm, nxt)))
  }
}

// ------------------------------------------------------------ tile mode
// Mode 1 (fp32, 8x8 tiles, L = 64): lane w of tile seg/2 owns its rows
// 4w..4w+3, loaded/stored as 4 rows of 8 floats.
__device__ __forceinline__ void load_tile(const Job& J, const float* __restrict__ p, bool ex,
                                          float (&v)[32]) {
#pragma unroll
  for (int r = 0; r < 4; ++r) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      f4u t = ex ? *(const f4u*)(p + r * (uint64_t)J.nx + 4 * h) : f4u{0, 0, 0, 0};
      v[8 * r + 4 * h] = t.x; v[8 * r + 4 * h + 1] = t.y;
      v[8 * r + 4 * h + 2] = t.z; v[8 * r + 4 * h + 3] = t.w;
    }
  }
}
__device__ __forceinline__ void store_tile(const Job& J, float* __restrict__ p,
                                           const float (&v)[32]) {
#pragma unroll
  for (int r = 0; r < 4; ++r) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      f4u t;
      t.x = v[8 * r + 4 * h]; t.y = v[8 * r + 4 * h + 1];
      t.z = v[8 * r + 4 * h + 2]; t.w = v[8 * r + 4 * h + 3];
      *(f4u*)(p + r * (uint64_t)J.nx + 4 * h) = t;
    }
  }
}

template <bool FULL>
__device__ __forceinline__ void compress_tiles_body(const Job& J, uint64_t s, uint64_t gs,
                                                    const Ctl& C, Smem& sm, uint32_t& tk) {
  const uint64_t seg = s * blockDim.x + threadIdx.x;
  const bool ex = FULL || (seg >> 1) < J.B;
  float v[32];
  load_tile(J, (const float*)J.in + (ex ? seg_first<1>(J, seg) : 0), ex, v);
  LaneCode lc;
  analyze_tile(J, threadIdx.x & 1u, v, ex, sm.wts, lc);
  emit_strip<float, 64, 1, false, FULL>(J, s, gs, C, sm, ex ? 32u : 0u, lc, nullptr, false, tk);
}

__device__ __forceinline__ void load_weights(const Ctl& C, Smem& sm) {
  for (uint32_t k = threadIdx.x; k < 189; k += blockDim.x) sm.wts[k] = ((const uint32_t*)C.blob)[k];
  __syncthreads();
}

__global__ GZ_TILE_ATTR void k_compress_tiles(Job J, Ctl C) {
  __shared__ Smem sm;
  load_weights(C, sm);
  uint32_t t = first_ticket(C, sm);
  while (t < J.nstrips) {
    uint32_t nxt = 0xFFFFFFFFu;  // the next ticket, taken after the look-back
    if ((t + 1) * (uint64_t)blockDim.x <= 2 * J.B) compress_tiles_body<true>(J, t, t, C, sm, nxt);
    else compress_tiles_body<false>(J, t, t, C, sm, nxt);
    __syncthreads();
    if (threadIdx.x == 0) sm.cur = nxt;
    __syncthreads();
    t = sm.cur;
  }
  epilogue(C);
}

__global__ __launch_bounds__(MAX_TPB_WIDE)
__attribute__((amdgpu_waves_per_eu(4, 8))) void k_decompress_tiles(Job J, Ctl C) {
  __shared__ Smem sm;
  uint32_t t = first_ticket(C, sm);
  while (t < J.nstrips) {
    uint32_t nxt = 0;
    if (threadIdx.x == 0) nxt = atomicAdd(&C.ctrl->ticket, 1u);
    const uint64_t seg = t * (uint64_t)blockDim.x + threadIdx.x;
    const bool ex = (seg >> 1) < J.B;
    float v[32];
    DecInfo di;
    if (decode_strip<float, 64, false, 1>(J, (const uint8_t*)J.in, J.in_bytes, t, C, sm, v,
                                          ex ? 32u : 0u, di) && ex)
      store_tile(J, (float*)J.out + seg_first<1>(J, seg), v);
    __syncthreads();
    if (threadIdx.x == 0) sm.cur = nxt;
    __syncthreads();
    t = sm.cur;
  }
  epilogue(C);
}

// Training data of the selector: per tile the 16 features, the sizes of the
// three encodings and the exhaustive-trial label (255: RAW or ZERO tile).
__global__ __launch_bounds__(256) void k_tile_trial(Job J, int8_t* __restrict__ feat,
                                                   uint32_t* __restrict__ sizes,
                                                   uint8_t* __restrict__ label) {
  const uint64_t nseg = 2 * J.B;
  for (uint64_t seg = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
       seg - threadIdx.x < nseg; seg += (uint64_t)gridDim.x * blockDim.x) {
    // whole waves iterate together (the tile's two lanes shuffle)
    const bool ex = seg < nseg;
    const uint32_t w = threadIdx.x & 1u;
    float v[32];
    load_tile(J, (const float*)J.in + (ex ? seg_first<1>(J, seg) : 0), ex, v);
    int32_t q[32];
    bool bad;
    tile_quant(J, v, q, bad);
    int32_t up[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) up[c] = __shfl_up(q[24 + c], 1);
    uint32_t f[4];
    tile_features(q, w, f);
    const uint32_t o0 = tile_or<0>(q, up, w), o1 = tile_or<1>(q, up, w), o2 = tile_or<2>(q, up, w);
    const uint32_t s0 = size_of(K_NONE, o0 ? 32u - __clz(o0) : 0u);
    const uint32_t s1 = size_of(K_L1D, o1 ? 32u - __clz(o1) : 0u);
    const uint32_t s2 = size_of(K_L2D, o2 ? 32u - __clz(o2) : 0u);
    uint32_t best = 0, bs = s0;
    if (s1 < bs) { best = 1; bs = s1; }
    if (s2 < bs) best = 2;
    const bool zero = (grp_or<2>(q[0] != 0 ? 1u : 0u) | o0) == 0;
    if (ex && w == 0) {
      const uint64_t b = seg >> 1;
      ((uint32_t*)feat)[4 * b + 0] = f[0];
      ((uint32_t*)feat)[4 * b + 1] = f[1];
      ((uint32_t*)feat)[4 * b + 2] = f[2];
      ((uint32_t*)feat)[4 * b + 3] = f[3];
      sizes[3 * b + 0] = 4 * s0;
      sizes[3 * b + 1] = 4 * s1;
      sizes[3 * b + 2] = 4 * s2;
      label[b] = (bad || zero) ? 255 : (uint8_t)best;
    }
  }
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

// Reports the sticky device status of a launch (GZ_OK 0, GZ_ECORRUPT 3,
// GZ_ETIMEOUT 7) into *out (when given) and clears it, so that the next
// launch on the same workspace starts clean.
__global__ void k_finish(Ctl C, uint32_t* out) {
  if (threadIdx.x == 0) {
    const uint32_t e = ld_agent32(&C.ctrl->err);
    if (out) *out = (e & ERRF_CORRUPT) ? 3u : (e & ERRF_TIMEOUT) ? 7u : 0u;
    if (e) atomicAnd(&C.ctrl->err, 0u);
  }
}

// ------------------------------------------------------------ launchers
// Dynamic LDS: the strip staging buffer (largest strip payload + headroom).
static size_t stage_bytes(uint32_t dtype, uint32_t tpb) {
  return 32 + (size_t)tpb * (SEG * (dtype == 0 ? 1 : 2) + 4) * 4;  // padded segment layout
}

size_t lds_bytes(uint32_t wide, uint32_t tpb) { return stage_bytes(wide, tpb) + sizeof(Smem); }

template <typename T, int L>
static hipError_t launch_c(const Job& J, const Ctl& C, uint32_t tpb, uint32_t grid,
                           hipStream_t st) {
  hipLaunchKernelGGL((k_compress<T, L>), dim3(grid), dim3(tpb), stage_bytes(J.dtype, tpb), st, J,
                     C);
  return hipGetLastError();
}
template <typename T, int L>
static hipError_t launch_d(const Job& J, const Ctl& C, uint32_t tpb, uint32_t grid,
                           hipStream_t st) {
  hipLaunchKernelGGL((k_decompress<T, L>), dim3(grid), dim3(tpb), stage_bytes(J.dtype, tpb), st,
                     J, C);
  return hipGetLastError();
}
template <typename T, int L>
static hipError_t launch_dw(const Job& J, const Ctl& C, uint32_t grid, hipStream_t st) {
  const size_t lds = (size_t)WaveDec<T>::WAVES * WaveDec<T>::REGION * 4;
  hipLaunchKernelGGL((k_decompress_w<T, L>), dim3(grid), dim3(WaveDec<T>::WAVES * 64), lds, st, J,
                     C);
  return hipGetLastError();
}

hipError_t launch_decompress_wave(const Job& J, const Ctl& C, uint32_t cus, hipStream_t st) {
  const uint32_t waves = J.dtype == 0 ? WaveDec<float>::WAVES : WaveDec<double>::WAVES;
  const uint64_t need = (J.NS + waves - 1) / waves;
  const uint32_t grid = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(cus, need));
  switch ((J.dtype << 3) | J.log2L) {
    case 5: return launch_dw<float, 32>(J, C, grid, st);
    case 6: return launch_dw<float, 64>(J, C, grid, st);
    case 7: return launch_dw<float, 128>(J, C, grid, st);
    case 13: return launch_dw<double, 32>(J, C, grid, st);
    case 14: return launch_dw<double, 64>(J, C, grid, st);
    case 15: return launch_dw<double, 128>(J, C, grid, st);
  }
  return hipErrorInvalidValue;
}

size_t wave_encode_lds() {
  return (size_t)WaveEnc::WAVES * WaveEnc::REGION * 4 + sizeof(WaveSched);
}

template <int L, bool FUSED>
static hipError_t launch_ew(const Job* d_jobs, const Job& J, uint32_t njobs, uint32_t total,
                            const Ctl& C, uint32_t cus, hipStream_t st) {
  // one workgroup per round in flight, at most one per CU (the LDS allows one)
  const uint32_t grid = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(cus, total));
  const size_t lds = (size_t)WaveEnc::WAVES * WaveEnc::REGION * 4;
  if (d_jobs)
    hipLaunchKernelGGL((k_batch_encode_w<L, FUSED>), dim3(grid), dim3(WaveEnc::WAVES * 64), lds,
                       st, d_jobs, njobs, total, C);
  else
    hipLaunchKernelGGL((k_encode_w<L, FUSED>), dim3(grid), dim3(WaveEnc::WAVES * 64), lds, st,
                       J, C);
  return hipGetLastError();
}

hipError_t launch_encode_wave(uint32_t op, const Job* d_jobs, const Job& J, uint32_t njobs,
                              uint32_t total, uint32_t log2L, const Ctl& C, uint32_t cus,
                              hipStream_t st) {
  const bool fused = op == 2;
  switch (log2L) {
    case 5: return fused ? launch_ew<32, true>(d_jobs, J, njobs, total, C, cus, st)
                         : launch_ew<32, false>(d_jobs, J, njobs, total, C, cus, st);
    case 6: return fused ? launch_ew<64, true>(d_jobs, J, njobs, total, C, cus, st)
                         : launch_ew<64, false>(d_jobs, J, njobs, total, C, cus, st);
    case 7: return fused ? launch_ew<128, true>(d_jobs, J, njobs, total, C, cus, st)
                         : launch_ew<128, false>(d_jobs, J, njobs, total, C, cus, st);
  }
  return hipErrorInvalidValue;
}

template <int L>
static hipError_t launch_aw(const Job& J, const Ctl& C, uint32_t grid, hipStream_t st) {
  const size_t lds = (size_t)WaveDec<float>::WAVES * WaveDec<float>::REGION * 4;
  hipLaunchKernelGGL((k_accum_w<L>), dim3(grid), dim3(WaveDec<float>::WAVES * 64), lds, st, J, C);
  return hipGetLastError();
}

hipError_t launch_accum_wave(const Job& J, const Ctl& C, uint32_t cus, hipStream_t st) {
  const uint64_t need = (J.NS + WaveDec<float>::WAVES - 1) / WaveDec<float>::WAVES;
  const uint32_t grid = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(cus, need));
  switch (J.log2L) {
    case 5: return launch_aw<32>(J, C, grid, st);
    case 6: return launch_aw<64>(J, C, grid, st);
    case 7: return launch_aw<128>(J, C, grid, st);
  }
  return hipErrorInvalidValue;
}

template <bool WIDE, uint32_t OP>
static hipError_t launch_bdw(const Job* d_jobs, const uint32_t* d_map, uint32_t njobs,
                             uint32_t total, uint32_t jw, uint32_t cus, const Ctl& C,
                             hipStream_t st) {
  constexpr uint32_t WAVES = WIDE ? WaveDec<double>::WAVES : WaveDec<float>::WAVES;
  const size_t lds = (size_t)WAVES * (WIDE ? WaveDec<double>::REGION : WaveDec<float>::REGION) * 4;
  const uint64_t need = ((uint64_t)(jw ? jw : total) + WAVES - 1) / WAVES;
  const uint32_t grid = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(cus, need));
  hipLaunchKernelGGL((k_batch_decode_w<WIDE, OP>), dim3(grid), dim3(WAVES * 64), lds, st, d_jobs,
                     d_map, njobs, total, jw, C);
  return hipGetLastError();
}

hipError_t launch_decode_wave_batch(uint32_t op, const Job* d_jobs, const uint32_t* d_map,
                                    uint32_t njobs, uint32_t total, bool wide, uint32_t jw,
                                    uint32_t cus, const Ctl& C, hipStream_t st) {
  if (op == 1)
    return wide ? launch_bdw<true, 1>(d_jobs, d_map, njobs, total, 0, cus, C, st)
                : launch_bdw<false, 1>(d_jobs, d_map, njobs, total, jw, cus, C, st);
  if (op == 3 && !wide) return launch_bdw<false, 3>(d_jobs, d_map, njobs, total, 0, cus, C, st);
  return hipErrorInvalidValue;
}

size_t wave_decode_lds(uint32_t dtype) {
  return dtype == 0 ? (size_t)WaveDec<float>::WAVES * WaveDec<float>::REGION * 4
                    : (size_t)WaveDec<double>::WAVES * WaveDec<double>::REGION * 4;
}

template <int L>
static hipError_t launch_a(const Job& J, const Ctl& C, uint32_t tpb, uint32_t grid,
                           hipStream_t st) {
  hipLaunchKernelGGL((k_accum<L>), dim3(grid), dim3(tpb), stage_bytes(0, tpb), st, J, C);
  return hipGetLastError();
}
template <int L>
static hipError_t launch_f(const Job& J, const Ctl& C, uint32_t tpb, uint32_t grid,
                           hipStream_t st) {
  hipLaunchKernelGGL((k_fused<L>), dim3(grid), dim3(tpb), stage_bytes(0, tpb), st, J, C);
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
  } else if (op == 3) {
    switch (key) {
      case 5: return launch_a<32>(J, C, tpb, grid, st);
      case 6: return launch_a<64>(J, C, tpb, grid, st);
      case 7: return launch_a<128>(J, C, tpb, grid, st);
    }
  }
  return hipErrorInvalidValue;
}

static const void* batch_kernel(uint32_t op, bool wide) {
  switch (op * 2 + (wide ? 1 : 0)) {
    case 0: return (const void*)k_batch<0, false>;
    case 1: return (const void*)k_batch<0, true>;
    case 2: return (const void*)k_batch<1, false>;
    case 3: return (const void*)k_batch<1, true>;
    case 4: return (const void*)k_batch<2, false>;
    default: return (const void*)k_batch<3, false>;
  }
}

hipError_t launch_batch(uint32_t op, const Job* d_jobs, const uint32_t* d_strip_job,
                        uint32_t njobs, uint32_t total, const Ctl& C, uint32_t tpb, uint32_t grid, bool wide,
                        hipStream_t st) {
  const size_t lds = stage_bytes(wide ? 1 : 0, tpb);
  if (op == 0 && !wide)
    hipLaunchKernelGGL((k_batch<0, false>), dim3(grid), dim3(tpb), lds, st, d_jobs, d_strip_job,
                       njobs, total, C);
  else if (op == 0)
    hipLaunchKernelGGL((k_batch<0, true>), dim3(grid), dim3(tpb), lds, st, d_jobs, d_strip_job,
                       njobs, total, C);
  else if (op == 1 && !wide)
    hipLaunchKernelGGL((k_batch<1, false>), dim3(grid), dim3(tpb), lds, st, d_jobs, d_strip_job,
                       njobs, total, C);
  else if (op == 1)
    hipLaunchKernelGGL((k_batch<1, true>), dim3(grid), dim3(tpb), lds, st, d_jobs, d_strip_job,
                       njobs, total, C);
  else if (op == 2)
    hipLaunchKernelGGL((k_batch<2, false>), dim3(grid), dim3(tpb), lds, st, d_jobs, d_strip_job,
                       njobs, total, C);
  else if (op == 3 && !wide)
    hipLaunchKernelGGL((k_batch<3, false>), dim3(grid), dim3(tpb), lds, st, d_jobs, d_strip_job,
                       njobs, total, C);
  else
    return hipErrorInvalidValue;
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

hipError_t launch_tiles(uint32_t op, const Job& J, const Ctl& C, uint32_t tpb, uint32_t grid,
                        hipStream_t st) {
  if (op == 0)
    hipLaunchKernelGGL(k_compress_tiles, dim3(grid), dim3(tpb), stage_bytes(0, tpb), st, J, C);
  else
    hipLaunchKernelGGL(k_decompress_tiles, dim3(grid), dim3(tpb), stage_bytes(0, tpb), st, J, C);
  return hipGetLastError();
}

hipError_t launch_tile_trial(const Job& J, int8_t* feat, uint32_t* sizes, uint8_t* label,
                             hipStream_t st) {
  // every tile is read from J.in and written to the three outputs
  if (J.B && (!J.in || !feat || !sizes || !label || J.nx == 0 || J.nx % 8 != 0 ||
              J.n != 64 * J.B || J.n % (8ull * J.nx) != 0))
    return hipErrorInvalidValue;
  const uint64_t segs = 2 * J.B;
  uint64_t blocks = (segs + 255) / 256;
  const uint32_t grid = (uint32_t)(blocks < 8192 ? (blocks ? blocks : 1) : 8192);
  hipLaunchKernelGGL(k_tile_trial, dim3(grid), dim3(256), 0, st, J, feat, sizes, label);
  return hipGetLastError();
}

hipError_t launch_finish(const Ctl& C, uint32_t* status, hipStream_t st) {
  hipLaunchKernelGGL(k_finish, dim3(1), dim3(64), 0, st, C, status);
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
  } else if (op == OCC_TILE_C) {
    f = (const void*)k_compress_tiles;
  } else if (op == OCC_TILE_D) {
    f = (const void*)k_decompress_tiles;
  } else if (op == OCC_ACCUM) {
    switch (log2L) {
      case 5: f = (const void*)k_accum<32>; break;
      case 6: f = (const void*)k_accum<64>; break;
      case 7: f = (const void*)k_accum<128>; break;
    }
  } else {
    f = batch_kernel(op - OCC_BATCH, dtype != 0);  // batched op (op - OCC_BATCH)
  }
  if (!f) return 1;
  const bool f32_only = op == 2 || op >= OCC_BATCH + 2;  // fused, accumulate, tiles
  const size_t lds = stage_bytes(f32_only ? 0 : dtype, tpb);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, f, (int)tpb, lds) != hipSuccess || nb < 1)
    nb = 1;
  return nb;
}

}  // namespace gzk
