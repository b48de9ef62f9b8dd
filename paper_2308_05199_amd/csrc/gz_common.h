// gz_common.h -- types shared by the HIP kernels and the host runtime.
#pragma once
#include <stdint.h>

namespace gzk {

constexpr uint32_t SEG = 32;      // elements per lane segment
constexpr uint32_t SUPER = 4096;  // elements per superblock (one table entry)
constexpr uint32_t HDR = 64;      // stream header bytes
// Largest workgroup the kernels are built for: fp32 1D kernels take
// 1024-thread strips (32768 elements), fp64 and tile kernels 512.
constexpr uint32_t MAX_TPB = 1024;
constexpr uint32_t MAX_TPB_WIDE = 512;

enum : uint32_t { K_ZERO = 0, K_L1D = 1, K_NONE = 2, K_L2D = 3, K_RAW = 7 };
enum : uint32_t { ERRF_CORRUPT = 1u, ERRF_TIMEOUT = 2u };

// Per-context control block (device).  ticket/done drive the persistent
// workgroup loop; epoch tags look-back words so that they never need
// clearing; err is the sticky device status.
struct Ctrl {
  uint32_t ticket;
  uint32_t done;
  uint32_t epoch;
  uint32_t err;
  uint32_t pad[60];
};

// Device code sees the job's buffers as global-address-space pointers: a
// generic pointer read from memory (a batch's job table) would make every
// access through it a flat instruction, which waits on the LDS counter too
// and is ordered against LDS accesses.  The layout is the same on the host.
#if defined(__HIP_DEVICE_COMPILE__)
#define GZ_GLOBAL __attribute__((address_space(1)))
#else
#define GZ_GLOBAL
#endif

// Host code stores plain device pointers into a Job through this cast.
template <typename T>
inline GZ_GLOBAL T* job_ptr(T* p) {
  return (GZ_GLOBAL T*)p;
}

// One independent stream to encode, decode or fuse.  Geometry fields
// describe the stream written (encode/fused) or expected (decode).
struct Job {
  GZ_GLOBAL const void* in;                   // T[n] | stream
  GZ_GLOBAL const float* local;               // fused addend
  GZ_GLOBAL void* out;                        // stream | T[n]
  GZ_GLOBAL unsigned long long* out_bytes;    // encode: size of the stream written
  GZ_GLOBAL unsigned long long* chunk_off;    // scatter: offset of this stream
  GZ_GLOBAL const unsigned long long* in_off; // scatter decode: offset of this stream in `in`
  uint64_t n;
  uint64_t in_bytes;                // decode/fused: bytes readable at `in`
  uint64_t strip0;                  // first global strip of this job
  uint64_t chain0;                  // first global strip of its look-back chain
  uint64_t fixed_off;               // packed output: fixed bytes of earlier streams
  uint64_t NS, B, hdr_off, pay_off; // stream geometry
  double eb;
  double rinv;                      // 1 / (double)t32
  double t64;                       // fp64 step
  float t32;                        // fp32 step
  float eblo;                       // largest float <= eb
  uint32_t dtype, log2L, mode, nx, select, nstrips, job, pad;
};

struct Ctl {
  Ctrl* ctrl;
  unsigned long long* status;   // one look-back word per global strip
  unsigned long long* jobbase;  // one word per job of a packed chain
  const uint8_t* blob;          // selector weights
  uint64_t wait_ticks;          // longest inter-workgroup wait (constant-rate clock ticks)
};

}  // namespace gzk
