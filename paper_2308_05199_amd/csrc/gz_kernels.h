// gz_kernels.h -- launchers exported by gz_kernels.hip to the host runtime.
#pragma once
#include <hip/hip_runtime.h>

#include "gz_common.h"

namespace gzk {

// op: 0 compress, 1 decompress, 2 fused step, 3 decode-and-accumulate (2, 3:
// fp32 only)
hipError_t launch_single(uint32_t op, const Job& J, const Ctl& C, uint32_t tpb, uint32_t grid,
                         hipStream_t st);
// LDS one workgroup of tpb threads uses (wide: fp64 strips)
size_t lds_bytes(uint32_t wide, uint32_t tpb);
// op: as launch_single.  wide: the batch holds fp64 jobs (larger LDS staging).  d_strip_job: total
// (job, strip) pairs in ticket order, unused when njobs > 0 (njobs jobs of
// equal strip counts, interleaved round-robin).
hipError_t launch_batch(uint32_t op, const Job* d_jobs, const uint32_t* d_strip_job,
                        uint32_t njobs, uint32_t total, const Ctl& C, uint32_t tpb,
                        uint32_t grid, bool wide, hipStream_t st);
// Per-wave decoding of one stream (mode 0): every wave decodes whole
// superblocks, assigned statically; grid = min(CUs, superblocks per wave).
hipError_t launch_decompress_wave(const Job& J, const Ctl& C, uint32_t cus, hipStream_t st);
size_t wave_decode_lds(uint32_t dtype);  // its workgroup's LDS bytes
// Per-wave decode-and-accumulate of one fp32 stream (as launch_decompress_wave).
hipError_t launch_accum_wave(const Job& J, const Ctl& C, uint32_t cus, hipStream_t st);
// Per-wave batched decoding (op 1) or decode-and-accumulate (op 3, fp32):
// total superblocks, superblock i = (d_map[2i], d_map[2i+1]) as (job,
// superblock), or without a map (jobs of equal superblock counts) superblock
// i / njobs of job i % njobs.  wide: the batch holds fp64 jobs.  jw (op 1,
// fp32 1D jobs): d_map holds jw (job, first superblock, stride) triples,
// one per wave's share of a job (each job's whole superblocks decoded as a
// pipeline); 0 otherwise.
hipError_t launch_decode_wave_batch(uint32_t op, const Job* d_jobs, const uint32_t* d_map,
                                    uint32_t njobs, uint32_t total, bool wide, uint32_t jw,
                                    uint32_t cus, const Ctl& C, hipStream_t st);
// Per-wave fp32 1D encoding (op 0) or fused step (op 2): every wave encodes
// whole superblocks, a workgroup's waves the 8 of a round (one chain
// element).  d_jobs null: the one job J, total = rounds_of(J.NS); else njobs
// jobs of the same superblock count and block length 2^log2L in device
// memory, total = njobs * rounds_of(NS), round ticket t = round t / njobs
// of job t % njobs.
hipError_t launch_encode_wave(uint32_t op, const Job* d_jobs, const Job& J, uint32_t njobs,
                              uint32_t total, uint32_t log2L, const Ctl& C, uint32_t cus,
                              hipStream_t st);
size_t wave_encode_lds();  // its workgroup's LDS bytes
constexpr uint64_t WAVE_ROUND = 8;  // superblocks per round of the per-wave encoder
constexpr uint64_t DEC_WAVES_F32 = 8;  // waves per workgroup of the fp32 per-wave decoders
inline uint64_t wave_rounds(uint64_t NS) { return (NS + WAVE_ROUND - 1) / WAVE_ROUND; }
hipError_t launch_quantize(const void* x, uint64_t n, const Job& J, int32_t* q, uint8_t* fail,
                           hipStream_t st);
// mode 1 (8x8 tiles, fp32): op 0 compress, 1 decompress
hipError_t launch_tiles(uint32_t op, const Job& J, const Ctl& C, uint32_t tpb, uint32_t grid,
                        hipStream_t st);
hipError_t launch_tile_trial(const Job& J, int8_t* feat, uint32_t* sizes, uint8_t* label,
                             hipStream_t st);
hipError_t launch_reset(const Ctl& C, hipStream_t st);
// writes the sticky device status (a gz_status code) to *status, if given,
// and clears it
hipError_t launch_finish(const Ctl& C, uint32_t* status, hipStream_t st);
// Kernels of occupancy_blocks: ops 0-2 as launch_single, OCC_BATCH + k = batched
// op k (dtype 1: a batch with fp64), tile compress/decompress, single-stream
// decode-and-accumulate.
enum : uint32_t { OCC_BATCH = 3, OCC_TILE_C = 7, OCC_TILE_D = 8, OCC_ACCUM = 9 };
// resident workgroups per CU of a kernel
int occupancy_blocks(uint32_t op, uint32_t dtype, uint32_t log2L, uint32_t tpb);

}  // namespace gzk
