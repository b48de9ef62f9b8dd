/*
 * gzccl.h -- C ABI of the MI355X (gfx950) compression hot path of gZCCL
 * (arXiv 2308.05199): error-bounded compression, decompression, the fused
 * decompress -> reduce -> recompress step of a ring Reduce_scatter, Scatter
 * compression, batched launches and the learned predictor selector.
 *
 * Conventions (every call):
 *   - Data pointers named d_* are device pointers owned by the caller; h_*
 *     are host pointers read during the call only.
 *   - Calls only enqueue work on `stream` and return; no call synchronises
 *     the host, except gz_ctx_create, gz_ctx_status, gz_plan_create,
 *     gz_graph_create, gz_selector_load and the tuners, which say so.  Compressed sizes land in
 *     caller-provided device words; read them after the stream completes
 *     (the paper syncs the streams before reading the sizes, Sec. 3.3.4).
 *   - The context owns all temporary device memory: a workspace allocated
 *     once at gz_ctx_create (the paper's pre-allocated GPU buffer pool,
 *     Sec. 3.3.1, and its reused temporary buffers, Sec. 3.3.2), including
 *     the arena that holds plan descriptors.  No other call allocates device
 *     memory.  One context serves one stream at a time;
 *     contexts share nothing, so several contexts may run concurrently on
 *     different streams (the per-stream buffers of Sec. 3.3.4).
 *   - Argument errors found on the host return at once and enqueue nothing.
 *     Errors found on the device (corrupt stream, look-back time-out) set a
 *     sticky word in the context, read and cleared by gz_ctx_status; the
 *     kernels never write out of bounds, but outputs of a failed call are
 *     unspecified.  No exception or abort crosses the ABI.
 *   - Output bytes depend only on (input, n, dtype, eb, block length, mode,
 *     nx, selector weights); thread counts, grid sizes, streams and batching
 *     never change them.
 *
 * Stream format GZ1 (little-endian):
 *   t = (T)(2*eb).  Per element: r = x/t in T; FAIL if x is not finite or
 *   |r| > 2^29-1; q = rint(r) (ties to even); xh = (T)q*t; FAIL unless
 *   |x - xh| <= eb.  Blocks of L elements (mode 0) or 8x8 tiles of an
 *   nx-wide field (mode 1, L = 64).  Residuals: L1D (d0 = 0 with the first q
 *   stored as a base, then q_i - q_{i-1}; in mode 1 along rows, the first
 *   column vertically), L2D (mode 1: second-order 2D Lorenzo), NONE (mode 1:
 *   d = q).  F = bit length of max|d|.  A block is RAW (values bit for bit)
 *   if an element FAILs or RAW is smaller, ZERO if all q are 0.  Payload:
 *   [int32 base][sign plane][F magnitude planes], a plane being L/32 u32.
 *   Stream = 64-byte header | u32 offset/4 of every 4096-element superblock
 *   | one header byte (kind<<5 | F) per block, padded to 4 | payload.
 *   Header: "GZC1", u16 version 1, u8 dtype, u8 log2 L, u64 n, f64 eb,
 *   u64 payload bytes, u32 mode, u32 nx, u32 4096, 20 zero bytes.
 */
#ifndef GZCCL_H
#define GZCCL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t* gz_stream_t; /* same type as hipStream_t */

typedef enum {
  GZ_OK = 0,
  GZ_EINVAL = 1,       /* bad argument (null pointer, eb, sizes, params) */
  GZ_ENOSPC = 2,       /* output capacity below the bound / workspace too small */
  GZ_ECORRUPT = 3,     /* device: malformed or mismatching input stream */
  GZ_EHIP = 4,         /* a HIP runtime call failed */
  GZ_ENOMEM = 5,       /* allocation failed (context or plan creation only) */
  GZ_EUNSUPPORTED = 6, /* combination not built (e.g. fused step on fp64) */
  GZ_ETIMEOUT = 7      /* device: bounded look-back wait expired */
} gz_status;

typedef enum { GZ_F32 = 0, GZ_F64 = 1 } gz_dtype;

typedef struct gz_ctx gz_ctx;
typedef struct gz_plan gz_plan;
typedef struct gz_graph gz_graph;

/* Encoding parameters.  block_len 32|64|128 (0 = 32); threads per workgroup
 * 128|256|512|1024 (0 = tuned/default; 1024 is built for fp32 1D work only, and
 * it or a size whose LDS staging exceeds the device's per-workgroup limit gives
 * GZ_EUNSUPPORTED) and grid (persistent workgroups, 0 = default) never change
 * the bytes.  threads 64 selects the per-wave kernels, in which each wave
 * codes whole 4096-element superblocks on its own (grid ignored): 1D
 * decompression of either type (also batched and scatter), fp32 1D
 * compression, the fused step and decode-and-accumulate; GZ_EUNSUPPORTED
 * elsewhere.  With no shape given or tuned, decompression (single and
 * batched; scatter decompression of fp32 chunks) and the fused step take
 * them; compression, decode-and-accumulate and fp64 scatter decompression
 * take strips.  mode 0 = 1D blocks, 1 = 8x8 tiles (block_len 64,
 * nx = row length, multiple of 8, n a multiple of 8*nx); select (mode 1):
 * 0 = int8 MLP selector, 1 = exhaustive trial, 2 = always L1D. */
typedef struct {
  uint32_t block_len;
  uint32_t threads;
  uint32_t grid;
  uint32_t mode;
  uint32_t select;
  uint32_t nx;
} gz_params;

/* One independent request of a batch (mode 0).  block_len 0 takes the
 * context's tuned block length for the dtype (set by gz_tune with
 * block_len 0; 32 before any tuning).  Compression: in = T[n],
 * out = stream buffer of out_cap bytes, d_out_bytes receives its size.
 * Decompression: in = stream of in_bytes, out = T[n] (n and dtype and
 * block_len are what the stream must declare).  Fused step: in = fp32
 * stream of n elements, local = fp32[n] addend, out/out_cap/d_out_bytes as
 * for compression.  Accumulate: in = fp32 stream of in_bytes, out = fp32[n]
 * accumulator updated in place (see gz_decompress_add). */
typedef struct {
  const void* in;
  const float* local;
  void* out;
  uint64_t* d_out_bytes;
  uint64_t n;
  uint64_t in_bytes;
  uint64_t out_cap;
  double eb;
  uint32_t dtype;
  uint32_t block_len;
} gz_request;

typedef enum {
  GZ_OP_COMPRESS = 0,
  GZ_OP_DECOMPRESS = 1,
  GZ_OP_FUSED = 2,
  GZ_OP_ACCUMULATE = 3
} gz_op;

/* Creates a context on `device` whose workspace covers calls of up to
 * max_elems elements in total and max_requests requests per batch.
 * Synchronous.  Sec. 3.3.1 (buffer pool allocated once at initialisation,
 * size set by the user). */
gz_status gz_ctx_create(gz_ctx** ctx, int device, uint64_t max_elems,
                        uint32_t max_requests);
void gz_ctx_destroy(gz_ctx* ctx);

/* Waits for `stream` (the stream the context's work was enqueued on; other
 * streams are not waited for), returns the sticky device status (GZ_OK,
 * GZ_ECORRUPT or GZ_ETIMEOUT) in *device_status and clears it.  The paper
 * reads compressed sizes after such a stream sync (Sec. 3.3.4). */
gz_status gz_ctx_status(gz_ctx* ctx, gz_stream_t stream, gz_status* device_status);

/* Clears the context's look-back and ticket state (after a device error). */
gz_status gz_ctx_reset(gz_ctx* ctx, gz_stream_t stream);

/* Bound of every wait between workgroups or waves of one launch (the
 * look-back of Sec. 3.3.4's offset scan, the per-wave encoder's rounds), in
 * microseconds of the device's constant-rate clock; default one second.  A
 * wait that expires sets GZ_ETIMEOUT in the device status (the stream being
 * written is then invalid) and its kernel finishes instead of waiting on.
 * 0 is allowed: a test of that path.  Plans read the bound at each launch;
 * a captured graph keeps the one it was captured with.  Host only. */
gz_status gz_ctx_set_wait(gz_ctx* ctx, uint64_t usec);

/* Largest stream a compression of n elements can produce:
 * 64 + 4*ceil(n/4096) + roundup4(ceil(n/L)) + n*sizeof(T); 0 for an invalid
 * dtype or block length.  Compressed sizes are known only after the kernel
 * has run (Sec. 3.3.4 reads them after a stream sync), so output buffers --
 * the paper's pre-allocated device buffers (Sec. 3.3.1) -- are sized by
 * this bound in advance; with it, capacity errors are host-side. */
uint64_t gz_compress_bound(uint64_t n, gz_dtype dtype, uint32_t block_len);

/* Elementwise quantisation (the q and FAIL steps above) into d_q (int32,
 * 0 where failed) and d_fail (uint8 0/1).  Exposes the first step of the
 * compressor for verification. */
gz_status gz_quantize(gz_ctx* ctx, const void* d_in, uint64_t n, gz_dtype dtype,
                      double eb, int32_t* d_q, uint8_t* d_fail,
                      gz_stream_t stream);

/* Compresses d_in[0..n) under absolute bound eb (Sec. 4.1: absolute error
 * bound) into d_out (out_cap >= gz_compress_bound); the stream size goes to
 * *d_out_bytes.  One launch; block offsets come from a single-pass
 * decoupled look-back scan (Sec. 3.3.2: offsets kept on the device, no
 * unified memory). */
gz_status gz_compress(gz_ctx* ctx, const void* d_in, uint64_t n, gz_dtype dtype,
                      double eb, const gz_params* p, void* d_out,
                      uint64_t out_cap, uint64_t* d_out_bytes,
                      gz_stream_t stream);

/* Decompresses a stream of in_bytes into d_out[0..n) (caller-owned device
 * memory, n elements of dtype): the decompression each rank runs on the
 * data it receives (Sec. 3.3.3: N-1 decompressions in a ring Allreduce's
 * Allgather stage; Sec. 3.2.2 characterises it with compression).  The
 * caller states what it expects (n, dtype, block length, mode, nx); a
 * stream that says otherwise, or is malformed, sets GZ_ECORRUPT on the
 * device and leaves d_out unspecified; the kernel never reads past in_bytes
 * nor writes past n elements.  Overlapping input and output, null pointers
 * or bad params return GZ_EINVAL with nothing enqueued. */
gz_status gz_decompress(gz_ctx* ctx, const void* d_in, uint64_t in_bytes,
                        uint64_t n, gz_dtype dtype, const gz_params* p,
                        void* d_out, gz_stream_t stream);

/* One round of a compressed ring Reduce_scatter for one rank (Sec. 3.2.3):
 * decode the incoming fp32 stream (its own eb), add d_local in fp32 in the
 * order incoming + local, and encode the sum under eb into d_cmp_out, in
 * one kernel that never writes the sum to memory. */
gz_status gz_fused_reduce_step(gz_ctx* ctx, const void* d_cmp_in,
                               uint64_t in_bytes, const float* d_local,
                               uint64_t n, double eb, const gz_params* p,
                               void* d_cmp_out, uint64_t out_cap,
                               uint64_t* d_out_bytes, gz_stream_t stream);

/* The reduction after a receive in recursive-doubling gZ-Allreduce (Sec.
 * 3.3.4): decode the fp32 stream of in_bytes (n elements, block length and
 * mode 0 as in p) and add it into d_acc in place, d_acc[i] = fl32(decoded[i]
 * + d_acc[i]), in one kernel that never writes the decoded values.  d_acc
 * (caller-owned device memory, n floats) must not overlap the stream.  A
 * malformed or mismatching stream leaves d_acc unchanged and sets
 * GZ_ECORRUPT on the device; argument errors return GZ_EINVAL with nothing
 * enqueued; tile mode is GZ_EINVAL. */
gz_status gz_decompress_add(gz_ctx* ctx, const void* d_in, uint64_t in_bytes,
                            uint64_t n, const gz_params* p, float* d_acc,
                            gz_stream_t stream);

/* gZ-Scatter compression (Sec. 3.3.4): chunk j = d_root[h_displs[j] ..
 * + h_counts[j]) is compressed as its own stream; all chunks in one
 * persistent launch, packed back to back into d_out (out_cap >= sum of the
 * chunk bounds) with sizes in d_chunk_bytes[j] and offsets (exclusive sum)
 * in d_chunk_offsets[j]. */
gz_status gz_scatter_compress(gz_ctx* ctx, const void* d_root, gz_dtype dtype,
                              const uint64_t* h_counts, const uint64_t* h_displs,
                              uint32_t nchunks, double eb, const gz_params* p,
                              void* d_out, uint64_t out_cap,
                              uint64_t* d_chunk_bytes, uint64_t* d_chunk_offsets,
                              gz_stream_t stream);

/* Inverse of gz_scatter_compress in one batched launch -- each destination
 * of gZ-Scatter decompresses the chunk it received (Sec. 3.3.4; the paper
 * overlaps these decompressions on several streams, here they share one
 * launch): chunk j starts at d_packed + d_chunk_offsets[j] (device array of
 * nchunks offsets) and decodes h_counts[j] elements into d_root +
 * h_displs[j].  A chunk whose stream is malformed or says otherwise sets
 * GZ_ECORRUPT on the device; nothing is read past packed_bytes. */
gz_status gz_scatter_decompress(gz_ctx* ctx, const void* d_packed,
                                uint64_t packed_bytes,
                                const uint64_t* d_chunk_offsets,
                                gz_dtype dtype, const uint64_t* h_counts,
                                const uint64_t* h_displs, uint32_t nchunks,
                                const gz_params* p, void* d_root,
                                gz_stream_t stream);

/* Batched independent requests (fp32 and fp64 mixed, per-request eb and
 * block length) in one persistent launch: the many small compressions that
 * under-use the GPU one by one (Sec. 3.2.2, Sec. 3.3.3 "total compression
 * cost") share one grid.  op selects compress, decompress, fused step or
 * decode-and-accumulate (fp32 only, as gz_decompress_add); p gives
 * threads/grid only (0: the shapes gz_tune_batch stored for this op and
 * element-type mix, else defaults).  threads 64 selects the per-wave
 * kernels: for any decompress or decode-and-accumulate batch whose jobs
 * each hold at least one element, and for a compress or fused batch whose
 * jobs are all fp32 with the same block length and superblock count
 * (GZ_EUNSUPPORTED for other batches).  By default decompress and fused
 * batches run on them where they can. */
gz_status gz_batch(gz_ctx* ctx, gz_op op, const gz_request* h_reqs,
                   uint32_t nreq, const gz_params* p, gz_stream_t stream);

/* A plan uploads a batch's descriptors once (synchronous: it first waits for
 * the device, then copies) into the context's plan arena, so that
 * gz_plan_launch is a single kernel launch with no host work, suitable for
 * stream capture.  No device memory is allocated: the arena, sized at
 * gz_ctx_create, holds 16 * max_requests + 64 descriptors and the strip
 * maps of 16 batches of max_elems elements; a plan that does not fit
 * returns GZ_ENOSPC.  Plans of one context must run in order on one stream.
 * Destroy graphs and plans before their context (a plan outliving its
 * context can only be destroyed). */
gz_status gz_plan_create(gz_ctx* ctx, gz_op op, const gz_request* h_reqs,
                         uint32_t nreq, const gz_params* p, gz_plan** plan);
gz_status gz_plan_launch(gz_plan* plan, gz_stream_t stream);
void gz_plan_destroy(gz_plan* plan);

/* Captures the launches of nplans plans, in order, into one HIP graph and
 * instantiates it (synchronous). */
gz_status gz_graph_create(gz_plan* const* plans, uint32_t nplans,
                          gz_graph** graph);
gz_status gz_graph_launch(gz_graph* graph, gz_stream_t stream);
void gz_graph_destroy(gz_graph* graph);

/* The autotuner (block size and threads per block, the batching extension
 * for the small-input under-use of Sec. 3.2.2).  Times the launch shapes
 * (threads, grid; threads 64 = the per-wave kernels) of compress and
 * decompress for (dtype, block_len)
 * on the caller's sample d_sample[0..n) (read only) and stores the fastest
 * in the context; with block_len 0 it tries 32, 64 and 128 and stores the
 * fastest as the block length of requests that give 0.  d_work is a
 * caller-owned device buffer of at least
 *   roundup256(n * sizeof(T)) + roundup256(gz_compress_bound(n, dtype, 32)) + 8
 * bytes (decoded values, stream, size word) that must not overlap the
 * sample (GZ_ENOSPC if smaller).  Runs on `stream` and waits for it; with a
 * non-null cache_path, reads and appends a JSON-lines cache of shapes there.
 * Allocates nothing.  Synchronous. */
gz_status gz_tune(gz_ctx* ctx, gz_dtype dtype, uint32_t block_len, const void* d_sample,
                  uint64_t n, void* d_work, uint64_t work_bytes, const char* cache_path,
                  gz_params* best, gz_stream_t stream);

/* Times the caller's own batch (op compress, decompress or fused step; the
 * accumulate op updates in place and is refused with GZ_EINVAL) over
 * threads {128..1024} x grid {1, 2, occupancy, 2 x occupancy} x CUs, plus
 * the per-wave kernels where the batch qualifies (as gz_batch), and
 * stores the fastest shape for (op, batch holds fp64) in the context, where
 * gz_batch and gz_plan_create take it.  Runs the batch 4 times per shape in
 * place on `stream` (outputs are rewritten with the same bytes) and waits
 * for it; allocates nothing.  Synchronous. */
gz_status gz_tune_batch(gz_ctx* ctx, gz_op op, const gz_request* h_reqs, uint32_t nreq,
                        const char* cache_path, gz_params* best, gz_stream_t stream);

/* Learned selector (mode 1, select 0): loads the int8 weight blob
 * ("GZM1", u32 shift, int8 W1[32][16], int32 b1[32], int8 W2[3][32],
 * int32 b2[3]; 756 bytes).  Synchronous. */
gz_status gz_selector_load(gz_ctx* ctx, const void* h_blob, uint64_t bytes);

/* Training data of the selector: for each 8x8 tile of an nx-wide fp32 field
 * writes its 16 int8 features (d_feat[16*tile]), the byte sizes of its
 * NONE, L1D and L2D encodings (d_sizes[3*tile]) and the exhaustive-trial
 * label (d_label[tile], 0 NONE, 1 L1D, 2 L2D; 255 for RAW/ZERO tiles). */
gz_status gz_tile_trial(gz_ctx* ctx, const float* d_in, uint64_t n, uint32_t nx,
                        double eb, int8_t* d_feat, uint32_t* d_sizes,
                        uint8_t* d_label, gz_stream_t stream);

/* fp32 training of the selector's shadow network (16 -> 32 ReLU -> 3,
 * softmax cross-entropy).  d_w holds W1[32][16], b1[32], W2[3][32], b2[3]
 * (643 floats); d_feat/d_label as produced by gz_tile_trial (label 255 is
 * skipped).  gz_mlp_grad writes the mean-loss gradient of the first nsamp
 * samples into d_grad (643 floats) and the mean loss into *d_loss;
 * gz_mlp_adam applies one Adam step (state d_m, d_v, step count `step`). */
gz_status gz_mlp_grad(gz_ctx* ctx, const float* d_w, const int8_t* d_feat,
                      const uint8_t* d_label, uint64_t nsamp, float* d_grad,
                      float* d_loss, gz_stream_t stream);
gz_status gz_mlp_adam(gz_ctx* ctx, float* d_w, const float* d_grad, float* d_m,
                      float* d_v, uint32_t step, float lr, gz_stream_t stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): gz_compress
 * without a context.  Arguments, bytes and host-side errors are those of
 * gz_compress, except that the MLP selector (mode 1, select 0) is not
 * available (GZ_EINVAL).  The workspace is a device-resident array of
 * 263,424 bytes that the library holds on each device until the process
 * ends; it serves streams of at most 32768 strips (2^30 fp32 elements at the
 * default 1024 threads, 2^28 fp64 elements at 256) or, with threads 64,
 * 32768 rounds of 8 superblocks (also 2^30 fp32 elements); larger inputs
 * return GZ_ENOSPC with nothing enqueued.  The call allocates nothing: its first
 * call on a device only looks up the array's address.  It enqueues the
 * compression and a one-wave kernel that writes the device status of the
 * call (GZ_OK, or GZ_ETIMEOUT when a look-back wait expired and the stream
 * is invalid) to *d_status (a caller-owned device word; may be NULL) and
 * clears it.  Every call on one device shares that device's array: calls
 * that overlap in time on one device (several streams or threads) race and
 * must be serialised by the caller. */
gz_status gz_compress_noalloc(const void* d_in, uint64_t n, gz_dtype dtype, double eb,
                              const gz_params* p, void* d_out, uint64_t out_cap,
                              uint64_t* d_out_bytes, uint32_t* d_status,
                              gz_stream_t stream);

const char* gz_status_str(gz_status s);

#ifdef __cplusplus
}
#endif
#endif
