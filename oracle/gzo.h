/*
 * gzo.h -- CPU oracle for the GZ1 error-bounded stream codec.
 *
 * TEST INFRASTRUCTURE ONLY.  Only tests/, the smoke check and the benchmark's
 * CPU-baseline leg may load this library.  It shares no code, header, table
 * or constant with the HIP library under paper_2308_05199_amd/csrc.
 *
 * What the paper fixes (gZCCL, arXiv 2308.05199):
 *   - messages are compressed by an error-bounded lossy compressor under an
 *     ABSOLUTE error bound (Sec. 4.1, default 1E-4), so the compressed size is
 *     only known after compression (Sec. 2 / Sec. 3.3.2);
 *   - compression keeps its block offsets and flags in separate buffers
 *     (Sec. 3.3.2, Sec. 3.3.4 "multi-stream lossy compression");
 *   - each ring Reduce_scatter round decompresses the incoming chunk, reduces
 *     it with the local chunk and recompresses (Sec. 3.2.3, Sec. 3.3.3);
 *   - a Scatter compresses every destination chunk on its own and packs the
 *     compressed chunks back to back, keeping sizes and offsets (Sec. 3.3.4,
 *     gZ-Scatter);
 *   - every compression adds at most the error bound, and the expected
 *     accumulated error is zero (Sec. 3.3.3, "Accuracy loss").
 * The paper treats the compressor itself as a black box (cuSZp).  The codec
 * below is the project's own: q = rint(x / (2 eb)), in-block Lorenzo
 * prediction, fixed-length bit planes per block, block offsets from an
 * exclusive prefix sum.  Its byte format ("GZ1", version 1) is:
 *
 *   t       = (T)(2*eb)               (fp64 product, one rounding to T)
 *   per element x (arithmetic in T, round-to-nearest-even, no fused ops):
 *     r = x / t ;  FAIL if x not finite or |r| > 536870911 (2^29-1)
 *     q = (int32) rint(r)             (ties to even)
 *     xh = (T)q * t ;  FAIL unless |(double)x - (double)xh| <= eb
 *   blocks : mode 0 -> L consecutive elements (L in {32,64,128}); the last
 *            block may be short (m valid elements); positions past m repeat
 *            q[m-1], i.e. carry residual 0.
 *            mode 1 -> 8x8 tiles of a row-major nx-wide field (L = 64);
 *            tile b = R*(nx/8)+C, local index i = 8r+c.
 *   residuals: L1D  (mode 0) d0 = 0, di = qi - q(i-1)
 *              L1D  (mode 1) d(0,0)=0; c>0: q(r,c)-q(r,c-1); c=0: q(r,0)-q(r-1,0)
 *              L2D  (mode 1) first row/column as L1D, else
 *                   q(r,c)-q(r,c-1)-q(r-1,c)+q(r-1,c-1)
 *              NONE (mode 1) d = q, no base
 *   F = bit length of max |d| (0..31); sign bit = (d < 0)
 *   kind: RAW(7) if any valid element FAILs; else ZERO(0) if all valid q are
 *         0; else L1D(1) in mode 0, or the selector's choice among NONE(2),
 *         L1D(1), L2D(3) in mode 1; finally RAW if size(kind) > size(RAW).
 *   size (bytes): ZERO 0; L1D/L2D 4 + (F ? (F+1)*L/8 : 0);
 *                 NONE (F ? (F+1)*L/8 : 0); RAW m*sizeof(T)
 *   payload of a block: [int32 base (L1D/L2D)] [sign plane] [plane 0] ...
 *                       [plane F-1]; a plane is L/32 little-endian u32 words,
 *                       element i is bit (i%32) of word i/32.  RAW: the m
 *                       input values bit for bit.
 *   block header byte  = kind<<5 | F  (F = 0 for ZERO and RAW)
 *   stream = 64-byte header | NS u32 superblock entries | B header bytes
 *            zero-padded to 4 | payload (blocks in order, no gaps)
 *     header: 0 u32 magic "GZC1", 4 u16 version 1, 6 u8 dtype (0 f32, 1 f64),
 *             7 u8 log2 L, 8 u64 n, 16 f64 eb, 24 u64 payload bytes,
 *             32 u32 mode, 36 u32 nx (0 in mode 0), 40 u32 S = 4096,
 *             44..63 zero
 *     superblock k = elements [4096k, 4096(k+1)) in block order; its entry
 *     is (payload offset of its first block) / 4.  NS = ceil(n/4096),
 *     B = ceil(n/L).
 *   decode: ZERO -> +0, RAW -> bit copy, else rebuild q and x' = (T)q * t.
 *
 * Fused reduction step (fp32): y = fl32(x' + local), then encode y.
 * Scatter: chunk j = elements [displs[j], displs[j]+counts[j]) encoded as its
 * own stream; streams packed back to back; offsets = exclusive sum of sizes.
 *
 * Selector (mode 1, select = 0): 16 int8 features of the tile's q, an int8
 * MLP 16->32->3 with int32 accumulation, a rounding arithmetic shift and a
 * [0,127] clamp between the layers, argmax with the lowest index winning
 * ties; output 0 NONE, 1 L1D, 2 L2D.  The features are bit lengths:
 *   f0..f3   |q(r,c)|                                at (0,0) (2,5) (5,2) (7,7)
 *   f4..f7   |q(r,c) - q(r,c-1)|                     at (1,1) (3,6) (4,3) (6,7)
 *   f8..f11  |q(r,c) - q(r-1,c)|                     at (1,3) (3,1) (5,6) (7,4)
 *   f12..f15 |q(r,c) - q(r,c-1) - q(r-1,c) + q(r-1,c-1)| at (1,5) (2,2) (5,5) (6,1)  select = 1 is the exhaustive trial:
 * smallest size among NONE, L1D, L2D, ties to the first in that order.
 * select = 2 always uses L1D.
 */
#ifndef GZO_H
#define GZO_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { GZO_OK = 0, GZO_EINVAL = 1, GZO_ENOSPC = 2, GZO_ECORRUPT = 3 };

/* Weight blob of the selector network: see gzo_mlp_blob_bytes(). */
#define GZO_MLP_IN 16
#define GZO_MLP_HID 32
#define GZO_MLP_OUT 3

uint64_t gzo_compress_bound(uint64_t n, int dtype, int block_len);

/* Per-element quantisation (steps r, q, xh, FAIL above).  q[i] is 0 where
 * fail[i] is 1. */
int gzo_quantize(const void* x, uint64_t n, int dtype, double eb,
                 int32_t* q, uint8_t* fail);

int gzo_compress(const void* x, uint64_t n, int dtype, double eb,
                 int block_len, int mode, uint32_t nx, int select,
                 const uint8_t* mlp_blob, uint8_t* out, uint64_t out_cap,
                 uint64_t* out_bytes);

/* Reads the stream header; returns GZO_ECORRUPT if it is not a GZ1 stream. */
int gzo_stream_info(const uint8_t* in, uint64_t in_bytes, uint64_t* n,
                    int* dtype, int* block_len, int* mode, uint32_t* nx,
                    double* eb, uint64_t* total_bytes);

int gzo_decompress(const uint8_t* in, uint64_t in_bytes, void* out,
                   uint64_t out_cap_elems, uint64_t* n_out);

/* The incoming stream must be fp32, mode 0, n elements, block length
 * block_len; it is decoded with its own eb and y is encoded with eb. */
int gzo_fused_step(const uint8_t* in, uint64_t in_bytes, const float* local,
                   uint64_t n, double eb, int block_len, uint8_t* out,
                   uint64_t out_cap, uint64_t* out_bytes);

int gzo_scatter_compress(const void* root, int dtype, const uint64_t* counts,
                         const uint64_t* displs, uint32_t nchunks, double eb,
                         int block_len, uint8_t* out, uint64_t out_cap,
                         uint64_t* chunk_bytes, uint64_t* chunk_offsets);

/* Selector pieces on one 8x8 tile of quantised values (q[8*r+c]). */
void gzo_tile_features(const int32_t* q, int8_t* feat);
int gzo_mlp_forward(const uint8_t* blob, const int8_t* feat, int32_t* logits);
uint64_t gzo_mlp_blob_bytes(void);
/* Sizes in bytes of the NONE, L1D and L2D encodings of a tile. */
void gzo_tile_sizes(const int32_t* q, uint32_t* sizes3);
/* Features, sizes and exhaustive-trial labels of every tile of a field. */
int gzo_tile_trial(const float* x, uint64_t n, uint32_t nx, double eb, int8_t* feat,
                   uint32_t* sizes, uint8_t* label);

/* All-core variants: superblocks encoded (decoded) by the host's threads at
 * once, the offset scan kept serial; the same bytes as the calls above.
 * gzo_threads() is the thread count they use (OMP_NUM_THREADS). */
int gzo_threads(void);
int gzo_compress_mt(const void* x, uint64_t n, int dtype, double eb,
                    int block_len, int mode, uint32_t nx, int select,
                    const uint8_t* mlp_blob, uint8_t* out, uint64_t out_cap,
                    uint64_t* out_bytes);
int gzo_decompress_mt(const uint8_t* in, uint64_t in_bytes, void* out,
                      uint64_t out_cap_elems, uint64_t* n_out);
int gzo_fused_step_mt(const uint8_t* in, uint64_t in_bytes, const float* local,
                      uint64_t n, double eb, int block_len, uint8_t* out,
                      uint64_t out_cap, uint64_t* out_bytes);

#ifdef __cplusplus
}
#endif
#endif
