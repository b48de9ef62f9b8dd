/*
 * gzo.c -- plain, slow CPU oracle of the GZ1 codec (test infrastructure only;
 * see gzo.h for the format it follows and the paper passages it rests on).
 *
 * Written for readability: one element, one block at a time, in the order the
 * format states the steps.  Build with -O2 -ffp-contract=off -fno-fast-math
 * so that every float operation is one IEEE operation in its own type.
 */
#include "gzo.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define SUPER 4096u          /* elements per superblock */
#define HDR_BYTES 64u
#define Q_LIMIT 536870911.0  /* 2^29 - 1 */

enum { K_ZERO = 0, K_L1D = 1, K_NONE = 2, K_L2D = 3, K_RAW = 7 };

/* ---------------------------------------------------------------- bytes */
static void put_u16(uint8_t* p, uint16_t v) { p[0] = v & 0xff; p[1] = v >> 8; }
static void put_u32(uint8_t* p, uint32_t v) {
  for (int i = 0; i < 4; ++i) p[i] = (uint8_t)(v >> (8 * i));
}
static void put_u64(uint8_t* p, uint64_t v) {
  for (int i = 0; i < 8; ++i) p[i] = (uint8_t)(v >> (8 * i));
}
static uint16_t get_u16(const uint8_t* p) { return (uint16_t)(p[0] | (p[1] << 8)); }
static uint32_t get_u32(const uint8_t* p) {
  uint32_t v = 0;
  for (int i = 3; i >= 0; --i) v = (v << 8) | p[i];
  return v;
}
static uint64_t get_u64(const uint8_t* p) {
  uint64_t v = 0;
  for (int i = 7; i >= 0; --i) v = (v << 8) | p[i];
  return v;
}

static uint64_t cdiv(uint64_t a, uint64_t b) { return (a + b - 1) / b; }
static uint64_t round4(uint64_t a) { return (a + 3) & ~(uint64_t)3; }
static int log2_of(int L) { return L == 32 ? 5 : L == 64 ? 6 : 7; }
static int elem_size(int dtype) { return dtype == 0 ? 4 : 8; }

/* bit length of |v|: 0 for v == 0 */
static int bitlen(int64_t v) {
  uint64_t a = v < 0 ? (uint64_t)(-v) : (uint64_t)v;
  int n = 0;
  while (a) { ++n; a >>= 1; }
  return n;
}

/* -------------------------------------------------------- quantisation */
/* Returns 1 (FAIL) or 0 and sets *q.  Arithmetic in float throughout. */
static int quant_f32(float x, float t, double eb, int32_t* q) {
  if (!isfinite(x)) return 1;
  float r = x / t;
  if (fabs((double)r) > Q_LIMIT) return 1;
  *q = (int32_t)rintf(r);
  float xh = (float)(*q) * t;
  if (!(fabs((double)x - (double)xh) <= eb)) return 1;
  return 0;
}

static int quant_f64(double x, double t, double eb, int32_t* q) {
  if (!isfinite(x)) return 1;
  double r = x / t;
  if (fabs(r) > Q_LIMIT) return 1;
  *q = (int32_t)rint(r);
  double xh = (double)(*q) * t;
  if (!(fabs(x - xh) <= eb)) return 1;
  return 0;
}

/* t = (T)(2 eb); returns 0 when t is unusable (zero or not finite). */
static int make_step(int dtype, double eb, float* t32, double* t64) {
  if (!(eb > 0.0) || !isfinite(eb)) return 0;
  double two_eb = 2.0 * eb;
  if (dtype == 0) {
    *t32 = (float)two_eb;
    return isfinite(*t32) && *t32 != 0.0f;
  }
  *t64 = two_eb;
  return isfinite(*t64) && *t64 != 0.0;
}

int gzo_quantize(const void* x, uint64_t n, int dtype, double eb, int32_t* q,
                 uint8_t* fail) {
  float t32 = 0;
  double t64 = 0;
  if ((dtype != 0 && dtype != 1) || !make_step(dtype, eb, &t32, &t64))
    return GZO_EINVAL;
  for (uint64_t i = 0; i < n; ++i) {
    int32_t qi = 0;
    int f = dtype == 0 ? quant_f32(((const float*)x)[i], t32, eb, &qi)
                       : quant_f64(((const double*)x)[i], t64, eb, &qi);
    q[i] = f ? 0 : qi;
    fail[i] = (uint8_t)f;
  }
  return GZO_OK;
}

/* -------------------------------------------------------------- layout */
typedef struct {
  uint64_t n;
  int dtype, L, mode, select;
  uint32_t nx;
  double eb;
  float t32;
  double t64;
  uint64_t B, NS, hdr_off, pay_off;
} Geom;

static void geom_fill(Geom* g) {
  g->B = cdiv(g->n, (uint64_t)g->L);
  g->NS = cdiv(g->n, SUPER);
  g->hdr_off = HDR_BYTES + 4 * g->NS;
  g->pay_off = g->hdr_off + round4(g->B);
}

uint64_t gzo_compress_bound(uint64_t n, int dtype, int block_len) {
  return HDR_BYTES + 4 * cdiv(n, SUPER) + round4(cdiv(n, (uint64_t)block_len)) +
         n * (uint64_t)elem_size(dtype);
}

/* Global element index of position i of block b. */
static uint64_t elem_index(const Geom* g, uint64_t b, int i) {
  if (g->mode == 0) return b * (uint64_t)g->L + (uint64_t)i;
  uint64_t tiles_per_row = g->nx / 8;
  uint64_t R = b / tiles_per_row, C = b % tiles_per_row;
  int r = i / 8, c = i % 8;
  return (8 * R + (uint64_t)r) * g->nx + 8 * C + (uint64_t)c;
}

static int valid_count(const Geom* g, uint64_t b) {
  uint64_t start = b * (uint64_t)g->L;
  uint64_t m = g->n - start;
  return m < (uint64_t)g->L ? (int)m : g->L;
}

/* --------------------------------------------------------- predictors */
/* Residuals d[0..L) of a block whose q[] is already tail-extended. */
static void residuals(int kind, int mode, int L, const int32_t* q, int32_t* d) {
  if (kind == K_NONE) {
    for (int i = 0; i < L; ++i) d[i] = q[i];
    return;
  }
  if (mode == 0) { /* L1D along the block */
    d[0] = 0;
    for (int i = 1; i < L; ++i) d[i] = q[i] - q[i - 1];
    return;
  }
  for (int r = 0; r < 8; ++r) {
    for (int c = 0; c < 8; ++c) {
      int32_t v;
      if (r == 0 && c == 0) v = 0;
      else if (r == 0) v = q[c] - q[c - 1];
      else if (c == 0) v = q[8 * r] - q[8 * (r - 1)];
      else if (kind == K_L1D) v = q[8 * r + c] - q[8 * r + c - 1];
      else
        v = q[8 * r + c] - q[8 * r + c - 1] - q[8 * (r - 1) + c] +
            q[8 * (r - 1) + c - 1];
      d[8 * r + c] = v;
    }
  }
}

static int width_of(const int32_t* d, int L) {
  int64_t mx = 0;
  for (int i = 0; i < L; ++i) {
    int64_t a = d[i] < 0 ? -(int64_t)d[i] : d[i];
    if (a > mx) mx = a;
  }
  return bitlen(mx);
}

static uint32_t pred_size(int kind, int F, int L) {
  uint32_t planes = F ? (uint32_t)(F + 1) * (uint32_t)(L / 8) : 0;
  return kind == K_NONE ? planes : 4 + planes;
}

/* ----------------------------------------------------------- selector */
/* Blob: "GZM1", u32 shift, int8 W1[32][16], int32 b1[32], int8 W2[3][32],
 * int32 b2[3]. */
#define BLOB_W1 8
#define BLOB_B1 (BLOB_W1 + GZO_MLP_HID * GZO_MLP_IN)
#define BLOB_W2 (BLOB_B1 + 4 * GZO_MLP_HID)
#define BLOB_B2 (BLOB_W2 + GZO_MLP_OUT * GZO_MLP_HID)
#define BLOB_END (BLOB_B2 + 4 * GZO_MLP_OUT)

uint64_t gzo_mlp_blob_bytes(void) { return BLOB_END; }

static int blob_ok(const uint8_t* blob) {
  if (!blob || get_u32(blob) != 0x314D5A47u) return 0;
  if (get_u32(blob + 4) > 24) return 0;
  for (int k = 0; k < GZO_MLP_HID; ++k) {
    int32_t b = (int32_t)get_u32(blob + BLOB_B1 + 4 * k);
    if (b <= -(1 << 24) || b >= (1 << 24)) return 0;
  }
  for (int o = 0; o < GZO_MLP_OUT; ++o) {
    int32_t b = (int32_t)get_u32(blob + BLOB_B2 + 4 * o);
    if (b <= -(1 << 24) || b >= (1 << 24)) return 0;
  }
  return 1;
}

/* floor(a / 2^s) for any sign of a */
static int64_t floor_shift(int64_t a, int s) {
  int64_t p = (int64_t)1 << s;
  int64_t qt = a / p;
  if (a % p != 0 && a < 0) qt -= 1;
  return qt;
}

int gzo_mlp_forward(const uint8_t* blob, const int8_t* f, int32_t* logits) {
  if (!blob_ok(blob)) return -1;
  int s = (int)get_u32(blob + 4);
  int64_t h[GZO_MLP_HID];
  for (int k = 0; k < GZO_MLP_HID; ++k) {
    int64_t acc = (int32_t)get_u32(blob + BLOB_B1 + 4 * k);
    for (int i = 0; i < GZO_MLP_IN; ++i)
      acc += (int64_t)(int8_t)blob[BLOB_W1 + GZO_MLP_IN * k + i] * f[i];
    int64_t v = s ? floor_shift(acc + ((int64_t)1 << (s - 1)), s) : acc;
    h[k] = v < 0 ? 0 : v > 127 ? 127 : v;
  }
  int best = 0;
  int64_t best_v = 0;
  for (int o = 0; o < GZO_MLP_OUT; ++o) {
    int64_t acc = (int32_t)get_u32(blob + BLOB_B2 + 4 * o);
    for (int k = 0; k < GZO_MLP_HID; ++k)
      acc += (int64_t)(int8_t)blob[BLOB_W2 + GZO_MLP_HID * o + k] * h[k];
    if (logits) logits[o] = (int32_t)acc;
    if (o == 0 || acc > best_v) { best = o; best_v = acc; }
  }
  return best;
}

/* Features: bit lengths of sampled values and sampled residuals of the tile:
 * four magnitudes, four horizontal differences, four vertical differences
 * and four second-order (2D Lorenzo) residuals. */
#define TQ(r, c) ((int64_t)q[8 * (r) + (c)])
static int64_t l2d_at(const int32_t* q, int r, int c) {
  return TQ(r, c) - TQ(r, c - 1) - TQ(r - 1, c) + TQ(r - 1, c - 1);
}
void gzo_tile_features(const int32_t* q, int8_t* f) {
  f[0] = (int8_t)bitlen(TQ(0, 0));
  f[1] = (int8_t)bitlen(TQ(2, 5));
  f[2] = (int8_t)bitlen(TQ(5, 2));
  f[3] = (int8_t)bitlen(TQ(7, 7));
  f[4] = (int8_t)bitlen(TQ(1, 1) - TQ(1, 0));
  f[5] = (int8_t)bitlen(TQ(3, 6) - TQ(3, 5));
  f[6] = (int8_t)bitlen(TQ(4, 3) - TQ(4, 2));
  f[7] = (int8_t)bitlen(TQ(6, 7) - TQ(6, 6));
  f[8] = (int8_t)bitlen(TQ(1, 3) - TQ(0, 3));
  f[9] = (int8_t)bitlen(TQ(3, 1) - TQ(2, 1));
  f[10] = (int8_t)bitlen(TQ(5, 6) - TQ(4, 6));
  f[11] = (int8_t)bitlen(TQ(7, 4) - TQ(6, 4));
  f[12] = (int8_t)bitlen(l2d_at(q, 1, 5));
  f[13] = (int8_t)bitlen(l2d_at(q, 2, 2));
  f[14] = (int8_t)bitlen(l2d_at(q, 5, 5));
  f[15] = (int8_t)bitlen(l2d_at(q, 6, 1));
}
#undef TQ

void gzo_tile_sizes(const int32_t* q, uint32_t* sizes3) {
  static const int kinds[3] = {K_NONE, K_L1D, K_L2D};
  int32_t d[64];
  for (int k = 0; k < 3; ++k) {
    residuals(kinds[k], 1, 64, q, d);
    sizes3[k] = pred_size(kinds[k], width_of(d, 64), 64);
  }
}

/* Predictor kind of a mode-1 tile that is neither RAW nor ZERO. */
static int choose_kind(const Geom* g, const int32_t* q, const uint8_t* blob) {
  static const int kinds[3] = {K_NONE, K_L1D, K_L2D};
  if (g->select == 2) return K_L1D;
  if (g->select == 1) {
    uint32_t s[3];
    gzo_tile_sizes(q, s);
    int best = 0;
    for (int k = 1; k < 3; ++k)
      if (s[k] < s[best]) best = k;
    return kinds[best];
  }
  int8_t f[GZO_MLP_IN];
  gzo_tile_features(q, f);
  return kinds[gzo_mlp_forward(blob, f, NULL)];
}

/* ------------------------------------------------------------- encode */
static int check_params(const Geom* g, const uint8_t* blob) {
  if (g->dtype != 0 && g->dtype != 1) return 0;
  if (g->L != 32 && g->L != 64 && g->L != 128) return 0;
  if (g->mode != 0 && g->mode != 1) return 0;
  if (g->mode == 1) {
    if (g->L != 64 || g->nx == 0 || g->nx % 8 != 0) return 0;
    if (g->n % (8 * (uint64_t)g->nx) != 0) return 0;
    if (g->select < 0 || g->select > 2) return 0;
    if (g->select == 0 && !blob_ok(blob)) return 0;
  } else if (g->nx != 0) {
    return 0;
  }
  /* payload offsets are kept in u32 words: at most 16 GiB of payload */
  if (g->n * (uint64_t)elem_size(g->dtype) >= ((uint64_t)1 << 34)) return 0;
  return 1;
}

static void write_header(uint8_t* out, const Geom* g, uint64_t payload) {
  memset(out, 0, HDR_BYTES);
  out[0] = 'G'; out[1] = 'Z'; out[2] = 'C'; out[3] = '1';
  put_u16(out + 4, 1);
  out[6] = (uint8_t)g->dtype;
  out[7] = (uint8_t)log2_of(g->L);
  put_u64(out + 8, g->n);
  uint64_t ebits;
  memcpy(&ebits, &g->eb, 8);
  put_u64(out + 16, ebits);
  put_u64(out + 24, payload);
  put_u32(out + 32, (uint32_t)g->mode);
  put_u32(out + 36, g->nx);
  put_u32(out + 40, SUPER);
}

/* Encodes block b; writes its payload at p and returns the header byte and
 * the payload size. */
static uint8_t encode_block(const Geom* g, const void* x, uint64_t b,
                            const uint8_t* blob, uint8_t* p, uint32_t* size) {
  int L = g->L, m = valid_count(g, b), es = elem_size(g->dtype);
  int32_t q[128], d[128];
  int fail = 0, nonzero = 0;
  for (int i = 0; i < m; ++i) {
    uint64_t e = elem_index(g, b, i);
    int32_t qi = 0;
    fail |= g->dtype == 0 ? quant_f32(((const float*)x)[e], g->t32, g->eb, &qi)
                          : quant_f64(((const double*)x)[e], g->t64, g->eb, &qi);
    q[i] = qi;
    nonzero |= qi != 0;
  }
  uint32_t raw_size = (uint32_t)(m * es);
  int kind;
  if (fail) kind = K_RAW;
  else if (!nonzero) kind = K_ZERO;
  else {
    for (int i = m; i < L; ++i) q[i] = q[m - 1]; /* tail repeats q[m-1] */
    kind = g->mode == 0 ? K_L1D : choose_kind(g, q, blob);
  }
  int F = 0;
  if (kind != K_RAW && kind != K_ZERO) {
    residuals(kind, g->mode, L, q, d);
    F = width_of(d, L);
    if (pred_size(kind, F, L) > raw_size) kind = K_RAW;
  }
  if (kind == K_ZERO) {
    *size = 0;
    return 0;
  }
  if (kind == K_RAW) {
    for (int i = 0; i < m; ++i)
      memcpy(p + (size_t)i * es, (const uint8_t*)x + elem_index(g, b, i) * es, es);
    *size = raw_size;
    return (uint8_t)(K_RAW << 5);
  }
  uint32_t sz = pred_size(kind, F, L);
  memset(p, 0, sz);
  uint8_t* w = p;
  if (kind != K_NONE) {
    put_u32(w, (uint32_t)q[0]);
    w += 4;
  }
  if (F > 0) {
    int words = L / 32;
    /* sign plane */
    for (int i = 0; i < L; ++i)
      if (d[i] < 0) w[4 * (i / 32) + (i % 32) / 8] |= (uint8_t)(1u << (i % 8));
    w += 4 * words;
    for (int j = 0; j < F; ++j) {
      for (int i = 0; i < L; ++i) {
        uint32_t a = d[i] < 0 ? (uint32_t)(-(int64_t)d[i]) : (uint32_t)d[i];
        if ((a >> j) & 1u) w[4 * (i / 32) + (i % 32) / 8] |= (uint8_t)(1u << (i % 8));
      }
      w += 4 * words;
    }
  }
  *size = sz;
  return (uint8_t)((kind << 5) | F);
}

int gzo_compress(const void* x, uint64_t n, int dtype, double eb, int block_len,
                 int mode, uint32_t nx, int select, const uint8_t* mlp_blob,
                 uint8_t* out, uint64_t out_cap, uint64_t* out_bytes) {
  Geom g;
  memset(&g, 0, sizeof g);
  g.n = n; g.dtype = dtype; g.L = block_len; g.mode = mode; g.nx = nx;
  g.select = mode == 1 ? select : 0; g.eb = eb;
  if (!check_params(&g, mlp_blob)) return GZO_EINVAL;
  if (!make_step(dtype, eb, &g.t32, &g.t64)) return GZO_EINVAL;
  geom_fill(&g);
  if (out_cap < gzo_compress_bound(n, dtype, block_len)) return GZO_ENOSPC;

  memset(out, 0, g.pay_off);
  uint64_t payload = 0;
  uint64_t blocks_per_super = SUPER / (uint64_t)g.L;
  for (uint64_t b = 0; b < g.B; ++b) {
    if (b % blocks_per_super == 0)
      put_u32(out + HDR_BYTES + 4 * (b / blocks_per_super), (uint32_t)(payload / 4));
    uint32_t sz = 0;
    out[g.hdr_off + b] = encode_block(&g, x, b, mlp_blob, out + g.pay_off + payload, &sz);
    payload += sz;
  }
  write_header(out, &g, payload);
  *out_bytes = g.pay_off + payload;
  return GZO_OK;
}

/* ------------------------------------------------------------- decode */
static int parse_header(const uint8_t* in, uint64_t in_bytes, Geom* g,
                        uint64_t* payload) {
  if (in_bytes < HDR_BYTES) return 0;
  if (in[0] != 'G' || in[1] != 'Z' || in[2] != 'C' || in[3] != '1') return 0;
  if (get_u16(in + 4) != 1) return 0;
  for (int i = 44; i < 64; ++i)
    if (in[i]) return 0;
  if (get_u32(in + 40) != SUPER) return 0;
  memset(g, 0, sizeof *g);
  g->dtype = in[6];
  int l2 = in[7];
  if (l2 < 5 || l2 > 7) return 0;
  g->L = 1 << l2;
  g->n = get_u64(in + 8);
  uint64_t ebits = get_u64(in + 16);
  memcpy(&g->eb, &ebits, 8);
  *payload = get_u64(in + 24);
  g->mode = (int)get_u32(in + 32);
  g->nx = get_u32(in + 36);
  g->select = 2; /* decoding never consults the selector */
  if (!check_params(g, NULL)) return 0;
  if (!make_step(g->dtype, g->eb, &g->t32, &g->t64)) return 0;
  geom_fill(g);
  if (*payload % 4 != 0) return 0;
  if (*payload > in_bytes || g->pay_off > in_bytes - *payload) return 0;
  return 1;
}

int gzo_stream_info(const uint8_t* in, uint64_t in_bytes, uint64_t* n,
                    int* dtype, int* block_len, int* mode, uint32_t* nx,
                    double* eb, uint64_t* total_bytes) {
  Geom g;
  uint64_t payload;
  if (!parse_header(in, in_bytes, &g, &payload)) return GZO_ECORRUPT;
  if (n) *n = g.n;
  if (dtype) *dtype = g.dtype;
  if (block_len) *block_len = g.L;
  if (mode) *mode = g.mode;
  if (nx) *nx = g.nx;
  if (eb) *eb = g.eb;
  if (total_bytes) *total_bytes = g.pay_off + payload;
  return GZO_OK;
}

/* Block size implied by a header byte; returns 0 on a reserved or
 * inconsistent header byte. */
static int header_size(const Geom* g, uint64_t b, uint8_t h, uint32_t* size) {
  int kind = h >> 5, F = h & 31;
  int m = valid_count(g, b);
  switch (kind) {
    case K_ZERO: if (F) return 0; *size = 0; return 1;
    case K_RAW: if (F) return 0; *size = (uint32_t)(m * elem_size(g->dtype)); return 1;
    case K_L1D: *size = pred_size(K_L1D, F, g->L); return 1;
    case K_NONE: if (g->mode != 1 || F == 0) return 0;
                 *size = pred_size(K_NONE, F, g->L); return 1;
    case K_L2D: if (g->mode != 1) return 0;
                *size = pred_size(K_L2D, F, g->L); return 1;
    default: return 0;
  }
}

static void put_elem(const Geom* g, void* out, uint64_t e, int32_t q) {
  if (g->dtype == 0) ((float*)out)[e] = (float)q * g->t32;
  else ((double*)out)[e] = (double)q * g->t64;
}

static void decode_block(const Geom* g, uint64_t b, uint8_t h, const uint8_t* p,
                         void* out) {
  int kind = h >> 5, F = h & 31, L = g->L, m = valid_count(g, b);
  int es = elem_size(g->dtype);
  if (kind == K_ZERO) {
    for (int i = 0; i < m; ++i) put_elem(g, out, elem_index(g, b, i), 0);
    return;
  }
  if (kind == K_RAW) {
    for (int i = 0; i < m; ++i)
      memcpy((uint8_t*)out + elem_index(g, b, i) * es, p + (size_t)i * es, es);
    return;
  }
  int32_t base = 0, d[128], q[128];
  const uint8_t* w = p;
  if (kind != K_NONE) {
    base = (int32_t)get_u32(w);
    w += 4;
  }
  int words = L / 32;
  for (int i = 0; i < L; ++i) d[i] = 0;
  if (F > 0) {
    const uint8_t* sign = w;
    w += 4 * words;
    for (int j = 0; j < F; ++j, w += 4 * words)
      for (int i = 0; i < L; ++i)
        if ((w[4 * (i / 32) + (i % 32) / 8] >> (i % 8)) & 1) d[i] |= (int32_t)(1u << j);
    for (int i = 0; i < L; ++i)
      if ((sign[4 * (i / 32) + (i % 32) / 8] >> (i % 8)) & 1) d[i] = -d[i];
  }
  /* Sums wrap modulo 2^32: a well-formed stream never wraps, and a damaged
   * one must still decode without undefined behaviour. */
  uint32_t u[128];
  if (kind == K_NONE) {
    for (int i = 0; i < L; ++i) u[i] = (uint32_t)d[i];
  } else if (g->mode == 0) {
    u[0] = (uint32_t)base;
    for (int i = 1; i < L; ++i) u[i] = u[i - 1] + (uint32_t)d[i];
  } else {
    for (int r = 0; r < 8; ++r)
      for (int c = 0; c < 8; ++c) {
        uint32_t v, di = (uint32_t)d[8 * r + c];
        if (r == 0 && c == 0) v = (uint32_t)base;
        else if (r == 0) v = u[c - 1] + di;
        else if (c == 0) v = u[8 * (r - 1)] + di;
        else if (kind == K_L1D) v = u[8 * r + c - 1] + di;
        else v = di + u[8 * r + c - 1] + u[8 * (r - 1) + c] - u[8 * (r - 1) + c - 1];
        u[8 * r + c] = v;
      }
  }
  for (int i = 0; i < L; ++i) q[i] = (int32_t)u[i];
  for (int i = 0; i < m; ++i) put_elem(g, out, elem_index(g, b, i), q[i]);
}

int gzo_decompress(const uint8_t* in, uint64_t in_bytes, void* out,
                   uint64_t out_cap_elems, uint64_t* n_out) {
  Geom g;
  uint64_t payload;
  if (!parse_header(in, in_bytes, &g, &payload)) return GZO_ECORRUPT;
  if (g.n > out_cap_elems) return GZO_ENOSPC;
  /* validate every header byte and the superblock table before writing */
  uint64_t blocks_per_super = SUPER / (uint64_t)g.L, off = 0;
  for (uint64_t b = 0; b < g.B; ++b) {
    if (b % blocks_per_super == 0 &&
        (uint64_t)get_u32(in + HDR_BYTES + 4 * (b / blocks_per_super)) * 4 != off)
      return GZO_ECORRUPT;
    uint32_t sz;
    if (!header_size(&g, b, in[g.hdr_off + b], &sz)) return GZO_ECORRUPT;
    off += sz;
  }
  if (off != payload) return GZO_ECORRUPT;
  for (uint64_t i = g.B; i < round4(g.B); ++i)
    if (in[g.hdr_off + i]) return GZO_ECORRUPT;
  off = 0;
  for (uint64_t b = 0; b < g.B; ++b) {
    uint32_t sz;
    header_size(&g, b, in[g.hdr_off + b], &sz);
    decode_block(&g, b, in[g.hdr_off + b], in + g.pay_off + off, out);
    off += sz;
  }
  if (n_out) *n_out = g.n;
  return GZO_OK;
}

/* --------------------------------------------------------- fused step */
int gzo_fused_step(const uint8_t* in, uint64_t in_bytes, const float* local,
                   uint64_t n, double eb, int block_len, uint8_t* out,
                   uint64_t out_cap, uint64_t* out_bytes) {
  uint64_t sn;
  int dt, L, mode;
  uint32_t nx;
  if (gzo_stream_info(in, in_bytes, &sn, &dt, &L, &mode, &nx, NULL, NULL) != GZO_OK)
    return GZO_ECORRUPT;
  if (dt != 0 || mode != 0 || sn != n || L != block_len) return GZO_ECORRUPT;
  float* y = (float*)malloc((n ? n : 1) * sizeof(float));
  if (!y) return GZO_EINVAL;
  int st = gzo_decompress(in, in_bytes, y, n, NULL);
  if (st == GZO_OK) {
    for (uint64_t i = 0; i < n; ++i) y[i] = y[i] + local[i]; /* fixed order */
    st = gzo_compress(y, n, 0, eb, block_len, 0, 0, 0, NULL, out, out_cap, out_bytes);
  }
  free(y);
  return st;
}

/* ------------------------------------------------------------ scatter */
int gzo_scatter_compress(const void* root, int dtype, const uint64_t* counts,
                         const uint64_t* displs, uint32_t nchunks, double eb,
                         int block_len, uint8_t* out, uint64_t out_cap,
                         uint64_t* chunk_bytes, uint64_t* chunk_offsets) {
  uint64_t off = 0, need = 0;
  int es = dtype == 0 ? 4 : 8;
  for (uint32_t j = 0; j < nchunks; ++j)
    need += gzo_compress_bound(counts[j], dtype, block_len);
  if (out_cap < need) return GZO_ENOSPC;
  for (uint32_t j = 0; j < nchunks; ++j) {
    uint64_t nb = 0;
    int st = gzo_compress((const uint8_t*)root + displs[j] * es, counts[j], dtype,
                          eb, block_len, 0, 0, 0, NULL, out + off, out_cap - off, &nb);
    if (st != GZO_OK) return st;
    chunk_bytes[j] = nb;
    chunk_offsets[j] = off;
    off += nb;
  }
  return GZO_OK;
}

/* ------------------------------------------------------ selector data */
/* Per 8x8 tile of an nx-wide fp32 field: its features, the sizes of its
 * NONE, L1D and L2D encodings and the exhaustive-trial label (0 NONE,
 * 1 L1D, 2 L2D; 255 when the tile is RAW or ZERO, whose features and sizes
 * are then left as computed from q = 0 for failing elements). */
int gzo_tile_trial(const float* x, uint64_t n, uint32_t nx, double eb, int8_t* feat,
                   uint32_t* sizes, uint8_t* label) {
  Geom g;
  memset(&g, 0, sizeof g);
  g.n = n; g.dtype = 0; g.L = 64; g.mode = 1; g.nx = nx; g.select = 1; g.eb = eb;
  if (!check_params(&g, NULL) || !make_step(0, eb, &g.t32, &g.t64)) return GZO_EINVAL;
  geom_fill(&g);
  for (uint64_t b = 0; b < g.B; ++b) {
    int32_t q[64];
    int fail = 0, nonzero = 0;
    for (int i = 0; i < 64; ++i) {
      int32_t qi = 0;
      fail |= quant_f32(x[elem_index(&g, b, i)], g.t32, eb, &qi);
      q[i] = qi;
      nonzero |= qi != 0;
    }
    gzo_tile_features(q, feat + 16 * b);
    gzo_tile_sizes(q, sizes + 3 * b);
    int best = 0;
    for (int k = 1; k < 3; ++k)
      if (sizes[3 * b + k] < sizes[3 * b + best]) best = k;
    label[b] = (fail || !nonzero) ? 255 : (uint8_t)best;
  }
  return GZO_OK;
}

/* ------------------------------------------- all-core variants (OpenMP)
 * The same encodings with the host's cores working on superblocks at
 * once: every superblock's blocks are encoded, in order, into a scratch
 * area of their own; the offsets of the superblocks are then summed one
 * after another (the exclusive scan stays serial), and the payloads copied
 * into place.  Decoding validates the stream serially as gzo_decompress
 * does, then decodes superblocks at once from their table entries.  The
 * bytes are those of gzo_compress / gzo_decompress. */
int gzo_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

int gzo_compress_mt(const void* x, uint64_t n, int dtype, double eb, int block_len,
                    int mode, uint32_t nx, int select, const uint8_t* mlp_blob,
                    uint8_t* out, uint64_t out_cap, uint64_t* out_bytes) {
  Geom g;
  memset(&g, 0, sizeof g);
  g.n = n; g.dtype = dtype; g.L = block_len; g.mode = mode; g.nx = nx;
  g.select = mode == 1 ? select : 0; g.eb = eb;
  if (!check_params(&g, mlp_blob)) return GZO_EINVAL;
  if (!make_step(dtype, eb, &g.t32, &g.t64)) return GZO_EINVAL;
  geom_fill(&g);
  if (out_cap < gzo_compress_bound(n, dtype, block_len)) return GZO_ENOSPC;
  memset(out, 0, g.pay_off);
  const uint64_t bps = SUPER / (uint64_t)g.L, room = (uint64_t)SUPER * elem_size(dtype);
  uint8_t* scratch = (uint8_t*)malloc(g.NS ? g.NS * room : 1);
  uint64_t* sizes = (uint64_t*)malloc((g.NS ? g.NS : 1) * sizeof(uint64_t));
  if (!scratch || !sizes) {
    free(scratch);
    free(sizes);
    return GZO_EINVAL;
  }
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t k = 0; k < (int64_t)g.NS; ++k) {
    uint64_t used = 0;
    for (uint64_t b = (uint64_t)k * bps; b < g.B && b < ((uint64_t)k + 1) * bps; ++b) {
      uint32_t sz = 0;
      out[g.hdr_off + b] = encode_block(&g, x, b, mlp_blob, scratch + k * room + used, &sz);
      used += sz;
    }
    sizes[k] = used;
  }
  uint64_t payload = 0;
  for (uint64_t k = 0; k < g.NS; ++k) {  /* exclusive scan, in order */
    put_u32(out + HDR_BYTES + 4 * k, (uint32_t)(payload / 4));
    payload += sizes[k];
  }
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t k = 0; k < (int64_t)g.NS; ++k) {
    uint64_t at = (uint64_t)get_u32(out + HDR_BYTES + 4 * k) * 4;
    memcpy(out + g.pay_off + at, scratch + k * room, sizes[k]);
  }
  free(scratch);
  free(sizes);
  write_header(out, &g, payload);
  *out_bytes = g.pay_off + payload;
  return GZO_OK;
}

int gzo_decompress_mt(const uint8_t* in, uint64_t in_bytes, void* out,
                      uint64_t out_cap_elems, uint64_t* n_out) {
  Geom g;
  uint64_t payload;
  if (!parse_header(in, in_bytes, &g, &payload)) return GZO_ECORRUPT;
  if (g.n > out_cap_elems) return GZO_ENOSPC;
  uint64_t bps = SUPER / (uint64_t)g.L, off = 0;
  for (uint64_t b = 0; b < g.B; ++b) {
    if (b % bps == 0 && (uint64_t)get_u32(in + HDR_BYTES + 4 * (b / bps)) * 4 != off)
      return GZO_ECORRUPT;
    uint32_t sz;
    if (!header_size(&g, b, in[g.hdr_off + b], &sz)) return GZO_ECORRUPT;
    off += sz;
  }
  if (off != payload) return GZO_ECORRUPT;
  for (uint64_t i = g.B; i < round4(g.B); ++i)
    if (in[g.hdr_off + i]) return GZO_ECORRUPT;
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t k = 0; k < (int64_t)g.NS; ++k) {
    uint64_t at = (uint64_t)get_u32(in + HDR_BYTES + 4 * k) * 4;
    for (uint64_t b = (uint64_t)k * bps; b < g.B && b < ((uint64_t)k + 1) * bps; ++b) {
      uint32_t sz;
      header_size(&g, b, in[g.hdr_off + b], &sz);
      decode_block(&g, b, in[g.hdr_off + b], in + g.pay_off + at, out);
      at += sz;
    }
  }
  if (n_out) *n_out = g.n;
  return GZO_OK;
}

int gzo_fused_step_mt(const uint8_t* in, uint64_t in_bytes, const float* local,
                      uint64_t n, double eb, int block_len, uint8_t* out,
                      uint64_t out_cap, uint64_t* out_bytes) {
  uint64_t sn;
  int dt, L, mode;
  uint32_t nx;
  if (gzo_stream_info(in, in_bytes, &sn, &dt, &L, &mode, &nx, NULL, NULL) != GZO_OK)
    return GZO_ECORRUPT;
  if (dt != 0 || mode != 0 || sn != n || L != block_len) return GZO_ECORRUPT;
  float* y = (float*)malloc((n ? n : 1) * sizeof(float));
  if (!y) return GZO_EINVAL;
  int st = gzo_decompress_mt(in, in_bytes, y, n, NULL);
  if (st == GZO_OK) {
#pragma omp parallel for
    for (int64_t i = 0; i < (int64_t)n; ++i) y[i] = y[i] + local[i]; /* elementwise */
    st = gzo_compress_mt(y, n, 0, eb, block_len, 0, 0, 0, NULL, out, out_cap, out_bytes);
  }
  free(y);
  return st;
}
