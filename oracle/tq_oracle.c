/*
 * Oracle for threshold and symmetric queries over bitmaps.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the library links or calls this
 * file; only the tests, the smoke check and the CPU baseline of the
 * benchmark do.  It shares no code, header or table with the GPU path.
 *
 * What it computes is the plain definition, written out the slow and
 * obvious way:
 *
 *  - Problem statement (Introduction, "Formulation"; section 2.3, threshold
 *    functions): given N bitmaps over positions 0..r-1 and a threshold T,
 *    output bit p is 1 iff at least T of the inputs have bit p set.
 *  - Symmetric functions (section 2.2; section 4.2 notes that counter-based
 *    methods take any user map from [0, N] to {0, 1}): output bit p is
 *    f(count(p)).
 *  - The evaluation is the per-position counter method ScanCount (section
 *    4.2, appendix D): one counter per position, incremented once per input
 *    that has the bit, then compared.  Here the counters of one 64-bit word
 *    column are kept at a time.
 *  - Bit layout (section 2.1, uncompressed bitmaps): position p is bit
 *    (p mod 64) of word p div 64, little-endian 64-bit words.  Bits of the
 *    last word at positions >= r are ignored on input and zero on output.
 *  - Run-length encoding (section 2.1, compressed bitmaps, word-aligned RLE
 *    with EWAH-style markers that give both a fill-run length and a count of
 *    following dirty words).  The paper gives the model, not bit widths; the
 *    marker layout used here is: bit 0 = fill value, bits 1..32 = number of
 *    fill words, bits 33..63 = number of literal (dirty) words that follow
 *    the marker.  A stream is a sequence of markers each followed by its
 *    literal words; the fill and literal counts must add up to exactly
 *    ceil(r/64) words.
 *  - Canonical encoding (the paper is silent; this is the reading used):
 *    a marker starts at word 0 and at every clean word (all zeros or all
 *    ones) whose predecessor is dirty or a clean word of the other fill
 *    value.  It covers the maximal run of equal clean words there (possibly
 *    empty at word 0) followed by the maximal run of dirty words.  Clean
 *    words are never emitted as literals.  With ceil(r/64) < 2^31 the count
 *    fields never overflow, so no run is ever split.
 */
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_OK 0
#define ORACLE_EFORMAT (-3)
#define ORACLE_EINVAL (-1)

static uint64_t words_for_bits(uint64_t r_bits) { return (r_bits + 63) / 64; }

/* valid-bit mask of word w of an r-bit bitmap */
static uint64_t valid_mask(uint64_t w, uint64_t r_bits) {
  uint64_t first = w * 64;
  if (first >= r_bits) return 0;
  if (r_bits - first >= 64) return ~(uint64_t)0;
  return ((uint64_t)1 << (r_bits - first)) - 1;
}

/*
 * Symmetric function over a matrix of words: words[j * m + c] is the word of
 * input j at column c; col_index[c] is that column's word index in the
 * bitmap (used only for the tail mask).  f has n + 1 entries, f[k] in {0,1}.
 * out[c] receives the output word.
 */
int oracle_symmetric_cols(const uint64_t* words, uint32_t n, uint64_t m,
                          const uint64_t* col_index, uint64_t r_bits,
                          const uint8_t* f, uint64_t* out) {
  if (n == 0) return ORACLE_EINVAL;
#pragma omp parallel for schedule(static)
  for (int64_t c = 0; c < (int64_t)m; ++c) {
    uint32_t count[64];
    uint64_t mask = valid_mask(col_index[c], r_bits);
    for (int b = 0; b < 64; ++b) count[b] = 0;
    for (uint32_t j = 0; j < n; ++j) {
      uint64_t x = words[(uint64_t)j * m + (uint64_t)c] & mask;
      for (int b = 0; b < 64; ++b) count[b] += (uint32_t)((x >> b) & 1);
    }
    uint64_t o = 0;
    for (int b = 0; b < 64; ++b)
      if (f[count[b]]) o |= (uint64_t)1 << b;
    out[c] = o & mask;
  }
  return ORACLE_OK;
}

/* Threshold over a matrix of words (same layout as above): out bit is 1 iff
 * the number of inputs with that bit set is at least theta. */
int oracle_threshold_cols(const uint64_t* words, uint32_t n, uint64_t m,
                          const uint64_t* col_index, uint64_t r_bits,
                          uint32_t theta, uint64_t* out) {
  if (n == 0) return ORACLE_EINVAL;
#pragma omp parallel for schedule(static)
  for (int64_t c = 0; c < (int64_t)m; ++c) {
    uint32_t count[64];
    uint64_t mask = valid_mask(col_index[c], r_bits);
    for (int b = 0; b < 64; ++b) count[b] = 0;
    for (uint32_t j = 0; j < n; ++j) {
      uint64_t x = words[(uint64_t)j * m + (uint64_t)c] & mask;
      for (int b = 0; b < 64; ++b) count[b] += (uint32_t)((x >> b) & 1);
    }
    uint64_t o = 0;
    for (int b = 0; b < 64; ++b)
      if (count[b] >= theta) o |= (uint64_t)1 << b;
    out[c] = o & mask;
  }
  return ORACLE_OK;
}

/* Whole bitmaps given as an array of n pointers to ceil(r/64) words each. */
int oracle_threshold(const uint64_t* const* bitmaps, uint32_t n, uint64_t r_bits,
                     uint32_t theta, uint64_t* out) {
  if (n == 0) return ORACLE_EINVAL;
  uint64_t nw = words_for_bits(r_bits);
#pragma omp parallel for schedule(static)
  for (int64_t w = 0; w < (int64_t)nw; ++w) {
    uint32_t count[64];
    uint64_t mask = valid_mask((uint64_t)w, r_bits);
    for (int b = 0; b < 64; ++b) count[b] = 0;
    for (uint32_t j = 0; j < n; ++j) {
      uint64_t x = bitmaps[j][w] & mask;
      for (int b = 0; b < 64; ++b) count[b] += (uint32_t)((x >> b) & 1);
    }
    uint64_t o = 0;
    for (int b = 0; b < 64; ++b)
      if (count[b] >= theta) o |= (uint64_t)1 << b;
    out[w] = o & mask;
  }
  return ORACLE_OK;
}

int oracle_symmetric(const uint64_t* const* bitmaps, uint32_t n, uint64_t r_bits,
                     const uint8_t* f, uint64_t* out) {
  if (n == 0) return ORACLE_EINVAL;
  uint64_t nw = words_for_bits(r_bits);
#pragma omp parallel for schedule(static)
  for (int64_t w = 0; w < (int64_t)nw; ++w) {
    uint32_t count[64];
    uint64_t mask = valid_mask((uint64_t)w, r_bits);
    for (int b = 0; b < 64; ++b) count[b] = 0;
    for (uint32_t j = 0; j < n; ++j) {
      uint64_t x = bitmaps[j][w] & mask;
      for (int b = 0; b < 64; ++b) count[b] += (uint32_t)((x >> b) & 1);
    }
    uint64_t o = 0;
    for (int b = 0; b < 64; ++b)
      if (f[count[b]]) o |= (uint64_t)1 << b;
    out[w] = o & mask;
  }
  return ORACLE_OK;
}

/*
 * Weighted threshold (section 2.3: inputs may carry positive integer
 * weights): output bit p is 1 iff the sum of weights[j] over the inputs j
 * that have bit p set is at least theta.
 */
int oracle_weighted_threshold(const uint64_t* const* bitmaps, uint32_t n, const uint32_t* weights,
                              uint64_t r_bits, uint64_t theta, uint64_t* out) {
  if (n == 0) return ORACLE_EINVAL;
  uint64_t nw = words_for_bits(r_bits);
#pragma omp parallel for schedule(static)
  for (int64_t w = 0; w < (int64_t)nw; ++w) {
    uint64_t sum[64];
    uint64_t mask = valid_mask((uint64_t)w, r_bits);
    for (int b = 0; b < 64; ++b) sum[b] = 0;
    for (uint32_t j = 0; j < n; ++j) {
      uint64_t x = bitmaps[j][w] & mask;
      for (int b = 0; b < 64; ++b)
        if ((x >> b) & 1) sum[b] += weights[j];
    }
    uint64_t o = 0;
    for (int b = 0; b < 64; ++b)
      if (sum[b] >= theta) o |= (uint64_t)1 << b;
    out[w] = o & mask;
  }
  return ORACLE_OK;
}

/* Number of positions p < r whose bit is set (the cardinality of a result
 * bitmap, counted one position at a time). */
uint64_t oracle_count(const uint64_t* words, uint64_t r_bits) {
  uint64_t c = 0;
  for (uint64_t p = 0; p < r_bits; ++p) c += (words[p / 64] >> (p % 64)) & 1;
  return c;
}

/* Threads of the OpenMP loops above (timing only; results do not depend on it). */
void oracle_set_threads(int n) {
  if (n > 0) omp_set_num_threads(n);
}

int oracle_max_threads(void) { return omp_get_max_threads(); }

/* ------------------------------------------------------------------ RLE */

static uint64_t marker_fill(uint64_t m) { return m & 1; }
static uint64_t marker_run(uint64_t m) { return (m >> 1) & 0xFFFFFFFFull; }
static uint64_t marker_lits(uint64_t m) { return m >> 33; }

static uint64_t make_marker(uint64_t fill, uint64_t run, uint64_t lits) {
  return (fill & 1) | (run << 1) | (lits << 33);
}

/*
 * Decode a stream of len words into nwords dense words.  Returns
 * ORACLE_EFORMAT when the stream does not cover exactly nwords words or a
 * marker's literals run past the end of the stream.
 */
int oracle_rle_decode(const uint64_t* s, uint64_t len, uint64_t nwords, uint64_t* out) {
  uint64_t pos = 0, w = 0;
  while (pos < len) {
    uint64_t m = s[pos++];
    uint64_t fill = marker_fill(m), run = marker_run(m), lits = marker_lits(m);
    if (run > nwords - w) return ORACLE_EFORMAT;
    for (uint64_t k = 0; k < run; ++k) out[w++] = fill ? ~(uint64_t)0 : 0;
    if (lits > nwords - w) return ORACLE_EFORMAT;
    if (lits > len - pos) return ORACLE_EFORMAT;
    for (uint64_t k = 0; k < lits; ++k) out[w++] = s[pos++];
  }
  if (w != nwords) return ORACLE_EFORMAT;
  return ORACLE_OK;
}

static int word_kind(uint64_t x) {  /* 0: zero fill, 1: ones fill, 2: dirty */
  if (x == 0) return 0;
  if (x == ~(uint64_t)0) return 1;
  return 2;
}

/*
 * Canonical encoding of nwords dense words of an r-bit bitmap (bits >= r are
 * cleared first).  Writes at most cap words to out (out may be NULL) and
 * returns the full encoded length.
 */
uint64_t oracle_rle_encode(const uint64_t* dense, uint64_t r_bits, uint64_t* out, uint64_t cap) {
  uint64_t nw = words_for_bits(r_bits);
  uint64_t len = 0, w = 0;
  while (w < nw) {
    uint64_t x = dense[w] & valid_mask(w, r_bits);
    int kind = word_kind(x);
    uint64_t fill = 0, run = 0, lits = 0;
    if (kind != 2) {
      fill = (uint64_t)kind;
      while (w < nw && word_kind(dense[w] & valid_mask(w, r_bits)) == kind) { ++run; ++w; }
    }
    uint64_t lit_start = w;
    while (w < nw && word_kind(dense[w] & valid_mask(w, r_bits)) == 2) { ++lits; ++w; }
    if (out && len < cap) out[len] = make_marker(fill, run, lits);
    ++len;
    for (uint64_t k = 0; k < lits; ++k) {
      if (out && len < cap) out[len] = dense[lit_start + k] & valid_mask(lit_start + k, r_bits);
      ++len;
    }
  }
  return len;
}

/* Number of runs of equal bits in positions 0..r-1 (the RunCount of one bitmap). */
uint64_t oracle_run_count(const uint64_t* dense, uint64_t r_bits) {
  if (r_bits == 0) return 0;
  uint64_t runs = 1;
  int prev = (int)(dense[0] & 1);
  for (uint64_t p = 1; p < r_bits; ++p) {
    int b = (int)((dense[p / 64] >> (p % 64)) & 1);
    if (b != prev) { ++runs; prev = b; }
  }
  return runs;
}
