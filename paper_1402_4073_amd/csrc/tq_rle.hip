// Run-length-encoded inputs and outputs (word-aligned RLE, section 2.1).
//
// Stream format: a sequence of marker words, each followed by its literal
// words.  Marker: bit 0 = fill value, bits 1..32 = number of fill words,
// bits 33..63 = number of literal (dirty) words that follow.
//
// Threshold over RLE inputs, one workgroup per tile of kTile words:
//
//  1. Every input is entered at the tile through its checkpoint index (one
//     entry per kTile uncompressed words: stream offset and start word of the
//     marker covering the checkpoint) and its markers are walked, one lane per
//     input.  Fill runs of ones add 1 to k (per column) and literal runs add 1
//     to d, both through a difference array in LDS; no literal word is read.
//  2. After a prefix sum, every column knows k (inputs that are a 1-fill there)
//     and d (inputs that are dirty there).  These are the cases of RBMrg
//     (section 4.1): theta - k <= 0 means the column is all ones, theta - k > d
//     means all zeros, and only in between do the dirty words matter, as a
//     (theta - k)-threshold over them.
//  3. The markers are walked again and only the literal words of undecided
//     columns are read and added into a bit-sliced counter per column kept in
//     LDS.  Lanes of different inputs may hit the same column, so the addition
//     ripples with atomic XOR: the old value that atomicXor returns gives the
//     exact carry of that addition whatever the interleaving.
//  4. One thread per column compares its counter with its own theta - k
//     (subtract-and-sign style, bit by bit with a per-lane mask), adds any
//     uncompressed inputs first (hybrid queries), and writes the dense word.
//
// The dense result is then encoded canonically: each word is classified
// (zero fill, ones fill, dirty), a marker starts at word 0 and at each clean
// word after a dirty word or a different fill, and one scan of the packed pair
// (markers, dirty words) before each word gives every output position.
#include <mutex>
#include <type_traits>

#include "tq_csa.hpp"

namespace tq {
namespace {

constexpr int kTile = TQ_RLE_INDEX_STRIDE;  // words per tile == checkpoint stride
constexpr uint32_t kXcds = 8;                // accelerator complex dies per device
constexpr int kTileThreads = 512;
// columns needing literal words in a tile from which on the next tile is done
// in one pass
constexpr int kOnePassColumns = kTile / 16;
// tiles whose k and d one marker walk gathers (spans without literal words)
constexpr int kSpan = 8;
// tiles a one-pass walk covers when the counters are at most 2 planes (their
// LDS then holds the counters of that many tiles)
constexpr int kOnePassSpan = 4;
__host__ __device__ constexpr int plane_tiles(int K, bool swar) { return (!swar && K <= 2) ? kOnePassSpan : 1; }
static_assert(kTile == kTileThreads && kTile % kSpan == 0, "phase 2 gives each thread kSpan columns of one tile");
constexpr int kEncBlock = 256;
constexpr int kEncPerThread = 8;
constexpr int kEncWords = kEncBlock * kEncPerThread;
static_assert(kEncWords % kTile == 0 && kEncWords / kTile <= kEncBlock, "whole checkpoint strides per encoder block");

__device__ __forceinline__ void set_status(int* status, int code) { atomicCAS(status, 0, code); }

__device__ __forceinline__ uint64_t valid_mask_dev(uint64_t w, uint64_t nwords, uint64_t tail_mask) {
  return w == nwords - 1 ? tail_mask : ~(uint64_t)0;
}

// --------------------------------------------------------- block scans
// inclusive scan of one value per thread over a 512-thread block (8 waves)
template <typename T>
__device__ __forceinline__ T wave_inclusive_scan(T v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    T o = __shfl_up(v, off, 64);
    if (lane >= off) v += o;
  }
  return v;
}

// The same for 32-bit values, with the permute indices derived from a lane
// number the compiler cannot hoist: in the tile loop the hoisted indices of
// the six steps would stay live across the stream walks and spill.
template <>
__device__ __forceinline__ int32_t wave_inclusive_scan<int32_t>(int32_t v) {
  int lane = threadIdx.x & 63;
  asm volatile("" : "+v"(lane));
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int32_t o = __builtin_amdgcn_ds_bpermute((lane - off) << 2, v);
    if (lane >= off) v += o;
  }
  return v;
}

template <typename T, int WAVES>
__device__ __forceinline__ T block_exclusive_scan(T v, T* wave_tot, T* total) {
  // (lane and wave derived here, not hoisted out of the tile loop of the caller)
  int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  asm volatile("" : "+v"(lane), "+v"(wave));
  T inc = wave_inclusive_scan(v);
  if (lane == 63) wave_tot[wave] = inc;
  __syncthreads();
  if (wave == 0) {
    T t = lane < WAVES ? wave_tot[lane] : (T)0;
    T ti = wave_inclusive_scan(t);
    if (lane < WAVES) wave_tot[lane] = ti - t;
    if (lane == WAVES - 1) *total = ti;
  }
  __syncthreads();
  T r = inc - v + wave_tot[wave];
  __syncthreads();
  return r;
}

// ------------------------------------------------------------ tile kernel
// Positions inside the kernel are 32-bit: the host admits only bitmaps of
// fewer than 2^32 - kTile words and streams of fewer than 2^32 words.
struct Walk {
  uint32_t pos, w;   // stream offset of a marker, uncompressed word where its run starts
};

// Enter a stream at the checkpoint of `tile`; returns false on a bad entry.
__device__ __forceinline__ bool seek(const RleDesc& d, uint32_t tile, uint32_t t0, Walk& wk) {
  const uint64_t pos = d.index[2 * (uint64_t)tile], w = d.index[2 * (uint64_t)tile + 1];
  wk.pos = (uint32_t)pos;
  wk.w = (uint32_t)w;
  return pos < d.len && w <= t0;
}

template <int K>
__device__ __forceinline__ void ripple_lds(uint64_t* planes, int col, uint64_t x) {
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const uint64_t old = atomicXor((unsigned long long*)&planes[k * kTile + col], (unsigned long long)x);
    x &= old;
    if (!x) break;
  }
}

// The same with a sticky top plane: planes 0..K-2 count exactly up to
// 2^(K-1) - 1, and the carry out of them sets plane K-1 for good, which then
// means "at least 2^(K-1)".  A threshold query needs nothing more when every
// column's threshold theta - k stays below 2^(K-1): a set top plane answers
// yes, a clear one leaves an exact count.
template <int K>
__device__ __forceinline__ void ripple_lds_sat(uint64_t* planes, int col, uint64_t x) {
#pragma unroll
  for (int k = 0; k < K - 1; ++k) {
    const uint64_t old = atomicXor((unsigned long long*)&planes[k * kTile + col], (unsigned long long)x);
    x &= old;
    if (!x) return;
  }
  atomicOr((unsigned long long*)&planes[(K - 1) * kTile + col], (unsigned long long)x);
}

// kd word of a column after the scan: bits 0..15 k (ones fills), bits 16..30
// d (dirty inputs), bit 31 set when the column is undecided
__device__ __forceinline__ void unpack_kd(int32_t v, int& k, int& d) {
  k = v & 0xFFFF;
  d = (v >> 16) & 0x7FFF;
}

// P += k for a per-lane constant k (bit-sliced ripple; the sum fits in K planes)
template <int K>
__device__ __forceinline__ void add_constant(uint64_t (&P)[K], uint32_t k) {
  uint64_t carry = 0;
#pragma unroll
  for (int q = 0; q < K; ++q) {
    const uint64_t kb = 0 - (uint64_t)((k >> q) & 1u);
    const uint64_t x = P[q] ^ kb;
    const uint64_t c2 = (P[q] & kb) | (carry & x);
    P[q] = x ^ carry;
    carry = c2;
  }
}

// count > a per lane (a differs between lanes), counter in registers
template <int K>
__device__ __forceinline__ uint64_t greater_than_lane(const uint64_t (&P)[K], uint32_t a) {
  uint64_t pm = ~(uint64_t)0, r = 0;
#pragma unroll
  for (int j = K - 1; j >= 0; --j) {
    const uint64_t m = 0 - (uint64_t)((a >> j) & 1u);  // all ones where a has a one
    r |= pm & P[j] & ~m;
    pm &= P[j] | ~m;
  }
  return r;
}

// the same comparison reading the counter planes of column c from LDS
template <int K>
__device__ __forceinline__ uint64_t greater_than_lds(const uint64_t* planes, int c, uint32_t a) {
  uint64_t pm = ~(uint64_t)0, r = 0;
#pragma unroll
  for (int j = K - 1; j >= 0; --j) {
    const uint64_t p = planes[j * kTile + c];
    const uint64_t m = 0 - (uint64_t)((a >> j) & 1u);
    r |= pm & p & ~m;
    pm &= p | ~m;
  }
  return r;
}

// Column counters of the literal words, kept in LDS.
//
// Bit-sliced: K planes per column; a word is added by a ripple of atomic
// XORs whose returned old values give the carries (see ripple_lds).  K x 4 KiB
// per tile, but each addition waits for its LDS round trips.
//
// Column c of a walk counts from the first tile of the walk; the counters of
// each tile are a block of their own (K x kTile words), so a walk over several
// tiles (one-pass spans) addresses block c / kTile.
template <int K>
struct SlicedAdd {
  uint64_t* planes;
  __device__ __forceinline__ void operator()(int c, uint64_t x) const {
    ripple_lds<K>(planes + (c / kTile) * (K * kTile), c % kTile, x);
  }
};

template <int K>
struct SaturatingAdd {
  uint64_t* planes;
  __device__ __forceinline__ void operator()(int c, uint64_t x) const {
    ripple_lds_sat<K>(planes + (c / kTile) * (K * kTile), c % kTile, x);
  }
};

// Parity needs only bit 0 of each count: one plane, one XOR per word, and no
// old value to wait for.
struct ParityAdd {
  uint64_t* planes;
  __device__ __forceinline__ void operator()(int c, uint64_t x) const {
    atomicXor((unsigned long long*)&planes[c], (unsigned long long)x);
  }
};

// Counter forms of the plane kernels (Swar = false)
constexpr int kFullPlanes = 0;    // K planes holding the exact count
constexpr int kSaturating = 1;    // top plane sticky (ripple_lds_sat): thresholds, and
                                  // symmetric f constant from some count on
constexpr int kParityPlane = 2;   // parity: one plane, the count modulo 2

// SWAR: 16 words per column, word q holding the 16-bit counts of positions
// q, q + 16, q + 32 and q + 48; a word x is added with 16 atomic adds of
// (x >> q) & E, none of which returns a value, so nothing waits on LDS.  The
// counts never exceed the number of inputs (< 2^16), so no field carries
// into the next.  64 KiB per tile.
constexpr uint64_t kSwarE = 0x0001000100010001ull;
constexpr uint64_t kSwarH = 0x8000800080008000ull;
struct SwarAdd {
  uint64_t* cnt;   // [16][kTile]
  __device__ __forceinline__ void operator()(int c, uint64_t x) const {
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const uint64_t v = (x >> q) & kSwarE;
      if (v) atomicAdd((unsigned long long*)&cnt[q * kTile + c], (unsigned long long)v);
    }
  }
};

// Sequential reader of one stream.  A lane walking its stream one marker at a
// time would keep a cache line of its own open for the whole walk; with every
// lane of the device doing so, the lines no longer fit in L2 and are fetched
// again and again.  The reader instead loads the whole sector of W words
// holding the word it needs into registers and serves the following words
// from there, so each sector is fetched once per walk.  A sector never
// crosses a page boundary, so loading all of it is safe whenever one of its
// words belongs to the stream; words outside the stream are never returned.
//
// W = 8 (64 bytes) suits walks that mostly only read markers: a lane then
// holds half of a 128-byte line, and the other half is often still in L2
// when the walk gets there.  W = 4 (32 bytes) suits walks that count most
// literal words: fewer registers and a shorter select per word, at the cost
// of lines fetched more often (up to four times).
template <int W>
struct SectorReader {
  static_assert(W == 4 || W == 8, "sectors of 4 or 8 words");
  const uint64_t* base;   // W * 8-byte aligned, at or below the stream start
  uint32_t off;           // words from base to the stream start (0..W-1)
  uint32_t cur;           // sector held (counted from base); kNone if none
  uint64_t b[W];
  static constexpr uint32_t kNone = 0xFFFFFFFFu;

  __device__ __forceinline__ void reset(const uint64_t* w, uint64_t) {
    const uintptr_t a = reinterpret_cast<uintptr_t>(w);
    base = reinterpret_cast<const uint64_t*>(a & ~(uintptr_t)(W * 8 - 1));
    off = (uint32_t)(a >> 3) & (uint32_t)(W - 1);
    cur = kNone;
  }
  __device__ __forceinline__ uint64_t at(uint32_t p) {
    const uint32_t g = off + p;
    const uint32_t sec = g / W;
    if (sec != cur) {
      // global address space: the loads wait on the vector memory counter
      // only, not on LDS operations still in flight
      typedef unsigned int U32x4 __attribute__((ext_vector_type(4)));
      typedef const __attribute__((address_space(1))) U32x4 GlobalSector;
      GlobalSector* q = (GlobalSector*)(base + (uint64_t)sec * W);
      U32x4 v[W / 2];
#pragma unroll
      for (int u = 0; u < W / 2; ++u) v[u] = q[u];
#pragma unroll
      for (int u = 0; u < W / 2; ++u) {
        b[2 * u] = v[u].x | ((uint64_t)v[u].y << 32);
        b[2 * u + 1] = v[u].z | ((uint64_t)v[u].w << 32);
      }
      cur = sec;
    }
    const unsigned i = g % W;
    const uint64_t x01 = (i & 1) ? b[1] : b[0], x23 = (i & 1) ? b[3] : b[2];
    const uint64_t x03 = (i & 2) ? x23 : x01;
    if constexpr (W == 4) {
      return x03;
    } else {
      const uint64_t x45 = (i & 1) ? b[5] : b[4], x67 = (i & 1) ? b[7] : b[6];
      const uint64_t x47 = (i & 2) ? x67 : x45;
      return (i & 4) ? x47 : x03;
    }
  }
};

// Word-at-a-time reader for the inputs past the first kTileThreads (few
// queries have them; a sector buffer for them would cost occupancy).
struct DirectReader {
  const uint64_t* words;
  __device__ __forceinline__ void reset(const uint64_t* w, uint64_t) { words = w; }
  __device__ __forceinline__ uint64_t at(uint32_t p) const { return words[p]; }
};

// Decode the marker at wk.pos and check it against the stream and the bitmap;
// on success w1 / w2 are the ends of its fill and literal runs.
template <typename Reader>
__device__ __forceinline__ bool read_marker(uint32_t len, Reader& rd, const Walk& wk, uint32_t nwords,
                                            uint64_t& m, uint32_t& w1, uint32_t& w2) {
  if (wk.pos >= len) return false;
  m = rd.at(wk.pos);
  const uint64_t run = (m >> 1) & 0xFFFFFFFFull, lits = m >> 33;
  const uint64_t e1 = (uint64_t)wk.w + run, e2 = e1 + lits;
  if (e2 > nwords || lits > len - wk.pos - 1) return false;
  w1 = (uint32_t)e1;
  w2 = (uint32_t)e2;
  return true;
}

// Marker walk of one input over [t0, t1): fills of ones and literal runs go
// into the difference array; with `lits` the literal words are also added to
// the column counters right away (the one-pass form of a tile).  On return
// `next` is the entry state of the following tile (the marker covering t1).
template <typename Add, typename Reader>
__device__ __forceinline__ void walk_markers(uint32_t len, Reader& rd, Walk wk, uint32_t t0, uint32_t t1,
                                             uint32_t nwords, int32_t* kd, int* status, bool lits,
                                             const Add& add, Walk& next) {
  next = wk;
  while (wk.w < t1) {
    uint64_t m;
    uint32_t w1, w2;
    if (!read_marker(len, rd, wk, nwords, m, w1, w2)) { set_status(status, TQ_EFORMAT); break; }
    if ((m & 1) && w1 > wk.w) {
      const uint32_t a = wk.w > t0 ? wk.w : t0, b = w1 < t1 ? w1 : t1;
      if (a < b) {
        atomicAdd(&kd[a - t0], 1);
        atomicSub(&kd[b - t0], 1);
      }
    }
    if (w2 > w1) {
      const uint32_t a = w1 > t0 ? w1 : t0, b = w2 < t1 ? w2 : t1;
      if (a < b) {
        atomicAdd(&kd[a - t0], 65536);
        atomicSub(&kd[b - t0], 65536);
        if (lits)
          for (uint32_t col = a; col < b; ++col)
            add((int)(col - t0), rd.at(wk.pos + 1 + (col - w1)));
      }
    }
    // a marker reaching past t1 is where the next tile enters this stream
    if (w2 > t1) {
      next = wk;
      return;
    }
    wk.pos += 1 + (w2 - w1);
    wk.w = w2;
    next = wk;
  }
}

// Literal words of the undecided columns of [t0, t1) into the LDS counters.
template <typename Add, typename Reader>
__device__ __forceinline__ void walk_literals(uint32_t len, Reader& rd, Walk wk, uint32_t t0, uint32_t t1,
                                              uint32_t nwords, const int32_t* kd, const Add& add) {
  while (wk.w < t1) {
    uint64_t m;
    uint32_t w1, w2;
    if (!read_marker(len, rd, wk, nwords, m, w1, w2)) break;
    const uint32_t a = w1 > t0 ? w1 : t0, b = w2 < t1 ? w2 : t1;
    for (uint32_t col = a; col < b; ++col) {
      const int c = (int)(col - t0);
      if (kd[c] < 0) add(c, rd.at(wk.pos + 1 + (col - w1)));
    }
    wk.pos += 1 + (w2 - w1);
    wk.w = w2;
  }
}

// Dense inputs of a hybrid query at word col, handed to f in groups of
// kDenseGroup whose loads are all in flight together (a load per input, each
// waiting for the one before, would cost a memory round trip per input).
// Past the last input f is handed zero words, which add nothing to a count.
constexpr uint32_t kDenseGroup = 8;
template <typename F>
__device__ __forceinline__ void for_dense_words(const uint64_t* const* dense, uint32_t n_dense, uint64_t col,
                                                F&& f) {
  for (uint32_t i = 0; i < n_dense; i += kDenseGroup) {
    uint64_t x[kDenseGroup];
#pragma unroll
    for (uint32_t u = 0; u < kDenseGroup; ++u) x[u] = i + u < n_dense ? dense[i + u][col] : 0;
#pragma unroll
    for (uint32_t u = 0; u < kDenseGroup; ++u) f(x[u]);
  }
}

// One workgroup processes a contiguous range of tiles.  The lane that owns
// input j < kTileThreads carries its stream position (and its reader) from
// one tile to the next, so a range reads each of its streams once, front to
// back, and enters through the checkpoint index only at the range start;
// further inputs (more than one per lane) enter every tile through the index.
//
// Sym = false: threshold theta (the RBMrg run cases of section 4.1: with k
// ones fills, theta - k <= 0 gives ones and theta - k > d zeros).  Sym = true:
// any symmetric f, decided where f is constant on [k, k + d] and otherwise
// evaluated on k plus the counted dirty bits.  Swar = true: SWAR column
// counters, every tile in one pass; otherwise K bit-sliced planes in the
// form Form: kSaturating makes the top plane sticky (see ripple_lds_sat), so
// K = bit_length(theta - 1) + 1 planes suffice for a threshold, and
// bit_length(tail_from) + 1 for a symmetric f constant from tail_from on;
// kParityPlane (the parity function and its complement) keeps one plane, the
// count modulo 2.  With K <= 4 planes (K <= 9 for plain thresholds, K <= 5
// for symmetric functions) the kernel is built for 8 waves per SIMD (how
// many are resident is then set by the LDS footprint: 3 or 4 workgroups per
// CU); the plain-threshold builds fit in those 64 registers without spilling
// (each lane keeps only its stream's length and reader, and is entered
// through the index once per range), the others spill a few registers,
// reloaded once per tile.
//
// Fused = true: consumers of each result word (sink): AND with a filter, and a
// count; each thread sums the popcounts of its words over the range, and each
// wave writes one partial count per workgroup (blockIdx.x * 8 + wave).
//
// Hybrid = true: n_dense uncompressed inputs are added column by column in
// step 4 (their loads batched, see for_dense_words); the other builds ignore
// n_dense and keep no registers for it.
template <int K, bool Sym, bool Swar, int Form = kFullPlanes, bool Fused = false, bool Hybrid = false>
__global__ __launch_bounds__(kTileThreads) __attribute__((amdgpu_waves_per_eu(
    ((Form != kFullPlanes && K <= 4) || (!Swar && !Fused && !Hybrid && K <= (Sym ? 5 : 9))) ? 8 : 6))) void rle_tile_kernel(
    const RleDesc* __restrict__ descs, uint32_t n_rle, const uint64_t* const* __restrict__ dense,
    uint32_t n_dense_arg, uint32_t nwords, uint64_t tail_mask, uint32_t theta, const RleSym* __restrict__ sym,
    uint32_t tiles_per_group,
    uint64_t* out, int* __restrict__ status, Sink sink) {
  static_assert(!(Fused && Hybrid), "fused consumers take compressed inputs only");
  const uint32_t n_dense = Hybrid ? n_dense_arg : 0;
  extern __shared__ uint64_t lds[];
  constexpr int kCounterWords = Swar ? 16 : K;
  constexpr int kPlaneTiles = plane_tiles(K, Swar);
  // counters: a block of kCounterWords x kTile words per tile of a one-pass span
  uint64_t* planes = lds;
  int32_t* kd = reinterpret_cast<int32_t*>(lds + kCounterWords * kTile * kPlaneTiles);   // kSpan * kTile + 1 packed (k | d << 16)
  constexpr bool Sat = Form == kSaturating, Par = Form == kParityPlane;
  static_assert(!Sat || !Swar, "saturating planes are bit planes");
  static_assert(!Par || (Sym && !Swar && K == 1), "the parity plane serves the parity function only");
  using Add = typename std::conditional<
      Swar, SwarAdd,
      typename std::conditional<Sat, SaturatingAdd<K>,
                                typename std::conditional<Par, ParityAdd, SlicedAdd<K>>::type>::type>::type;
  const Add add{planes};
  __shared__ int32_t wave_tot[kTileThreads / 64];
  __shared__ int32_t total;
  __shared__ int32_t needs[kSpan];   // undecided columns with literal words, per tile of the span

  // Workgroups are dealt to the eight XCDs round robin; give each XCD a
  // contiguous block of ranges so that the cache lines two neighbouring
  // ranges share are fetched into one L2.
  const uint32_t tiles = (nwords + kTile - 1) / kTile;
  const uint32_t ranges = (tiles + tiles_per_group - 1) / tiles_per_group;
  const uint32_t per_xcd = (ranges + kXcds - 1) / kXcds;
  const uint32_t range = (blockIdx.x % kXcds) * per_xcd + blockIdx.x / kXcds;
  if (range >= ranges) {
    if (Fused && sink.partial64 && (threadIdx.x & 63) == 0)
      sink.partial64[(uint64_t)blockIdx.x * (kTileThreads / 64) + (threadIdx.x >> 6)] = 0;
    return;
  }
  uint64_t popcount_sum = 0;   // Fused: ones of this thread's result words
  const uint32_t tile_begin = range * tiles_per_group;
  const uint32_t tile_end = tiles - tile_begin > tiles_per_group ? tile_begin + tiles_per_group : tiles;
  const int tid = threadIdx.x;
  const bool own = (uint32_t)tid < n_rle;   // this lane carries input tid
  // The lane's stream is entered once, at the range start; a bad entry
  // leaves the lane out of the whole range (the launch reports TQ_EFORMAT).
  uint32_t my_len = 0;
  Walk carry = {0, 0};
  bool carry_ok = false;
  // 32-byte sectors for the plain symmetric builds of more than 2 planes,
  // whose walks mostly count literal words (and which then spill no
  // register); 64-byte sectors elsewhere
  SectorReader<(!Swar && !Fused && !Hybrid && Sym && K > 2) ? 4 : 8> rd;
  DirectReader rx;
  rd.reset(nullptr, 0);
  if (own) {
    const RleDesc mine = descs[tid];
    my_len = (uint32_t)mine.len;
    rd.reset(mine.words, mine.len);
    carry_ok = seek(mine, tile_begin, tile_begin * kTile, carry);
    if (!carry_ok) set_status(status, TQ_EFORMAT);
  }
  // Tiles whose literal words are mostly needed are done in one pass (the
  // marker walk adds every literal word to the counters), saving the second
  // walk at the cost of counting literal words of decided columns too.  The
  // others are taken kSpan at a time: one marker walk over the span fills
  // k and d of all its columns (a lane waits at a barrier once per span, not
  // once per tile, so streams with more markers in one tile and fewer in the
  // next even out), and only tiles with undecided columns walk again for
  // their literal words, entering each stream through the index.  The choice
  // follows the previous span of the range: neighbouring tiles of a bitmap
  // tend to look alike.  A range starts in one pass where that is the likely
  // choice: parity needs the literal words of every column that has any,
  // thresholds up to 2 those of every column with fewer than 2 fills, and a
  // symmetric f constant only from a small count on (at most 5 planes)
  // those of most columns of sparse inputs (and adds them cheaply).
  bool one_pass = Swar || Par || (!Sym && K <= 2) || (Sym && K <= 5);

  for (uint32_t ta = tile_begin; ta < tile_end;) {
    // (a range starting in two passes takes its first tile alone: its kind
    // is not known yet)
    const uint32_t span = one_pass ? (uint32_t)kPlaneTiles : (ta == tile_begin ? 1u : (uint32_t)kSpan);
    const uint32_t nb = tile_end - ta < span ? tile_end - ta : span;
    const uint32_t lo = ta * kTile;
    const uint32_t hi = nwords - lo > nb * kTile ? lo + nb * kTile : nwords;
    const uint32_t ncols = hi - lo;
    if (ta != tile_begin) __syncthreads();   // the previous span's phase 4 is done with the LDS
    for (int i = tid; i < kCounterWords * kTile * (one_pass ? (int)nb : 1); i += kTileThreads) planes[i] = 0;
    for (int i = tid; i <= (int)ncols; i += kTileThreads) kd[i] = 0;
    if (tid < kSpan) needs[tid] = 0;
    __syncthreads();

    // 1. markers only: difference array of (ones fills) + 65536 * (dirty)
    const Walk entry = carry;
    const bool entry_ok = carry_ok;
    if (entry_ok) walk_markers(my_len, rd, entry, lo, hi, nwords, kd, status, one_pass, add, carry);
    for (uint32_t j = tid + kTileThreads; j < n_rle; j += kTileThreads) {
      const RleDesc dsc = descs[j];
      Walk wk, unused;
      if (!seek(dsc, ta, lo, wk)) { set_status(status, TQ_EFORMAT); continue; }
      rx.reset(dsc.words, dsc.len);
      walk_markers((uint32_t)dsc.len, rx, wk, lo, hi, nwords, kd, status, one_pass, add, unused);
    }
    __syncthreads();

    // 2. prefix sum: kd[c] = k + 65536 * d for column c, flagged if undecided;
    // thread i takes columns [kSpan * i, kSpan * i + kSpan), all in one tile
    // (addresses derived from a thread number the compiler cannot hoist)
    {
      int me = tid;
      asm volatile("" : "+v"(me));
      int32_t v[kSpan];
      int32_t sum = 0;
#pragma unroll
      for (int q = 0; q < kSpan; ++q) {
        const uint32_t col = (uint32_t)me * kSpan + q;
        v[q] = col < ncols ? kd[col] : 0;
        sum += v[q];
      }
      int32_t run = block_exclusive_scan<int32_t, kTileThreads / 64>(sum, wave_tot, &total);
      int undecided = 0;
#pragma unroll
      for (int q = 0; q < kSpan; ++q) {
        const uint32_t col = (uint32_t)me * kSpan + q;
        run += v[q];
        if (col < ncols) {
          int k, d;
          unpack_kd(run, k, d);
          bool und;
          if constexpr (Sym) {
            und = (uint32_t)(k + d) + n_dense > sym->run_end[k];
          } else {
            const int tp = (int)theta - k;
            und = tp >= 1 && tp <= d + (int)n_dense;
          }
          // literal words matter where the column is undecided and has some
          undecided += (und && d > 0) ? 1 : 0;
          kd[col] = run | (und ? (int32_t)0x80000000 : 0);
        }
      }
      if (undecided) atomicAdd(&needs[(me * kSpan) / kTile], undecided);
    }
    __syncthreads();
    int need = 0;
    for (uint32_t b = 0; b < nb; ++b) need += needs[b];
    const bool span_one_pass = one_pass;
    one_pass = Swar || need >= kOnePassColumns * (int)nb;

    bool planes_used = false;   // the counters hold literal words of an earlier tile of the span
    for (uint32_t b = 0; b < nb; ++b) {
      const uint32_t tile = ta + b;
      const uint32_t t0 = lo + b * kTile;
      const uint32_t t1 = hi - t0 > (uint32_t)kTile ? t0 + kTile : hi;
      int32_t* const tkd = kd + (t0 - lo);
      // a tile whose columns the fills alone decide needs no literal word
      const bool walk_again = !span_one_pass && needs[b] > 0;
      // the tile's counters (one block per tile of a one-pass span)
      const uint64_t* tplanes = planes + (span_one_pass ? b * (kCounterWords * kTile) : 0);
      if (planes_used) {
        __syncthreads();   // the previous tile's phase 4 is done with the counters
        for (int i = tid; i < kCounterWords * kTile; i += kTileThreads) planes[i] = 0;
        __syncthreads();
        planes_used = false;
      }

      // 3. literal words of undecided columns into the per-column LDS counters
      if (walk_again) {
        if (entry_ok) {
          Walk e = entry;
          bool ok = true;
          if (b > 0) {
            // (the descriptor's address derived here, not held across the walks)
            int me = tid;
            asm volatile("" : "+v"(me));
            ok = seek(descs[me], tile, t0, e);
            if (!ok) set_status(status, TQ_EFORMAT);
          }
          if (ok) walk_literals(my_len, rd, e, t0, t1, nwords, tkd, add);
        }
        for (uint32_t j = tid + kTileThreads; j < n_rle; j += kTileThreads) {
          const RleDesc dsc = descs[j];
          Walk wk;
          if (!seek(dsc, tile, t0, wk)) continue;
          rx.reset(dsc.words, dsc.len);
          walk_literals((uint32_t)dsc.len, rx, wk, t0, t1, nwords, tkd, add);
        }
        planes_used = true;
      }
      __syncthreads();

    // 4. one column per thread: decide, or count and compare
    // (the column's LDS addresses are derived here, not kept live across the
    // walks, where the registers are needed)
    int c = tid;
    asm volatile("" : "+v"(c));
    if (c < (int)(t1 - t0)) {
      const int32_t v = tkd[c];
      int k, d;
      unpack_kd(v, k, d);
      uint64_t res;
      if (v >= 0) {
        // decided by the fills: f(k), resp. k >= theta
        bool one;
        if constexpr (Sym)
          one = (sym->f[k >> 6] >> (k & 63)) & 1;
        else
          one = k >= (int)theta;
        res = one ? ~(uint64_t)0 : 0;
      } else if constexpr (Swar) {
        uint64_t C[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) C[q] = tplanes[q * kTile + c];
        const uint64_t col = (uint64_t)t0 + c;
        if constexpr (Hybrid)
          for_dense_words(dense, n_dense, col, [&](uint64_t x) {
#pragma unroll
            for (int q = 0; q < 16; ++q) C[q] += (x >> q) & kSwarE;
          });
        res = 0;
        if constexpr (!Sym) {
          // count >= theta - k per 16-bit field: bit 15 of count + 2^15 - (theta - k)
          const uint64_t m = (uint64_t)(0x8000u - (theta - (uint32_t)k)) * kSwarE;
#pragma unroll
          for (int q = 0; q < 16; ++q) res |= ((C[q] + m) & kSwarH) >> (15 - q);
        } else {
#pragma unroll
          for (int p = 0; p < 64; ++p) {
            const uint32_t tot = (uint32_t)k + (uint32_t)((C[p & 15] >> (16 * (p >> 4))) & 0xFFFF);
            res |= ((sym->f[tot >> 6] >> (tot & 63)) & 1) << p;
          }
        }
      } else if (!Sym && !Hybrid) {
        res = greater_than_lds<K>(tplanes, c, theta - (uint32_t)k - 1);
      } else {
        uint64_t P[K];
#pragma unroll
        for (int q = 0; q < K; ++q) P[q] = tplanes[q * kTile + c];
        const uint64_t col = (uint64_t)t0 + c;
        if constexpr (Hybrid)
          for_dense_words(dense, n_dense, col, [&](uint64_t x) {
#pragma unroll
            for (int q = 0; q < (Sat ? K - 1 : K); ++q) {
              const uint64_t t = P[q] & x;
              P[q] ^= x;
              x = t;
            }
            if constexpr (Sat) P[K - 1] |= x;
          });
        if constexpr (Par) {
          // bit 0 of the count: the ones fills' parity and the counted bits'
          res = P[0] ^ ((k & 1) ? ~(uint64_t)0 : 0);
          if (sym->epi.invert) res = ~res;
        } else if constexpr (Sym && Sat) {
          // An undecided column has k < tail_from, so with the sticky plane
          // clear the count k + (exact planes) is below 2^K and exact; a set
          // sticky plane means at least 2^(K-1) > tail_from counted bits,
          // where f is tail_value.
          const uint64_t sticky = P[K - 1];
          P[K - 1] = 0;
          add_constant<K>(P, (uint32_t)k);
          csa::Vec<1> V[K];
#pragma unroll
          for (int q = 0; q < K; ++q) V[q].w[0] = P[q];
          res = csa::epilogue<K, 1>(V, sym->epi, n_rle + n_dense, sym->epi.table).w[0];
          res = (res & ~sticky) | (sym->tail_value ? sticky : 0);
        } else if constexpr (Sym) {
          // the full count of the column: its ones fills plus the counted bits
          add_constant<K>(P, (uint32_t)k);
          csa::Vec<1> V[K];
#pragma unroll
          for (int q = 0; q < K; ++q) V[q].w[0] = P[q];
          res = csa::epilogue<K, 1>(V, sym->epi, n_rle + n_dense, sym->epi.table).w[0];
        } else {
          res = greater_than_lane<K>(P, theta - (uint32_t)k - 1);
        }
      }
      uint64_t word = res & valid_mask_dev((uint64_t)t0 + c, nwords, tail_mask);
      if constexpr (Fused) {
        // consumers: AND filter (it may be out itself: read before the store)
        if (sink.filter) word &= sink.filter[(uint64_t)t0 + c];
        if (out) out[(uint64_t)t0 + c] = word;
        popcount_sum += (uint64_t)__popcll(word);
      } else {
        out[(uint64_t)t0 + c] = word;
      }
    }
    }
    ta += nb;
  }
  if constexpr (Fused) {
    if (sink.partial64) {
      // a wave's range may hold up to 2^34 ones: 64-bit partial counts
      uint64_t pc = popcount_sum;
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) pc += __shfl_xor(pc, off, 64);
      if ((tid & 63) == 0) sink.partial64[(uint64_t)blockIdx.x * (kTileThreads / 64) + (tid >> 6)] = pc;
    }
  }
}

// ------------------------------------------------------------- encoder
// kind: 0 zero fill, 1 ones fill, 2 dirty
__device__ __forceinline__ int word_kind(uint64_t x) {
  return x == 0 ? 0 : (x == ~(uint64_t)0 ? 1 : 2);
}

struct EncArgs {
  const uint64_t* dense;
  uint64_t nwords;
  uint64_t tail_mask;
  uint64_t* block_sums;   // per block: (markers << 32) | dirty
  uint32_t* seg_start;    // per marker: first word
  uint32_t* seg_d0;       // per marker: dirty words before it
  uint32_t* chk_marker;   // per checkpoint: marker covering it
  uint64_t* totals;       // [0] = (markers << 32) | dirty
  uint64_t* out;
  uint64_t cap;
  uint64_t* out_len;
  uint64_t* index;        // optional: 2 words per checkpoint
  int* status;
};

__device__ __forceinline__ uint64_t enc_word(const EncArgs& a, uint64_t w) {
  return a.dense[w] & valid_mask_dev(w, a.nwords, a.tail_mask);
}

// The kEncPerThread consecutive words of a thread from `base` on, bits past r
// cleared (words past the bitmap read as zero and contribute nothing), and
// the packed contribution of each: (is a marker start) << 32 | (is dirty).
// Every load, the word before `base` included, is issued before any is used.
__device__ __forceinline__ void enc_span(const EncArgs& a, uint64_t base, uint64_t (&x)[kEncPerThread],
                                         uint64_t (&c)[kEncPerThread]) {
  const bool whole = base + kEncPerThread <= a.nwords;
  uint64_t before = 0;   // the word before base (never the last word, so never masked)
  if (whole) {
    before = a.dense[base > 0 ? base - 1 : 0];
#pragma unroll
    for (int q = 0; q < kEncPerThread; ++q) x[q] = a.dense[base + q];
  } else {
    if (base > 0 && base <= a.nwords) before = a.dense[base - 1];
#pragma unroll
    for (int q = 0; q < kEncPerThread; ++q) x[q] = base + q < a.nwords ? a.dense[base + q] : 0;
  }
#pragma unroll
  for (int q = 0; q < kEncPerThread; ++q)
    if (base + q == a.nwords - 1) x[q] &= a.tail_mask;
  int kind[kEncPerThread];
#pragma unroll
  for (int q = 0; q < kEncPerThread; ++q) kind[q] = word_kind(x[q]);
  int kp = word_kind(before);
#pragma unroll
  for (int q = 0; q < kEncPerThread; ++q) {
    const int kc = kind[q];
    const uint64_t start = (base + q == 0) ? 1 : (kc != 2 && (kp == 2 || kp != kc) ? 1 : 0);
    c[q] = base + q < a.nwords ? (start << 32) | (kc == 2 ? 1u : 0u) : 0;
    kp = kc;
  }
}

__global__ __launch_bounds__(kEncBlock) void enc_reduce_kernel(EncArgs a) {
  __shared__ uint64_t wave_tot[kEncBlock / 64];
  const uint64_t base = (uint64_t)blockIdx.x * kEncWords + (uint64_t)threadIdx.x * kEncPerThread;
  uint64_t x[kEncPerThread], c[kEncPerThread];
  enc_span(a, base, x, c);
  uint64_t s = 0;
#pragma unroll
  for (int q = 0; q < kEncPerThread; ++q) s += c[q];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if ((threadIdx.x & 63) == 0) wave_tot[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint64_t t = 0;
#pragma unroll
    for (int w = 0; w < kEncBlock / 64; ++w) t += wave_tot[w];
    a.block_sums[blockIdx.x] = t;
  }
}

// exclusive scan of the block sums (one workgroup), totals and output length
__global__ __launch_bounds__(1024) void enc_scan_kernel(EncArgs a, uint64_t nblocks) {
  __shared__ uint64_t wave_tot[16];
  __shared__ uint64_t total;
  uint64_t carry = 0;
  for (uint64_t b0 = 0; b0 < nblocks; b0 += 1024) {
    const uint64_t b = b0 + threadIdx.x;
    const uint64_t v = b < nblocks ? a.block_sums[b] : 0;
    const uint64_t ex = block_exclusive_scan<uint64_t, 16>(v, wave_tot, &total);
    if (b < nblocks) a.block_sums[b] = ex + carry;
    carry += total;
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    a.totals[0] = carry;
    const uint64_t len = (carry >> 32) + (carry & 0xFFFFFFFFull);
    *a.out_len = len;
    if (len > a.cap) set_status(a.status, TQ_ECAPACITY);
  }
}

__global__ __launch_bounds__(kEncBlock) void enc_scatter_kernel(EncArgs a) {
  __shared__ uint64_t wave_tot[kEncBlock / 64];
  __shared__ uint64_t total;
  // A block without marker starts and dirty words (its sum, the difference of
  // two exclusive prefixes, is zero) lies inside the marker that covers its
  // first word: only its checkpoints are written, and its words are not read.
  const uint64_t pre_block = a.block_sums[blockIdx.x];
  const uint64_t next_block = blockIdx.x + 1 < gridDim.x ? a.block_sums[blockIdx.x + 1] : a.totals[0];
  if (next_block == pre_block) {
    const uint64_t w = (uint64_t)blockIdx.x * kEncWords + (uint64_t)threadIdx.x * kTile;
    if (threadIdx.x < kEncWords / kTile && w < a.nwords) a.chk_marker[w / kTile] = (uint32_t)((pre_block >> 32) - 1);
    return;
  }
  const uint64_t base = (uint64_t)blockIdx.x * kEncWords + (uint64_t)threadIdx.x * kEncPerThread;
  uint64_t x[kEncPerThread], c[kEncPerThread];
  enc_span(a, base, x, c);
  uint64_t s = 0;
#pragma unroll
  for (int q = 0; q < kEncPerThread; ++q) s += c[q];
  uint64_t pre = block_exclusive_scan<uint64_t, kEncBlock / 64>(s, wave_tot, &total) + pre_block;
#pragma unroll
  for (int q = 0; q < kEncPerThread; ++q) {
    const uint64_t w = base + q;
    if (w >= a.nwords) break;
    const uint64_t ms = pre >> 32, ds = pre & 0xFFFFFFFFull;
    const uint64_t st = c[q] >> 32;
    if (st) {
      a.seg_start[ms] = (uint32_t)w;
      a.seg_d0[ms] = (uint32_t)ds;
    }
    if (w % kTile == 0) a.chk_marker[w / kTile] = (uint32_t)(ms + st - 1);
    if (c[q] & 1) {
      const uint64_t pos = ms + ds + st;
      if (pos < a.cap) a.out[pos] = x[q];
    }
    pre += c[q];
  }
}

__global__ void enc_marker_kernel(EncArgs a) {
  const uint64_t tot = a.totals[0];
  const uint64_t M = tot >> 32, D = tot & 0xFFFFFFFFull;
  for (uint64_t m = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; m < M;
       m += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t s = a.seg_start[m];
    const uint64_t s1 = m + 1 < M ? a.seg_start[m + 1] : a.nwords;
    const uint64_t d0 = a.seg_d0[m];
    const uint64_t d1 = m + 1 < M ? a.seg_d0[m + 1] : D;
    const uint64_t lits = d1 - d0;
    const uint64_t run = s1 - s - lits;
    const uint64_t fill = word_kind(enc_word(a, s)) == 1 ? 1 : 0;
    const uint64_t pos = m + d0;
    if (pos < a.cap) a.out[pos] = fill | (run << 1) | (lits << 33);
  }
}

__global__ void enc_index_kernel(EncArgs a, uint64_t nchk) {
  for (uint64_t c = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; c < nchk;
       c += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t m = a.chk_marker[c];
    a.index[2 * c] = m + a.seg_d0[m];
    a.index[2 * c + 1] = a.seg_start[m];
  }
}

// ------------------------------------------------------ index building
// One wave per stream decodes the stream's markers 64 words at a time.  A
// chunk is one coalesced load (the next one is requested before the current
// one is decoded).  The markers of a chunk form a chain: each says where the
// next one is, one word further plus its literal count.  With next(i) = i +
// 1 + literals(word i) for every lane i (64: not in this chunk), the powers
// next^(2^b) follow from five rounds of cross-lane permutes (pointer
// doubling), and lane m composes them along the bits of m to find the
// position of the chunk's m-th marker; the words the markers cover (run +
// literals) are summed along the chain by the same doubling, which gives
// each marker's first uncompressed word.  The checkpoints
// a marker covers (multiples of kTile in [start, end)) are its index
// entries.  Chunks that hold only literal words are skipped.
__device__ __forceinline__ uint64_t readlane64(uint64_t v, int lane) {
  const uint32_t lo = __builtin_amdgcn_readlane((int)(uint32_t)v, lane);
  const uint32_t hi = __builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), lane);
  return (uint64_t)lo | ((uint64_t)hi << 32);
}

// value v of lane src (src in [0, 63]); every lane of the wave takes part
__device__ __forceinline__ uint32_t lane_get(uint32_t v, uint32_t src) {
  return (uint32_t)__builtin_amdgcn_ds_bpermute((int)(src << 2), (int)v);
}
__device__ __forceinline__ uint64_t lane_get64(uint64_t v, uint32_t src) {
  return (uint64_t)lane_get((uint32_t)v, src) | ((uint64_t)lane_get((uint32_t)(v >> 32), src) << 32);
}

typedef const __attribute__((address_space(1))) uint64_t GlobalWord;

__device__ __forceinline__ void build_index_wave(const uint64_t* __restrict__ s, uint64_t len, uint64_t nwords,
                                                 uint64_t* __restrict__ index, int* __restrict__ status) {
  const uint32_t lane = threadIdx.x & 63;
  const uint64_t nchk = (nwords + kTile - 1) / kTile;
  if (len == 0) {   // only an empty bitmap has an empty stream (and no checkpoint)
    if (nwords != 0 && lane == 0) set_status(status, TQ_EFORMAT);
    return;
  }
  GlobalWord* words = (GlobalWord*)s;
  // every lane loads (addresses clamped into the stream, words past its end
  // taken as zero), so no branch separates a load from its use
  const uint64_t last = len - 1;
  auto load = [&](uint64_t cb) {
    const uint64_t p = 64 * cb + lane;
    const uint64_t w = words[p < last ? p : last];
    return p < len ? w : (uint64_t)0;
  };
  uint64_t c = 0;          // chunk: stream words [64c, 64c + 64)
  uint64_t next_pos = 0;   // stream position of the next marker
  uint64_t wnext = 0;      // uncompressed word where its run starts
  bool bad = false;
  uint64_t x = load(0);
  while (next_pos < len) {
    const uint64_t xn = load(c + 1);       // requested before this chunk is decoded
    const uint64_t avail = len - 64 * c;   // stream words from the chunk start
    const uint64_t first = next_pos - 64 * c;

    // chunk positions of the markers: lane m gets the m-th one's (64: none)
    // and the words the first m of them cover (run + literals, summed along
    // the chain by the same doubling)
    const uint64_t nx = (uint64_t)lane + 1 + (x >> 33);
    uint32_t P[6];
    uint64_t S[6];
    P[0] = ((uint64_t)lane < avail && nx < 64) ? (uint32_t)nx : 64;
    S[0] = ((x >> 1) & 0xFFFFFFFFull) + (x >> 33);
#pragma unroll
    for (int b = 1; b < 6; ++b) {
      const uint32_t q = P[b - 1] & 63;
      const uint32_t v = lane_get(P[b - 1], q);
      const uint64_t t = lane_get64(S[b - 1], q);
      P[b] = P[b - 1] >= 64 ? 64 : v;
      S[b] = P[b - 1] >= 64 ? S[b - 1] : S[b - 1] + t;
    }
    uint32_t o = first < 64 ? (uint32_t)first : 64;
    uint64_t acc = 0;
#pragma unroll
    for (int b = 0; b < 6; ++b) {
      const uint32_t v = lane_get(P[b], o & 63);
      const uint64_t t = lane_get64(S[b], o & 63);
      if ((lane >> b) & 1) {
        acc += o >= 64 ? 0 : t;
        o = o >= 64 ? 64 : v;
      }
    }
    const bool is_m = o < 64 && (uint64_t)o < avail;
    const uint64_t mask = __ballot(is_m);
    const uint64_t mw = lane_get64(x, o & 63);
    const uint64_t run = is_m ? (mw >> 1) & 0xFFFFFFFFull : 0;
    const uint64_t lits = is_m ? mw >> 33 : 0;
    const uint64_t wm = wnext + acc;
    const uint64_t end = wm + run + lits;
    const uint64_t mpos = 64 * c + o;
    // a marker must stay inside the bitmap and its literals inside the stream
    if (__ballot(is_m && (end > nwords || lits > len - mpos - 1))) {
      bad = true;
      break;
    }
    // index entries: checkpoints k with k * kTile in [wm, end), written by
    // the marker's lane; a marker covering more than 64 (a long fill) is
    // written by the whole wave
    const uint64_t k0 = (wm + kTile - 1) / kTile;
    uint64_t k1 = (end + kTile - 1) / kTile;
    if (k1 > nchk) k1 = nchk;
    const bool many = is_m && k1 > k0 + 64;
    if (is_m && !many)
      for (uint64_t k = k0; k < k1; ++k) {
        index[2 * k] = mpos;
        index[2 * k + 1] = wm;
      }
    for (uint64_t mm = __ballot(many); mm; mm &= mm - 1) {
      const int jl = __ffsll((unsigned long long)mm) - 1;
      const uint64_t jk0 = readlane64(k0, jl), jk1 = readlane64(k1, jl);
      const uint64_t jpos = readlane64(mpos, jl), jw = readlane64(wm, jl);
      for (uint64_t k = jk0 + lane; k < jk1; k += 64) {
        index[2 * k] = jpos;
        index[2 * k + 1] = jw;
      }
    }
    // the next marker follows the chunk's last one (every chunk decoded
    // holds one: it is the chunk of next_pos)
    const int lm = 63 - __clzll(mask);
    next_pos = readlane64(mpos, lm) + 1 + readlane64(lits, lm);
    wnext = readlane64(end, lm);
    // the chunk holding it (literal-only chunks between are not read)
    const uint64_t cn = next_pos >> 6;
    if (cn == c + 1) x = xn;
    else if (next_pos < len) x = load(cn);
    c = cn;
  }
  if (bad || next_pos != len || wnext != nwords) {
    if (lane == 0) set_status(status, TQ_EFORMAT);
  }
}

__global__ __launch_bounds__(64) void build_index_kernel(const uint64_t* __restrict__ s, uint64_t len,
                                                         uint64_t nwords, uint64_t* __restrict__ index,
                                                         int* __restrict__ status) {
  build_index_wave(s, len, nwords, index, status);
}

// The indexes of several streams of one query at once: workgroup b walks the
// stream of descriptor list[b] and writes the index that descriptor names.
__global__ __launch_bounds__(64) void build_indexes_kernel(const RleDesc* __restrict__ descs,
                                                           const uint32_t* __restrict__ list, uint64_t nwords,
                                                           int* __restrict__ status) {
  const RleDesc d = descs[list[blockIdx.x]];
  build_index_wave(d.words, d.len, nwords, const_cast<uint64_t*>(d.index), status);
}

uint32_t grid_cap(uint64_t want, uint32_t cap) {
  if (want == 0) return 1;
  return want > cap ? cap : (uint32_t)want;
}

typedef void (*TileFn)(const RleDesc*, uint32_t, const uint64_t* const*, uint32_t, uint32_t, uint64_t,
                       uint32_t, const RleSym*, uint32_t, uint64_t*, int*, Sink);

template <bool Sym, bool Fused, bool Hybrid>
TileFn pick_tile_k(int K) {
  switch (K) {
    case 4: return rle_tile_kernel<4, Sym, false, kFullPlanes, Fused, Hybrid>;
    case 5: return rle_tile_kernel<5, Sym, false, kFullPlanes, Fused, Hybrid>;
    case 6: return rle_tile_kernel<6, Sym, false, kFullPlanes, Fused, Hybrid>;
    case 7: return rle_tile_kernel<7, Sym, false, kFullPlanes, Fused, Hybrid>;
    case 8: return rle_tile_kernel<8, Sym, false, kFullPlanes, Fused, Hybrid>;
    case 9: return rle_tile_kernel<9, Sym, false, kFullPlanes, Fused, Hybrid>;
    case 10: return rle_tile_kernel<10, Sym, false, kFullPlanes, Fused, Hybrid>;
    case 11: return rle_tile_kernel<11, Sym, false, kFullPlanes, Fused, Hybrid>;
    case 12: return rle_tile_kernel<12, Sym, false, kFullPlanes, Fused, Hybrid>;
    case 13: return rle_tile_kernel<13, Sym, false, kFullPlanes, Fused, Hybrid>;
    case 16: return rle_tile_kernel<16, Sym, false, kFullPlanes, Fused, Hybrid>;
  }
  return nullptr;
}

// thresholds with bit_length(theta - 1) exact planes and a sticky one, or
// symmetric functions with bit_length(tail_from) exact planes and a sticky one
template <bool Sym, bool Fused, bool Hybrid>
TileFn pick_sat_k(int K) {
  switch (K) {
    case 1:
      if constexpr (!Sym) return rle_tile_kernel<1, false, false, kSaturating, Fused, Hybrid>;
      return nullptr;
    case 2: return rle_tile_kernel<2, Sym, false, kSaturating, Fused, Hybrid>;
    case 3: return rle_tile_kernel<3, Sym, false, kSaturating, Fused, Hybrid>;
    case 4: return rle_tile_kernel<4, Sym, false, kSaturating, Fused, Hybrid>;
    case 5: return rle_tile_kernel<5, Sym, false, kSaturating, Fused, Hybrid>;
    case 6: return rle_tile_kernel<6, Sym, false, kSaturating, Fused, Hybrid>;
    case 7: return rle_tile_kernel<7, Sym, false, kSaturating, Fused, Hybrid>;
    case 8: return rle_tile_kernel<8, Sym, false, kSaturating, Fused, Hybrid>;
    case 9: return rle_tile_kernel<9, Sym, false, kSaturating, Fused, Hybrid>;
    case 10: return rle_tile_kernel<10, Sym, false, kSaturating, Fused, Hybrid>;
    case 11: return rle_tile_kernel<11, Sym, false, kSaturating, Fused, Hybrid>;
    case 12: return rle_tile_kernel<12, Sym, false, kSaturating, Fused, Hybrid>;
    case 13: return rle_tile_kernel<13, Sym, false, kSaturating, Fused, Hybrid>;
  }
  return nullptr;
}

// The kernel of a query: its counter form and width (K), and a key of that
// choice for the per-device occupancy table.
struct TileChoice {
  TileFn fn = nullptr;
  int K = 0;
  int key = 0;
};

template <bool Fused, bool Hybrid>
TileChoice choose_tile(int K, uint32_t theta, const RleSym* sym, bool swar) {
  TileChoice c;
  c.K = K;
  if (swar) {
    c.fn = sym ? rle_tile_kernel<16, true, true, kFullPlanes, Fused, Hybrid>
               : rle_tile_kernel<16, false, true, kFullPlanes, Fused, Hybrid>;
    c.key = 34 + (sym ? 1 : 0);
    return c;
  }
  c.fn = sym ? pick_tile_k<true, Fused, Hybrid>(K) : pick_tile_k<false, Fused, Hybrid>(K);
  c.key = K + (sym ? 17 : 0);
  // A threshold asks of an undecided column whether its counted bits exceed
  // a = theta - k - 1 < theta.  Planes exact below 2^(K-1) and a sticky top
  // plane ("at least 2^(K-1)") answer that whenever 2^(K-1) > theta - 1, so
  // bit_length(theta - 1) exact planes and a sticky one decide it (theta = 1:
  // the sticky plane alone, "at least one"): less LDS per workgroup, and more
  // workgroups per CU, when that is fewer planes.
  if (!sym && theta >= 1) {
    const int ks = bit_length(theta - 1) + 1;
    if (ks < K && ks <= 13) {
      c.K = ks;
      c.fn = pick_sat_k<false, Fused, Hybrid>(ks);
      c.key = 36 + ks;
    }
  }
  // A symmetric f that is constant from tail_from on needs the count exactly
  // only below tail_from: bit_length(tail_from) exact planes and a sticky one.
  if (sym && sym->epi.kind != EPI_PARITY && sym->tail_from >= 1) {
    const int ks = bit_length(sym->tail_from) + 1;
    if (ks < K && ks <= 13) {
      c.K = ks;
      c.fn = pick_sat_k<true, Fused, Hybrid>(ks);
      c.key = 51 + ks;
    }
  }
  // the parity function (or its complement) needs the count modulo 2 only
  if (sym && sym->epi.kind == EPI_PARITY) {
    c.K = 1;
    c.fn = rle_tile_kernel<1, true, false, kParityPlane, Fused, Hybrid>;
    c.key = 50;
  }
  return c;
}

}  // namespace

size_t rle_tile_lds_bytes(int K, bool swar) {
  return (size_t)(swar ? 16 : K) * kTile * 8 * plane_tiles(K, swar) + (size_t)(kSpan * kTile + 2) * 4;
}

hipError_t launch_rle_tile(const RleDesc* d_descs, uint32_t n_rle, const uint64_t* const* d_dense,
                           uint32_t n_dense, uint64_t nwords, uint64_t tail_mask, uint32_t theta,
                           const RleSym* sym, const RleSym* d_sym, bool swar, int num_cus,
                           uint32_t tiles_per_group, uint64_t* d_out, int* d_status, hipStream_t stream,
                           const Sink& sink, uint64_t* slots_used) {
  if (sym && !d_sym) return hipErrorInvalidValue;
  const bool fused = sink.filter != nullptr || sink.partial64 != nullptr;
  const bool hybrid = n_dense > 0;
  if (fused && hybrid) return hipErrorInvalidValue;   // no such build
  const int K0 = dense_planes_for(n_rle + n_dense);
  const TileChoice ch = fused    ? choose_tile<true, false>(K0, theta, sym, swar)
                        : hybrid ? choose_tile<false, true>(K0, theta, sym, swar)
                                 : choose_tile<false, false>(K0, theta, sym, swar);
  TileFn fn = ch.fn;
  const int K = ch.K;
  // keys are below 65; fused and hybrid builds get their own ranges
  const int slot = ch.key + (fused ? 65 : 0) + (hybrid ? 130 : 0);
  if (!fn) return hipErrorInvalidValue;
  const uint64_t tiles = (nwords + kTile - 1) / kTile;
  if (tiles == 0) return hipSuccess;
  const size_t lds = rle_tile_lds_bytes(K, swar);
  // LDS limit and resident workgroups per CU, set and measured once per device
  constexpr int kMaxDevices = 64;
  static std::mutex mu;
  static int resident[kMaxDevices][195] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  int per_cu = 0;
  {
    std::lock_guard<std::mutex> lock(mu);
    if (dev >= 0 && dev < kMaxDevices) per_cu = resident[dev][slot];
    if (per_cu == 0) {
      e = hipFuncSetAttribute(reinterpret_cast<const void*>(fn), hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)lds);
      if (e != hipSuccess) return e;
      if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(fn), kTileThreads,
                                                       lds) != hipSuccess || per_cu < 1)
        per_cu = 1;
      if (dev >= 0 && dev < kMaxDevices) resident[dev][slot] = per_cu;
    }
  }
  // by default one range of consecutive tiles per resident workgroup
  const uint64_t slots = (uint64_t)(num_cus > 0 ? num_cus : 1) * (uint64_t)per_cu;
  uint64_t per_group = tiles_per_group ? tiles_per_group : (tiles + slots - 1) / slots;
  if (per_group > tiles) per_group = tiles;
  const uint64_t ranges = (tiles + per_group - 1) / per_group;
  const uint64_t grid = (ranges + kXcds - 1) / kXcds * kXcds;
  hipLaunchKernelGGL(fn, dim3((uint32_t)grid), dim3(kTileThreads), lds, stream, d_descs, n_rle, d_dense,
                     n_dense, (uint32_t)nwords, tail_mask, theta, d_sym, (uint32_t)per_group,
                     d_out, d_status, sink);
  if (slots_used) *slots_used = grid * (kTileThreads / 64);
  return hipGetLastError();
}

// workgroups of a launch are at most its tiles rounded up to a multiple of kXcds
uint64_t rle_tile_partials(uint64_t nwords) {
  return ((nwords + kTile - 1) / kTile + kXcds - 1) / kXcds * kXcds * (kTileThreads / 64);
}

size_t rle_encode_workspace_bytes(uint64_t nwords) {
  const uint64_t nblocks = (nwords + kEncWords - 1) / kEncWords;
  const uint64_t nchk = (nwords + kTile - 1) / kTile;
  return 256 + nblocks * 8 + nwords * 8 + nchk * 4 + 256;
}

hipError_t launch_rle_encode(const uint64_t* d_dense, uint64_t nwords, uint64_t tail_mask, uint64_t* d_out,
                             uint64_t cap, uint64_t* d_out_len, uint64_t* d_index, void* workspace,
                             int* d_status, hipStream_t stream) {
  const uint64_t nblocks = (nwords + kEncWords - 1) / kEncWords;
  const uint64_t nchk = (nwords + kTile - 1) / kTile;
  char* ws = static_cast<char*>(workspace);
  EncArgs a;
  a.dense = d_dense;
  a.nwords = nwords;
  a.tail_mask = tail_mask;
  a.totals = reinterpret_cast<uint64_t*>(ws);
  a.block_sums = reinterpret_cast<uint64_t*>(ws + 256);
  a.seg_start = reinterpret_cast<uint32_t*>(ws + 256 + nblocks * 8);
  a.seg_d0 = a.seg_start + nwords;
  a.chk_marker = a.seg_d0 + nwords;
  a.out = d_out;
  a.cap = cap;
  a.out_len = d_out_len;
  a.index = d_index;
  a.status = d_status;
  hipLaunchKernelGGL(enc_reduce_kernel, dim3((uint32_t)nblocks), dim3(kEncBlock), 0, stream, a);
  hipLaunchKernelGGL(enc_scan_kernel, dim3(1), dim3(1024), 0, stream, a, nblocks);
  hipLaunchKernelGGL(enc_scatter_kernel, dim3((uint32_t)nblocks), dim3(kEncBlock), 0, stream, a);
  // markers are at most nwords; the grid strides over however many there are
  hipLaunchKernelGGL(enc_marker_kernel, dim3(grid_cap((nwords + 255) / 256, 2048)), dim3(256), 0, stream, a);
  if (d_index)
    hipLaunchKernelGGL(enc_index_kernel, dim3(grid_cap((nchk + 255) / 256, 65536)), dim3(256), 0, stream, a,
                       nchk);
  return hipGetLastError();
}

hipError_t launch_build_index(const uint64_t* d_words, uint64_t len, uint64_t nwords, uint64_t* d_index,
                              int* d_status, hipStream_t stream) {
  hipLaunchKernelGGL(build_index_kernel, dim3(1), dim3(64), 0, stream, d_words, len, nwords, d_index,
                     d_status);
  return hipGetLastError();
}

hipError_t launch_build_indexes(const RleDesc* d_descs, const uint32_t* d_list, uint32_t count, uint64_t nwords,
                                int* d_status, hipStream_t stream) {
  if (count == 0) return hipSuccess;
  hipLaunchKernelGGL(build_indexes_kernel, dim3(count), dim3(64), 0, stream, d_descs, d_list, nwords, d_status);
  return hipGetLastError();
}

}  // namespace tq
