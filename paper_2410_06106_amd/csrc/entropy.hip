// Entropy code of a segment's DCT codes (the DCT message on the wire; Section
// 2.6 with the lossless stage of baseline JPEG replaced by universal codes):
// blocks row-major, codes in zigzag order, DC sent as the difference from the
// previous block's DC (from 0 at each restart interval of 64 blocks), AC as
// (zeros skipped + 1, level) pairs and an end-of-block symbol, every number an
// order-0 Exp-Golomb code; bits packed most significant first into 32-bit
// words.
//
// Encoding is three passes: the bit length of every block (one thread per
// block), one workgroup's exclusive scan of the lengths (block offsets, the
// restart table, the total), then every block writes its bits at its offset
// with atomic ORs (a block shares its first and last words with its
// neighbours).  Decoding runs one thread per restart interval.
#include "common.h"
#include "codec.h"

namespace tomo {

namespace {

__constant__ unsigned char kZigzag[64] = {   // natural (8u + v) index of each scan position
    0,  1,  8,  16, 9,  2,  3,  10, 17, 24, 32, 25, 18, 11, 4,  5,  12, 19, 26, 33, 40, 48,
    41, 34, 27, 20, 13, 6,  7,  14, 21, 28, 35, 42, 49, 56, 57, 50, 43, 36, 29, 22, 15, 23,
    30, 37, 44, 51, 58, 59, 52, 45, 38, 31, 39, 46, 53, 60, 61, 54, 47, 55, 62, 63};

__device__ __forceinline__ int eg_len(unsigned x) {      // length of EG(x)
  return 2 * (31 - __clz(x + 1)) + 1;
}

__device__ __forceinline__ unsigned zz_signed(int d) {   // 2d for d >= 0, -2d - 1 for d < 0
  return d >= 0 ? 2u * (unsigned)d : 2u * (unsigned)(-d) - 1u;
}

__device__ __forceinline__ unsigned level_code(int v) {  // 2 (|v| - 1) + (v < 0), v != 0
  return 2u * (unsigned)(abs(v) - 1) + (v < 0 ? 1u : 0u);
}

// Visit the symbols of block b as (value, length) pairs of Exp-Golomb codes.
template <class F>
__device__ void block_symbols(const int16_t* q, int ld, int n_bc, int b, F&& emit) {
  const int br = b / n_bc, bc = b - br * n_bc;
  const int16_t* blk = q + (size_t)(8 * br) * ld + 8 * bc;
  int prev = 0;
  if (b % ECODE_INTERVAL != 0) {
    const int pb = b - 1, pr = pb / n_bc, pc = pb - pr * n_bc;
    prev = q[(size_t)(8 * pr) * ld + 8 * pc];
  }
  const unsigned d = zz_signed((int)blk[0] - prev);
  emit(d + 1u, eg_len(d));
  int run = 0;
  for (int k = 1; k < 64; ++k) {
    const int nat = kZigzag[k];
    const int v = blk[(nat >> 3) * ld + (nat & 7)];
    if (v == 0) {
      ++run;
      continue;
    }
    emit((unsigned)run + 2u, eg_len((unsigned)run + 1u));
    const unsigned m = level_code(v);
    emit(m + 1u, eg_len(m));
    run = 0;
  }
  emit(1u, 1);                                            // end of block: EG(0)
}

}  // namespace

__global__ __launch_bounds__(256) void k_ecode_bits(const int16_t* q, int ld, int n_bc, int n_blocks,
                                                     unsigned* bits) {
  const int b = blockIdx.x * 256 + threadIdx.x;
  if (b >= n_blocks) return;
  unsigned total = 0;
  block_symbols(q, ld, n_bc, b, [&](unsigned, int len) { total += (unsigned)len; });
  bits[b] = total;
}

// One workgroup: exclusive scan of the block lengths in place (offsets), the
// restart table (offset of every 64th block) and the total.
__global__ __launch_bounds__(1024) void k_ecode_scan(unsigned* off, int n_blocks, unsigned* restart,
                                                      unsigned* total) {
  __shared__ unsigned part[1024];
  const int t = threadIdx.x;
  const int per = (n_blocks + 1023) / 1024;
  const int b0 = min(n_blocks, t * per), b1 = min(n_blocks, b0 + per);
  unsigned s = 0;
  for (int b = b0; b < b1; ++b) s += off[b];
  part[t] = s;
  __syncthreads();
  for (int d = 1; d < 1024; d <<= 1) {                    // inclusive scan of the thread sums
    const unsigned v = t >= d ? part[t - d] : 0u;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  unsigned run = part[t] - s;
  for (int b = b0; b < b1; ++b) {
    const unsigned len = off[b];
    off[b] = run;
    if (b % ECODE_INTERVAL == 0) restart[b / ECODE_INTERVAL] = run;
    run += len;
  }
  if (t == 1023) *total = part[1023];
}

__global__ __launch_bounds__(256) void k_ecode_zero(unsigned* w, long long n) {
  for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long long)gridDim.x * 256) w[i] = 0u;
}

__global__ __launch_bounds__(256) void k_ecode_write(const int16_t* q, int ld, int n_bc, int n_blocks,
                                                      const unsigned* off, unsigned* words) {
  const int b = blockIdx.x * 256 + threadIdx.x;
  if (b >= n_blocks) return;
  unsigned long long pos = off[b];
  block_symbols(q, ld, n_bc, b, [&](unsigned val, int len) {
    if (len > 32) {                                       // leading zeros of a long code
      pos += (unsigned)(len - 32);
      len = 32;
    }
    const unsigned w = (unsigned)(pos >> 5), o = (unsigned)(pos & 31);
    if (o + len <= 32) {
      atomicOr(words + w, val << (32 - o - len));
    } else {
      const int spill = (int)(o + len - 32);              // bits that go to the next word
      atomicOr(words + w, val >> spill);
      atomicOr(words + w + 1, val << (32 - spill));
    }
    pos += (unsigned)len;
  });
}

// One thread per restart interval.  A malformed stream (a code running past
// the total, more than 64 coefficients in a block) sets *status to 1.
__global__ __launch_bounds__(256) void k_ecode_decode(const unsigned* words, long long n_words,
                                                       const unsigned* restart, const unsigned* total,
                                                       int n_bc, int n_blocks, int16_t* q, int ld, int* status) {
  const int iv = blockIdx.x * 256 + threadIdx.x;
  const int first = iv * ECODE_INTERVAL;
  if (first >= n_blocks) return;
  const unsigned long long end = *total;
  unsigned long long pos = restart[iv];
  bool bad = false;
  auto peek64 = [&](unsigned long long p) -> unsigned long long {   // 64 stream bits from p
    const long long w = (long long)(p >> 5);
    const unsigned o = (unsigned)(p & 31);
    const unsigned long long a = w < n_words ? words[w] : 0u;
    const unsigned long long b = w + 1 < n_words ? words[w + 1] : 0u;
    const unsigned long long c = w + 2 < n_words ? words[w + 2] : 0u;
    const unsigned long long hi = (a << 32) | b;
    return o ? (hi << o) | (c >> (32 - o)) : hi;
  };
  auto read_eg = [&]() -> unsigned {
    const unsigned long long win = peek64(pos);
    const int z = win ? __clzll(win) : 64;
    if (z > 31 || pos + 2ull * z + 1ull > end) {
      bad = true;
      return 0u;
    }
    const unsigned y = (unsigned)(win >> (64 - (2 * z + 1)));    // z zeros then z + 1 value bits
    pos += 2ull * z + 1ull;
    return y - 1u;
  };
  int prev = 0;
  const int last = min(n_blocks, first + ECODE_INTERVAL);
  for (int b = first; b < last && !bad; ++b) {
    const int br = b / n_bc, bc = b - br * n_bc;
    int16_t* blk = q + (size_t)(8 * br) * ld + 8 * bc;
    for (int u = 0; u < 8; ++u)
      for (int v = 0; v < 8; ++v) blk[u * ld + v] = 0;
    const unsigned x = read_eg();
    const int dc = prev + ((x & 1u) ? -(int)((x + 1u) >> 1) : (int)(x >> 1));
    prev = dc;
    blk[0] = (int16_t)dc;
    int k = 1;
    while (!bad) {
      const unsigned r1 = read_eg();
      if (bad || r1 == 0u) break;
      k += (int)r1 - 1;
      const unsigned m = read_eg();
      if (bad || k > 63) {
        bad = true;
        break;
      }
      const int nat = kZigzag[k];
      blk[(nat >> 3) * ld + (nat & 7)] = (int16_t)((m & 1u) ? -(int)(m / 2u + 1u) : (int)(m / 2u + 1u));
      ++k;
    }
  }
  if (bad && status) atomicOr(status, 1);
}

}  // namespace tomo
