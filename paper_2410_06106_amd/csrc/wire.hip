// Wire format of a K-means message (Sections 2.6 and 3.3): a segment's labels
// packed at `bits` bits per value into a little-endian stream of 32-bit words,
// value i in stream bits [i*bits, (i+1)*bits), least significant bit first.
// Packing and unpacking are HBM-bound streaming passes.
#include "common.h"

namespace tomo {

// One thread per output word: ORs in the (at most 32/bits + 2) codes whose bits
// overlap stream bits [32w, 32w + 32); the first may start in the previous
// word, the last may continue into the next one.
__global__ __launch_bounds__(256) void k_pack_labels(const uint8_t* lab, int n, int bits, unsigned* out,
                                                      long long n_words) {
  const long long w = (long long)blockIdx.x * 256 + threadIdx.x;
  if (w >= n_words) return;
  const long long b0 = 32 * w;
  const unsigned mask = (1u << bits) - 1u;
  const int v0 = (int)(b0 / bits);
  const int v1 = (int)min((long long)n, (b0 + 32 + bits - 1) / bits);   // values starting before b0 + 32
  unsigned word = 0;
  for (int v = v0; v < v1; ++v) {
    const int s = (int)((long long)v * bits - b0);                       // -bits < s < 32
    const unsigned code = lab[v] & mask;
    word |= s >= 0 ? code << s : code >> -s;
  }
  out[w] = word;
}

// One thread per value: the code from one or two words, then the label and/or
// the centroid it stands for (codes >= k read the last centroid).
__global__ __launch_bounds__(256) void k_unpack_labels(const unsigned* in, int n, int bits, const float* cent, int k,
                                                        uint8_t* lab, float* a_hat) {
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const long long p = i * bits;
  const long long w = p >> 5;
  const int sh = (int)(p & 31);
  unsigned code = in[w] >> sh;
  if (sh + bits > 32) code |= in[w + 1] << (32 - sh);
  code &= (1u << bits) - 1u;
  if (lab) lab[i] = (uint8_t)code;
  if (a_hat) a_hat[i] = cent[min((int)code, k - 1)];
}

}  // namespace tomo
