// Lossless coding of the edit streams (Alg. 1, LosslesslyCompressEdits; Sec. IV-B, IV-D):
// symbols (flag bytes or int32 codes) are counted blockwise into a global frequency table,
// the host builds the Huffman code from that table, and the stream is encoded in parallel:
// every symbol's bit offset is an exclusive prefix sum of code lengths (block sums, one-block
// scan, block-local scan), and each symbol ORs its code into at most two 32-bit words.
//
// Stream layout (bits): codes most significant bit first, each 32-bit word filled from its
// top bit down.  The offset of every kHuffChunk-th symbol is kept, so the decoder runs one
// lane per chunk of symbols, each from its own starting bit.
#pragma once
#include <climits>

#include "common.hpp"

namespace ffcz {

constexpr int kHuffChunk = 256;       // symbols per decoder chunk
constexpr int kHuffBlock = 256;       // lanes per block
constexpr int kHuffPerLane = 8;       // symbols per lane in the offset passes
constexpr int64_t kHuffBlockSyms = (int64_t)kHuffBlock * kHuffPerLane;
constexpr int kHuffLdsBins = 8192;    // alphabets up to this size count in LDS
constexpr int kHuffDecBlock = 64;     // decoder lanes per block (one chunk each): small blocks
                                      // spread the few chunks of a stream over more CUs

// symbol i of a stream of 1-byte (width 1) or 4-byte signed (width 4) symbols
__device__ __forceinline__ int64_t huff_sym(const void* s, int width, int64_t i) {
  return width == 1 ? (int64_t)((const uint8_t*)s)[i] : (int64_t)((const int32_t*)s)[i];
}

// Block minima and maxima of the symbols (as offset-binary 64-bit keys).
__global__ void __launch_bounds__(kHuffBlock) huff_minmax_kernel(const void* s, int width, int64_t n,
                                                                 long long* part) {
  __shared__ long long rmin[4], rmax[4];
  long long mn = LLONG_MAX, mx = LLONG_MIN;
  for (int64_t i = (int64_t)blockIdx.x * kHuffBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kHuffBlock) {
    const long long v = huff_sym(s, width, i);
    mn = v < mn ? v : mn;
    mx = v > mx ? v : mx;
  }
  for (int off = 32; off > 0; off >>= 1) {
    const long long a = __shfl_xor(mn, off, 64), b = __shfl_xor(mx, off, 64);
    mn = a < mn ? a : mn;
    mx = b > mx ? b : mx;
  }
  if ((threadIdx.x & 63) == 0) {
    rmin[threadIdx.x >> 6] = mn;
    rmax[threadIdx.x >> 6] = mx;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < 4; ++w) {
      mn = rmin[w] < mn ? rmin[w] : mn;
      mx = rmax[w] > mx ? rmax[w] : mx;
    }
    part[2 * blockIdx.x] = mn;
    part[2 * blockIdx.x + 1] = mx;
  }
}

// The global frequency table over lo .. lo + nalpha - 1 (counts must start at zero): small
// alphabets count per block in LDS and add the block's table once, larger ones add straight
// into the global table.  Integer additions, so the table does not depend on the order.
__global__ void __launch_bounds__(kHuffBlock) huff_hist_kernel(const void* s, int width, int64_t n, int64_t lo,
                                                               int64_t nalpha, unsigned long long* counts) {
  __shared__ unsigned int h[kHuffLdsBins];
  const bool local = nalpha <= kHuffLdsBins;
  if (local)
    for (int i = threadIdx.x; i < nalpha; i += kHuffBlock) h[i] = 0u;
  __syncthreads();
  // Edit streams are dominated by one symbol (zero flag bytes, zero codes): the lanes of a
  // wave holding the same symbol as the wave's first active lane add once, by their number.
  const int64_t stride = (int64_t)gridDim.x * kHuffBlock;
  const int64_t start = (int64_t)blockIdx.x * kHuffBlock + threadIdx.x;
  const int64_t span = (n + kHuffBlock - 1) / kHuffBlock * kHuffBlock;  // whole waves stay in the loop
  for (int64_t i = start; i < span; i += stride) {
    const bool in = i < n;
    const int64_t b = in ? huff_sym(s, width, i) - lo : -1;
    const int64_t b0 = __builtin_amdgcn_readfirstlane((int)b);
    const unsigned long long same = __ballot(in && b == b0);
    const unsigned long long below = __builtin_amdgcn_mbcnt_hi((unsigned)(same >> 32),
                                                               __builtin_amdgcn_mbcnt_lo((unsigned)same, 0u));
    if (!in) continue;
    unsigned int add = 1u;
    if (b == b0) {
      if (below != 0) continue;  // not the first lane of the group
      add = (unsigned int)__popcll(same);
    }
    if (local) atomicAdd(&h[b], add);
    else atomicAdd(&counts[b], (unsigned long long)add);
  }
  __syncthreads();
  if (local)
    for (int i = threadIdx.x; i < nalpha; i += kHuffBlock)
      if (h[i]) atomicAdd(&counts[i], (unsigned long long)h[i]);
}

// Bits of the symbols of each block of kHuffBlockSyms symbols.
__global__ void __launch_bounds__(kHuffBlock) huff_bits_kernel(const void* s, int width, int64_t n, int64_t lo,
                                                               const uint8_t* len, unsigned long long* part) {
  __shared__ unsigned long long red[4];
  const int64_t base = (int64_t)blockIdx.x * kHuffBlockSyms;
  unsigned long long b = 0;
  for (int k = 0; k < kHuffPerLane; ++k) {
    const int64_t i = base + (int64_t)k * kHuffBlock + threadIdx.x;
    if (i < n) b += len[huff_sym(s, width, i) - lo];
  }
  for (int off = 32; off > 0; off >>= 1) b += __shfl_xor(b, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = b;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

// Encode: lane t of a block owns symbols base + t * kHuffPerLane + k (consecutive), so its bit
// offset is the block offset plus an exclusive scan of the lanes' bit counts.  Each code ORs
// into the one or two words it covers (words start at zero).  The lane holding symbol
// j * kHuffChunk records that symbol's offset.
__global__ void __launch_bounds__(kHuffBlock) huff_encode_kernel(const void* s, int width, int64_t n, int64_t lo,
                                                                 const uint8_t* len, const uint32_t* code,
                                                                 const unsigned long long* boff, unsigned int* words,
                                                                 unsigned long long* chunk_bits) {
  __shared__ unsigned long long wsum[4];
  const int64_t base = (int64_t)blockIdx.x * kHuffBlockSyms;
  const int t = threadIdx.x;
  int64_t sym[kHuffPerLane];
  unsigned long long mine = 0;
#pragma unroll
  for (int k = 0; k < kHuffPerLane; ++k) {
    const int64_t i = base + (int64_t)t * kHuffPerLane + k;
    sym[k] = i < n ? huff_sym(s, width, i) - lo : -1;
    mine += sym[k] >= 0 ? len[sym[k]] : 0;
  }
  // inclusive scan over the wave, then over the four waves
  unsigned long long inc = mine;
  for (int off = 1; off < 64; off <<= 1) {
    const unsigned long long o = __shfl_up(inc, off, 64);
    if ((t & 63) >= off) inc += o;
  }
  if ((t & 63) == 63) wsum[t >> 6] = inc;
  __syncthreads();
  unsigned long long pos = boff[blockIdx.x] + inc - mine;
  for (int w = 0; w < (t >> 6); ++w) pos += wsum[w];
#pragma unroll
  for (int k = 0; k < kHuffPerLane; ++k) {
    if (sym[k] < 0) break;
    const int64_t i = base + (int64_t)t * kHuffPerLane + k;
    if (i % kHuffChunk == 0) chunk_bits[i / kHuffChunk] = pos;
    const int l = len[sym[k]];
    const unsigned long long c = code[sym[k]];
    // the code's bits at stream positions pos .. pos + l - 1
    const int64_t w0 = (int64_t)(pos >> 5);
    const int sh = (int)(pos & 31);
    const unsigned long long aligned = (c << (64 - l)) >> sh;  // top of a 64-bit window at word w0
    atomicOr(&words[w0], (unsigned int)(aligned >> 32));
    if (sh + l > 32) atomicOr(&words[w0 + 1], (unsigned int)(aligned & 0xffffffffull));
    pos += l;
  }
}

// Decode: one lane per chunk walks its symbols from the chunk's first bit.  The lane keeps a
// 64-bit window of the stream (refilled a word at a time) and decodes against left-justified
// canonical limits: with v the window's top 32 bits, the code length is the smallest l with
// v < lim[l] = (first[l] + cnt[l]) << (32 - l), and the symbol is
// sorted[idx[l] + (v >> (32 - l)) - first[l]] (symbols ordered by length, then value).  The
// tables sit in LDS.
__global__ void __launch_bounds__(kHuffDecBlock) huff_decode_kernel(const unsigned int* words, int64_t nwords,
                                                                 const unsigned long long* chunk_bits, int64_t n,
                                                                 const uint32_t* first, const uint32_t* cnt,
                                                                 const uint32_t* idx, const int32_t* sorted,
                                                                 int64_t lo, int width, void* out,
                                                                 unsigned int* bad) {
  __shared__ unsigned long long lim[33];
  __shared__ uint32_t fst[33], ix[33];
  if (threadIdx.x < 33) {
    const int l = threadIdx.x;
    fst[l] = first[l];
    ix[l] = idx[l];
    // lengths without codes get a limit no window reaches past the previous length's
    lim[l] = l == 0 ? 0ull : ((unsigned long long)first[l] + cnt[l]) << (32 - l);
  }
  __syncthreads();
  const int64_t ch = (int64_t)blockIdx.x * kHuffDecBlock + threadIdx.x;
  const int64_t i0 = ch * kHuffChunk;
  if (i0 >= n) return;
  const int64_t i1 = i0 + kHuffChunk < n ? i0 + kHuffChunk : n;
  const unsigned long long p0 = chunk_bits[ch];
  // window: the stream's bits from position pos on, left-justified, nb of them valid
  int64_t w = (int64_t)(p0 >> 5);
  auto word = [&](int64_t k) -> unsigned long long { return k < nwords ? (unsigned long long)words[k] : 0ull; };
  unsigned long long buf = ((word(w) << 32) | word(w + 1)) << (p0 & 31);
  int nb = 64 - (int)(p0 & 31);
  w += 2;
  for (int64_t i = i0; i < i1; ++i) {
    if (nb <= 32) {  // refill one word below the valid bits
      buf |= word(w) << (32 - nb);
      nb += 32;
      ++w;
    }
    const unsigned long long v = buf >> 32;
    int l = 1;
    while (l <= 32 && v >= lim[l]) ++l;
    if (l > 32) {
      atomicOr(bad, 1u);
      return;
    }
    const uint32_t c = (uint32_t)(v >> (32 - l));
    const int64_t sym = sorted[ix[l] + (c - fst[l])];
    buf <<= l;
    nb -= l;
    if (width == 1) ((uint8_t*)out)[i] = (uint8_t)(sym + lo);
    else ((int32_t*)out)[i] = (int32_t)(sym + lo);
  }
}

}  // namespace ffcz
