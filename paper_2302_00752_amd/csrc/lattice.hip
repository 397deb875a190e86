// Random rank-1 lattices on the stamping sets (Sec. 8: the Definition of a reconstructing
// rank-1 lattice and Lemma RandomRank1Lattice).
//
// The lattice Lambda(z, M) pairs frequency k with the index k . z mod M of a length-M
// one-dimensional transform; it reconstructs a set I when that index separates the
// frequencies of I.  Here every key of a stamp gets its index (one thread per key, exact
// 64-bit integer arithmetic), and each problem's set is checked by sorting (problem, index)
// words and looking for equal neighbours: the keys of one problem are distinct, so two equal
// words are two frequencies the lattice does not separate.  The Lemma's modulus (the smallest
// prime above max(K, |I|^2 / sigma)) is found on the host by a deterministic Miller-Rabin test.
#include <hip/hip_runtime.h>

#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <cmath>
#include <vector>

#include "ss_internal.h"

namespace ss {

namespace {

constexpr int kLatBits = 40;                       // lattice indices are below 2^40
constexpr int64_t kLatMaxM = int64_t(1) << kLatBits;
constexpr int kLatChunk = 128;                     // coordinates summed between reductions mod M

// index k . z mod M of every key, one thread per key.  Between reductions the sum stays below
// 2^63: the carried value is below M <= 2^40 and each of the at most 128 terms is below
// 2^15 * 2^40 in size.  For even d each key starts 4-byte aligned and is read two coordinates
// per load.
template <bool EVEN>
__global__ void k_lattice_values(int64_t total, int d, const int16_t* __restrict__ keys,
                                 const int64_t* __restrict__ z, int64_t M, const int32_t* __restrict__ pid,
                                 int vbits, int64_t* __restrict__ values, uint64_t* __restrict__ words) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= total) return;
  const int16_t* k = keys + r * d;
  int64_t acc = 0;
  for (int i0 = 0; i0 < d; i0 += kLatChunk) {
    const int i1 = min(d, i0 + kLatChunk);
    if (EVEN) {   // i0 and i1 are even
      const uint32_t* k2 = reinterpret_cast<const uint32_t*>(k);
      for (int i = i0; i < i1; i += 2) {
        const uint32_t v = k2[i >> 1];
        acc += (int64_t)(int16_t)(v & 0xffff) * z[i] + (int64_t)(int16_t)(v >> 16) * z[i + 1];
      }
    } else {
      for (int i = i0; i < i1; ++i) acc += (int64_t)k[i] * z[i];
    }
    acc %= M;
  }
  if (acc < 0) acc += M;
  if (values) values[r] = acc;
  words[r] = ((uint64_t)pid[r] << vbits) | (uint64_t)acc;
}

// equal neighbours in the sorted words: the problem in the word's high bits is not separated
__global__ void k_lattice_dups(int64_t total, const uint64_t* __restrict__ sorted, int vbits, int32_t* __restrict__ bad) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r < 1 || r >= total) return;
  const uint64_t w = sorted[r];
  if (w == sorted[r - 1]) bad[w >> vbits] = 1;
}

inline unsigned lat_grid(int64_t n) { return (unsigned)std::max<int64_t>(1, ceil_div(n, kBlock)); }

uint64_t mulmod(uint64_t a, uint64_t b, uint64_t m) { return (uint64_t)((unsigned __int128)a * b % m); }

uint64_t powmod(uint64_t a, uint64_t e, uint64_t m) {
  uint64_t r = 1 % m;
  a %= m;
  for (; e; e >>= 1, a = mulmod(a, a, m))
    if (e & 1) r = mulmod(r, a, m);
  return r;
}

// Miller-Rabin with the first twelve primes as bases: exact for every n below 3.3e24
bool is_prime(uint64_t n) {
  static const uint64_t bases[] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
  if (n < 2) return false;
  for (uint64_t p : bases) {
    if (n % p == 0) return n == p;
  }
  uint64_t dd = n - 1;
  int s = 0;
  while (!(dd & 1)) dd >>= 1, ++s;
  for (uint64_t a : bases) {
    uint64_t x = powmod(a, dd, n);
    if (x == 1 || x == n - 1) continue;
    bool comp = true;
    for (int i = 1; i < s && comp; ++i) {
      x = mulmod(x, x, n);
      if (x == n - 1) comp = false;
    }
    if (comp) return false;
  }
  return true;
}

}  // namespace

ss_status lattice_modulus_impl(int64_t K, int64_t n, double sigma, int64_t* M) {
  if (!M) return fail(SS_EINVAL, "null output");
  if (K < 0 || n < 0) return fail(SS_EINVAL, "expansion and set size must be non-negative");
  if (!(sigma > 0.0 && sigma <= 1.0)) return fail(SS_EINVAL, "sigma must lie in (0, 1]");
  const double t = std::max((double)K, (double)n * (double)n / sigma);   // the smallest prime > t
  if (!(t < (double)kLatMaxM)) return fail(SS_ERANGE, "the modulus would not fit the 2^40 lattice indices");
  uint64_t c = (uint64_t)std::floor(t) + 1;
  while (!is_prime(c)) ++c;
  if (c > (uint64_t)kLatMaxM) return fail(SS_ERANGE, "the modulus would not fit the 2^40 lattice indices");
  *M = (int64_t)c;
  return SS_OK;
}

ss_status stamp_lattice_impl(const StampImpl* st, const int64_t* z, int64_t M, int64_t* values,
                             int32_t* reconstructing, hipStream_t s) {
  if (!z || !reconstructing) return fail(SS_EINVAL, "null argument");
  if (M < 2 || M > kLatMaxM) return fail(SS_EINVAL, "M must lie in [2, 2^40]");
  for (int i = 0; i < st->d; ++i)
    if (z[i] < 1 || z[i] >= M) return fail(SS_EINVAL, "every z_i must lie in [1, M - 1]");
  if (st->n_prob >= (1 << (63 - kLatBits))) return fail(SS_ERANGE, "too many problems for the sort words");
  const int np = st->n_prob;
  const int64_t n = st->total;
  std::vector<void*> blocks;
  struct Release {
    hipStream_t s;
    std::vector<void*>* b;
    ~Release() {
      (void)hipStreamSynchronize(s);   // queued work may still use the blocks (error paths)
      for (void* p : *b) pool_free(p);
    }
  } rel{s, &blocks};
  int64_t* dz = nullptr;
  uint64_t *w = nullptr, *w2 = nullptr;
  int32_t* bad = nullptr;
  SS_TRY(dalloc(&dz, st->d));
  blocks.push_back(dz);
  SS_TRY(dalloc(&w, n));
  blocks.push_back(w);
  SS_TRY(dalloc(&w2, n));
  blocks.push_back(w2);
  SS_TRY(dalloc(&bad, np));
  blocks.push_back(bad);
  SS_HIP(h2d(dz, z, (size_t)st->d * 8, s));
  SS_HIP(hipMemsetAsync(bad, 0, (size_t)np * 4, s));
  if (n > 0) {
    // sort words: the problem above the vbits bits an index below M needs, as few bits as the sort can take
    int vbits = 1;
    while ((int64_t(1) << vbits) < M) ++vbits;
    if (st->d % 2 == 0)
      k_lattice_values<true><<<lat_grid(n), kBlock, 0, s>>>(n, st->d, st->d_keys, dz, M, st->d_pid, vbits, values, w);
    else
      k_lattice_values<false><<<lat_grid(n), kBlock, 0, s>>>(n, st->d, st->d_keys, dz, M, st->d_pid, vbits, values, w);
    SS_HIP(hipGetLastError());
    int end_bit = vbits;
    while ((int64_t(1) << (end_bit - vbits)) < np) ++end_bit;
    size_t tmp_bytes = 0;
    SS_HIP(hipcub::DeviceRadixSort::SortKeys(nullptr, tmp_bytes, w, w2, n, 0, end_bit, s));
    void* tmp = nullptr;
    SS_TRY(dalloc((char**)&tmp, tmp_bytes));
    blocks.push_back(tmp);
    SS_HIP(hipcub::DeviceRadixSort::SortKeys(tmp, tmp_bytes, w, w2, n, 0, end_bit, s));
    k_lattice_dups<<<lat_grid(n), kBlock, 0, s>>>(n, w2, vbits, bad);
    SS_HIP(hipGetLastError());
  }
  std::vector<int32_t> hb(np);
  SS_HIP(hipMemcpyAsync(hb.data(), bad, (size_t)np * 4, hipMemcpyDeviceToHost, s));
  SS_HIP(hipStreamSynchronize(s));
  for (int p = 0; p < np; ++p) reconstructing[p] = hb[p] ? 0 : 1;
  return SS_OK;
}

}  // namespace ss
