// Stamping-set construction on the GPU (Sec. 6, Eq. StampSet; Alg. 1, step 3).
//
// S^0 = F and S^n = S^{n-1} + supp(a).  Because 0 is in supp(a), S^{n-1} is
// contained in S^n, and every key of S^n \ S^{n-1} is k + w for a key k of
// level n-1 (the frontier) and a nonzero w.  So each level only expands the
// frontier: every (frontier key, w) pair is a candidate, candidates are
// deduplicated through an open-addressing hash table, and the survivors are
// appended as the next frontier.  Among equal candidates the one with the
// smallest (frontier index, w index) wins, so the append order -- and with it
// everything downstream -- is deterministic.  Every key also records the
// forcing frequency its first (winning) path started from; connected classes
// are seeded from that root later.
//
// Hash: h(k) = sum_t k_t Z_t (mod 2^64) is linear, so h(k + w) = h(k) + h(w)
// and a neighbour lookup h(k - w) costs one subtraction.  Each problem owns a
// power-of-two region of the table, sized from the App. A count (exact when no
// sums coincide) and grown per level if needed, so a problem's probes stay in
// one small region (L2-resident while its keys are processed) and a slot
// never has to record its problem.  A slot is 16 bytes: {tag|index, hash};
// keys are verified coordinate by coordinate after a hash match.
//
// Canonical order (per problem, ascending lexicographic, coordinate 0 most
// significant): LSD radix sort over the coordinates, each biased by its
// minimum over the batch and packed into 64-bit words with only the bits its
// range needs (constant coordinates drop out); the problem id is the most
// significant field.
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <cmath>
#include <map>
#include <memory>
#include <set>

#include "ss_internal.h"

namespace ss {

namespace {

std::vector<uint64_t> hash_coefs(int d) {
  std::vector<uint64_t> z(d);
  for (int t = 0; t < d; ++t) z[t] = splitmix64(0x5eed0000ULL + (uint64_t)t * 7919u) | 1ull;
  return z;
}

// the lattice generating vector: entries drawn from [1, M - 1] by a fixed seeded generator
std::vector<uint64_t> lattice_z(int d) {
  std::vector<uint64_t> z(d);
  for (int t = 0; t < d; ++t) z[t] = 1 + splitmix64(0x1a77ce00ULL + (uint64_t)t * 104729u) % (kLatM - 1);
  return z;
}

__host__ __device__ inline uint64_t lat_of_key(const int16_t* k, const uint64_t* z, int d) {
  uint64_t acc = 0;
  for (int t = 0; t < d; ++t)
    if (k[t] != 0) acc = lat_add(acc, lat_mulmod(lat_of_coord(k[t]), z[t]));
  return acc;
}

__device__ inline uint64_t atomic_load_u64(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ void k_hash_keys(int64_t n, int d, const int16_t* __restrict__ keys, const uint64_t* __restrict__ z,
                            uint64_t* __restrict__ out) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint64_t h = 0;
  const int16_t* k = keys + i * d;
  for (int t = 0; t < d; ++t) h += (uint64_t)(int64_t)k[t] * z[t];
  out[i] = h;
}

__global__ void k_insert_main(int64_t n, const uint64_t* __restrict__ hash, const int32_t* __restrict__ pid,
                              const int64_t* __restrict__ toff, const uint64_t* __restrict__ tmask,
                              uint64_t* table) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int p = pid[i];
  const uint64_t h = hash[i], base = (uint64_t)toff[p], mask = tmask[p];
  uint64_t pos = slot_first(h, base, mask);
  while (true) {
    unsigned long long old = atomicCAS((unsigned long long*)&table[pos], 0ull, (unsigned long long)main_word(h, i));
    if (old == 0ull) return;
    pos = slot_next(pos, base, mask);
  }
}

struct ExpandArgs {
  int64_t n_cand;         // frontier size * smax1: an upper bound of the listed candidates
  const uint32_t* n_act;  // the listed candidates (device)
  const uint64_t* cand;   // [n_cand] listed candidates, (frontier key << kJBits) | a-table index
  int32_t d;
  const int16_t* keys;    // unsorted keys
  const uint64_t* hash;
  const int32_t* pid;
  const int16_t* wkeys;   // nonzero a-support, concatenated per problem
  const uint64_t* whash;
  const int32_t* woff;    // [n_prob+1]
  const int64_t* toff;    // [n_prob] first slot of each problem's region
  const uint64_t* tmask;  // [n_prob] region size - 1
  uint64_t* table;        // one word per slot
  uint32_t* cpos;         // [n_cand] slot of the candidate's key (region-relative), or kNoSlot
};

// In generic position every key of level n has a unique representation f + sum of n entries of
// the nonzero a-list, and it is generated exactly once when a key is extended only by entries at
// or after the last one that created it.  A problem runs in that mode until a level yields fewer
// new keys than the App. A count (a coincidence); that level is then completed by a second pass
// with every candidate, and the problem keeps full generation from there on.
__global__ void k_expand(ExpandArgs a) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)*a.n_act) return;
  const uint64_t c = a.cand[t];
  const int64_t i = (int64_t)(c >> kJBits);
  const int j = (int)(c & kJMask);
  const int p = a.pid[i];
  const int wo = a.woff[p];
  const int d = a.d;
  const int16_t* k = a.keys + i * d;
  const int16_t* w = a.wkeys + (int64_t)(wo + j) * d;
  // (every candidate stays in the int16 range: the build checks the ranges of S^n beforehand)
  const uint64_t h = a.hash[i] + a.whash[wo + j];
  const uint64_t my = kTagCand | c;
  const uint64_t base = (uint64_t)a.toff[p], mask = a.tmask[p];
  uint64_t pos = slot_first(h, base, mask);
  while (true) {
    uint64_t v = atomic_load_u64(&a.table[pos]);
    if (v == 0) {
      unsigned long long old = atomicCAS((unsigned long long*)&a.table[pos], 0ull, (unsigned long long)my);
      if (old == 0ull) {
        a.cpos[t] = (uint32_t)(pos - base);
        return;
      }
      v = old;
    }
    if ((v & kTagMask) == kTagMain) {
      const int64_t m = (int64_t)(v & kMainIdxMask);
      if (main_fp_eq(v, h) && key_eq_shift(a.keys + m * d, k, w, 1, d)) {
        a.cpos[t] = kNoSlot;   // already in an earlier level
        return;
      }
    } else {
      const int64_t i2 = (int64_t)((v & kIdxMask) >> kJBits);
      const int j2 = (int)(v & kJMask);
      const uint64_t h2 = a.hash[i2] + a.whash[wo + j2];     // same problem: same region
      if (h2 == h && key_eq_shift2(a.keys + i2 * d, a.wkeys + (int64_t)(wo + j2) * d, k, w, d)) {
        // equal key among this level's candidates: the smallest candidate keeps the slot
        while (my < v) {
          unsigned long long old = atomicCAS((unsigned long long*)&a.table[pos], (unsigned long long)v,
                                             (unsigned long long)my);
          if (old == (unsigned long long)v) break;
          v = old;
        }
        a.cpos[t] = (uint32_t)(pos - base);
        return;
      }
    }
    pos = slot_next(pos, base, mask);
  }
}

__global__ void k_winners(int64_t n_cand, const uint32_t* __restrict__ n_act, const uint64_t* __restrict__ cand,
                          const uint32_t* __restrict__ cpos, const int32_t* __restrict__ pid,
                          const int64_t* __restrict__ toff, const uint64_t* __restrict__ table,
                          uint32_t* __restrict__ flag) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_cand) return;
  uint32_t f = 0;
  if (t < (int64_t)*n_act && cpos[t] != kNoSlot) {
    const uint64_t c = cand[t];
    f = table[(uint64_t)toff[pid[c >> kJBits]] + cpos[t]] == (kTagCand | c) ? 1u : 0u;
  }
  flag[t] = f;
}

__global__ void k_append(ExpandArgs a, const uint32_t* __restrict__ flag, const uint32_t* __restrict__ idx,
                         int64_t base, int16_t* keys_out, uint64_t* hash_out, int32_t* pid_out,
                         int64_t* root, uint8_t* last_out, uint64_t* wide_src) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)*a.n_act || !flag[t]) return;
  const uint64_t c = a.cand[t];
  const int64_t i = (int64_t)(c >> kJBits);
  const int j = (int)(c & kJMask);
  const int p = a.pid[i];
  const int wo = a.woff[p];
  const int d = a.d;
  const int64_t m = base + idx[t];
  const int16_t* k = a.keys + i * d;
  const int16_t* w = a.wkeys + (int64_t)(wo + j) * d;
  int16_t* o = keys_out + m * d;
  if (wide_src) {       // long rows: k_append_keys_wide copies them, a wavefront per row
    wide_src[m - base] = c;
  } else if ((d & 1) == 0) {   // rows are 4-byte aligned: two coordinates per load and store
    const uint32_t* k32 = reinterpret_cast<const uint32_t*>(k);
    const uint32_t* w32 = reinterpret_cast<const uint32_t*>(w);
    uint32_t* o32 = reinterpret_cast<uint32_t*>(o);
    for (int c = 0; c < d; c += 2) {
      const uint32_t x = k32[c >> 1], y = w32[c >> 1];
      const uint32_t lo = (uint32_t)(uint16_t)((int16_t)(x & 0xffffu) + (int16_t)(y & 0xffffu));
      const uint32_t hi = (uint32_t)(uint16_t)((int16_t)(x >> 16) + (int16_t)(y >> 16));
      o32[c >> 1] = lo | (hi << 16);
    }
  } else {
    for (int c = 0; c < d; ++c) o[c] = (int16_t)((int)k[c] + (int)w[c]);
  }
  const uint64_t h = a.hash[i] + a.whash[wo + j];
  hash_out[m] = h;
  pid_out[m] = p;
  last_out[m] = (uint8_t)j;
  root[m] = root[i];
  const uint64_t s = (uint64_t)a.toff[p] + a.cpos[t];
  a.table[s] = main_word(h, (uint64_t)m);
}

// The new key rows of a level for large d: row base + m = parent key + w_j (source word
// wide_src[m] = parent << kJBits | j).  Each wavefront walks rows (grid-stride), its lanes over
// the row's coordinates, two per 32-bit word when d is even, so every load and store of a row is
// contiguous across the lanes.
constexpr unsigned kWideGrid = 2048;   // blocks of the grid-stride wide-row kernels (8 per CU)

__global__ __launch_bounds__(kBlock) void k_append_keys_wide(int64_t n_new, int64_t base, int d,
                                                             const uint64_t* __restrict__ wide_src,
                                                             const int32_t* __restrict__ pid,
                                                             const int32_t* __restrict__ woff,
                                                             const int16_t* __restrict__ wkeys, int16_t* keys) {
  const int lane = threadIdx.x & 63;
  const int64_t waves = (int64_t)gridDim.x * (kBlock / 64);
  for (int64_t m = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; m < n_new; m += waves) {
    const uint64_t c = wide_src[m];
    const int64_t i = (int64_t)(c >> kJBits);
    const int j = (int)(c & kJMask);
    const int16_t* k = keys + i * d;
    const int16_t* w = wkeys + (int64_t)(woff[pid[i]] + j) * d;
    int16_t* o = keys + (base + m) * d;
    if ((d & 1) == 0) {
      const uint32_t* k32 = reinterpret_cast<const uint32_t*>(k);
      const uint32_t* w32 = reinterpret_cast<const uint32_t*>(w);
      uint32_t* o32 = reinterpret_cast<uint32_t*>(o);
      for (int u = lane; u < d / 2; u += 64) {
        const uint32_t x = k32[u], y = w32[u];
        const uint32_t lo = (uint32_t)(uint16_t)((int16_t)(x & 0xffffu) + (int16_t)(y & 0xffffu));
        const uint32_t hi = (uint32_t)(uint16_t)((int16_t)(x >> 16) + (int16_t)(y >> 16));
        o32[u] = lo | (hi << 16);
      }
    } else {
      for (int u = lane; u < d; u += 64) o[u] = (int16_t)((int)k[u] + (int)w[u]);
    }
  }
}

// new keys per problem of the level just built (candidates are grouped by problem)
__global__ void k_level_counts(int n_prob, int64_t f0, const int64_t* __restrict__ fstart,
                               const int64_t* __restrict__ fcount, const uint32_t* __restrict__ coff,
                               const uint32_t* __restrict__ idx, const uint32_t* __restrict__ flag,
                               int64_t* __restrict__ out) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n_prob) return;
  const int64_t c0 = coff[fstart[p] - f0], c1 = coff[fstart[p] + fcount[p] - f0];
  out[p] = c1 > c0 ? (int64_t)idx[c1 - 1] + flag[c1 - 1] - (int64_t)idx[c0] : 0;
}

// Candidates of a level, listed densely: frontier key f0 + t takes its nonzero a-table entries
// from the one that created it on (every entry when its problem generates in full), none once
// its problem's level is reached.  Counts first, then, from their exclusive sum, the list.
__global__ void k_cand_count(int64_t n_front, int64_t f0, const int32_t* __restrict__ pid,
                             const int32_t* __restrict__ woff, const int32_t* __restrict__ plevel, int level,
                             const uint8_t* __restrict__ full, const uint8_t* __restrict__ last,
                             uint32_t* __restrict__ cnt) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t > n_front) return;
  if (t == n_front) {   // the scan's last element: the total lands in coff[n_front]
    cnt[t] = 0;
    return;
  }
  const int64_t i = f0 + t;
  const int p = pid[i];
  const int nw = woff[p + 1] - woff[p];
  cnt[t] = plevel[p] < level ? 0u : (uint32_t)(full[p] ? nw : nw - (int)last[i]);
}

__global__ void k_cand_fill(int64_t n_front, int64_t f0, const int32_t* __restrict__ pid,
                            const uint8_t* __restrict__ full, const uint8_t* __restrict__ last,
                            const uint32_t* __restrict__ coff, uint64_t* __restrict__ cand) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_front) return;
  const int64_t i = f0 + t;
  const uint32_t c0 = coff[t], n = coff[t + 1] - c0;
  const uint32_t lo = full[pid[i]] ? 0u : (uint32_t)last[i];
  for (uint32_t q = 0; q < n; ++q) cand[c0 + q] = ((uint64_t)i << kJBits) | (uint64_t)(lo + q);
}

// one packed field of a radix pass: coordinate t (or -1 = problem id), minus `lo`, at bit `shift`
struct Field {
  int32_t t;
  int32_t lo;
  int32_t shift;
  int32_t pad;
};

__global__ void k_digits(int64_t n, int d, const int16_t* __restrict__ keys, const int32_t* __restrict__ pid,
                         const uint32_t* __restrict__ perm, const Field* __restrict__ fields, int f0, int f1,
                         uint64_t* __restrict__ out) {
  int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  const int64_t s = perm ? perm[r] : r;
  const int16_t* k = keys + s * d;
  uint64_t v = 0;
  for (int q = f0; q < f1; ++q) {
    const Field f = fields[q];
    const int val = f.t >= 0 ? (int)k[f.t] : pid[s];
    v |= (uint64_t)(uint32_t)(val - f.lo) << f.shift;
  }
  out[r] = v;
}

// Every least-significant-first word of every row at once, a thread per (row, pass): a pass packs
// consecutive coordinates, so the threads of a row read it contiguously; out[q * n + r].
__global__ void k_digits_all(int64_t n, int n_pass, int d, const int16_t* __restrict__ keys,
                             const int32_t* __restrict__ pid, const Field* __restrict__ fields,
                             const int2* __restrict__ prange, uint64_t* __restrict__ out) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n * n_pass) return;
  const int64_t r = g / n_pass;
  const int q = (int)(g % n_pass);
  const int16_t* k = keys + r * d;
  uint64_t v = 0;
  for (int f = prange[q].x; f < prange[q].y; ++f) {
    const Field F = fields[f];
    const int val = F.t >= 0 ? (int)k[F.t] : pid[r];
    v |= (uint64_t)(uint32_t)(val - F.lo) << F.shift;
  }
  out[(int64_t)q * n + r] = v;
}

// flag = 1 if two neighbours of the sorted words are equal
__global__ void k_adjacent_ties(int64_t n, const uint64_t* __restrict__ w, int32_t* flag) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= 1 && r < n && w[r] == w[r - 1]) *flag = 1;
}

__global__ void k_gather_u64(int64_t n, const uint32_t* __restrict__ perm, const uint64_t* __restrict__ src,
                             uint64_t* __restrict__ dst) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r < n) dst[r] = src[perm[r]];
}

__global__ void k_iota_u32(int64_t n, uint32_t* p) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = (uint32_t)i;
}

// 64-bit sums over a wavefront (two 32-bit shuffles per step)
__device__ inline uint64_t shfl_xor_u64(uint64_t v, int m) {
  const uint32_t lo = __shfl_xor((uint32_t)v, m, 64), hi = __shfl_xor((uint32_t)(v >> 32), m, 64);
  return (uint64_t)hi << 32 | lo;
}

// k_permute_rows for large d: each wavefront walks sorted rows (grid-stride), its lanes over the
// coordinates (the source row and the output row are read and written contiguously); hash, |k|^2
// and lattice value summed over the lanes; one atomic per block for the largest |k|^2.
__global__ __launch_bounds__(kBlock) void k_permute_rows_wide(
    int64_t n, int d, const uint32_t* __restrict__ perm, const int16_t* __restrict__ ukeys,
    const uint64_t* __restrict__ words, int pid_shift, int pid_bits, const int64_t* __restrict__ lstart, int n_lev,
    const uint64_t* __restrict__ z, const uint64_t* __restrict__ lz, int16_t* __restrict__ keys, uint64_t* hash,
    uint64_t* lat, int32_t* pid, uint8_t* lev, int64_t* norm, uint32_t* inv, unsigned long long* max_norm) {
  const int lane = threadIdx.x & 63;
  const int64_t waves = (int64_t)gridDim.x * (kBlock / 64);
  int64_t nmax = 0;
  for (int64_t r = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; r < n; r += waves) {
    int64_t nn = 0;
    const int64_t s = perm[r];
    const int16_t* src = ukeys + s * d;
    int16_t* dst = keys + r * d;
    uint64_t h = 0;
    LatAcc la;
    for (int t = lane; t < d; t += 64) {
      const int v = src[t];
      dst[t] = (int16_t)v;
      h += (uint64_t)(int64_t)v * z[t];
      nn += (int64_t)v * v;
      la.add(v, lz[t]);
    }
    for (int m = 32; m > 0; m >>= 1) {
      h += shfl_xor_u64(h, m);
      nn += (int64_t)shfl_xor_u64((uint64_t)nn, m);
      la.lo += (int64_t)shfl_xor_u64((uint64_t)la.lo, m);
      la.hi += (int64_t)shfl_xor_u64((uint64_t)la.hi, m);
    }
    const uint64_t lv_ = la.value();
    if (lane == 0) {
      int lvl = 0;
      for (int q = 1; q < n_lev; ++q) lvl = lstart[q] <= s ? q : lvl;
      hash[r] = h;
      lat[r] = lv_;
      pid[r] = pid_bits > 0 ? (int32_t)((words[r] >> pid_shift) & ((uint64_t(1) << pid_bits) - 1)) : 0;
      lev[r] = (uint8_t)lvl;
      norm[r] = nn;
      inv[s] = (uint32_t)r;
    }
    nmax = nn > nmax ? nn : nmax;
  }
  __shared__ int64_t wmax[kBlock / 64];
  if (lane == 0) wmax[threadIdx.x >> 6] = nmax;
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t m = wmax[0];
    for (int q = 1; q < kBlock / 64; ++q) m = wmax[q] > m ? wmax[q] : m;
    atomicMax(max_norm, (unsigned long long)m);
  }
}

// Sorted row r from unsorted row perm[r]: the key (copied in 32-bit words when d is even); the
// problem id from the top bits of the row's sorted word; the level from where the unsorted row
// lies (levels were appended in order: level n holds rows [lstart[n], lstart[n+1])); hash and
// |k|^2 formed from the key on the way; inv[perm[r]] = r; the block maximum of |k|^2, one atomic
// per block.
__global__ void k_permute_rows(int64_t n, int d, const uint32_t* __restrict__ perm, const int16_t* __restrict__ ukeys,
                               const uint64_t* __restrict__ words, int pid_shift, int pid_bits,
                               const int64_t* __restrict__ lstart, int n_lev, const uint64_t* __restrict__ z,
                               const uint64_t* __restrict__ lz, int16_t* __restrict__ keys, uint64_t* hash,
                               uint64_t* lat, int32_t* pid, uint8_t* lev, int64_t* norm, uint32_t* inv,
                               unsigned long long* max_norm) {
  int64_t r = xcd_tid();
  int64_t nn = 0;
  if (r < n) {
    const int64_t s = perm[r];
    const int16_t* src = ukeys + s * d;
    int16_t* dst = keys + r * d;
    uint64_t h = 0;
    LatAcc la;
    if ((d & 1) == 0) {
      const uint32_t* s32 = reinterpret_cast<const uint32_t*>(src);
      uint32_t* d32 = reinterpret_cast<uint32_t*>(dst);
      for (int t = 0; t < d; t += 2) {
        const uint32_t w = s32[t >> 1];
        d32[t >> 1] = w;
        const int64_t lo = (int16_t)(w & 0xffffu), hi = (int16_t)(w >> 16);
        h += (uint64_t)lo * z[t] + (uint64_t)hi * z[t + 1];
        nn += lo * lo + hi * hi;
        la.add((int)lo, lz[t]);
        la.add((int)hi, lz[t + 1]);
      }
    } else {
      for (int t = 0; t < d; ++t) {
        const int64_t v = src[t];
        dst[t] = (int16_t)v;
        h += (uint64_t)v * z[t];
        nn += v * v;
        la.add((int)v, lz[t]);
      }
    }
    lat[r] = la.value();
    int lv = 0;
    for (int q = 1; q < n_lev; ++q) lv = lstart[q] <= s ? q : lv;
    hash[r] = h;
    pid[r] = pid_bits > 0 ? (int32_t)((words[r] >> pid_shift) & ((uint64_t(1) << pid_bits) - 1)) : 0;
    lev[r] = (uint8_t)lv;
    norm[r] = nn;
    inv[s] = (uint32_t)r;
  }
  for (int off = 32; off > 0; off >>= 1) {
    const int64_t o = __shfl_xor(nn, off, 64);
    nn = o > nn ? o : nn;
  }
  __shared__ int64_t wmax[kBlock / 64];
  if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = nn;
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t m = wmax[0];
    for (int q = 1; q < kBlock / 64; ++q) m = wmax[q] > m ? wmax[q] : m;
    atomicMax(max_norm, (unsigned long long)m);
  }
}

__global__ void k_root_out(int64_t n, const uint32_t* __restrict__ perm, const int64_t* __restrict__ uroot,
                           const uint32_t* __restrict__ inv, int64_t* __restrict__ root) {
  int64_t r = xcd_tid();
  if (r < n) root[r] = inv[uroot[perm[r]]];
}

// the lookup table from the build table, in place: same slots, one word each; with inv the build
// table still holds unsorted indices, which are mapped to canonical ones on the way.  Every slot
// is rewritten by its own thread only, and empty slots (most of them) are not written at all.
__global__ void k_lookup_table(uint64_t n_slots, uint64_t* table, const uint32_t* __restrict__ inv) {
  uint64_t s = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n_slots) return;
  const uint64_t v = table[s];
  if (v == 0) return;
  uint64_t out = 0;
  if ((v & kTagMask) == kTagMain) {
    const uint64_t m = v & kMainIdxMask;
    out = lslot_from_fp((v >> 31) & 0x7fffffffull, inv ? (uint64_t)inv[m] : m);
  }
  table[s] = out;
}


// first row of every problem (every problem has keys: F is not empty), and n after the last
__global__ void k_rowoff(int64_t n, int n_prob, const int32_t* __restrict__ pid, int64_t* rowoff) {
  int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  if (r == 0 || pid[r] != pid[r - 1]) rowoff[pid[r]] = r;
  if (r == n - 1) rowoff[n_prob] = n;
}

__global__ void k_iota_i64(int64_t n, int64_t* p) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = i;
}

// f in canonical order: zero, then each given forcing coefficient at its recorded slot
__global__ void k_scatter_f(int64_t n_f, const uint32_t* __restrict__ slot, const double2* __restrict__ vals,
                            double2* f) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n_f) f[slot[i]] = vals[i];
}

__global__ void k_zero_c128(int64_t n, double2* f) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) f[i] = make_double2(0.0, 0.0);
}

__global__ void k_lookup(int64_t nq, int d, const int16_t* __restrict__ q, int32_t prob,
                         const int32_t* __restrict__ probs, const uint64_t* __restrict__ z,
                         const int16_t* __restrict__ keys, const int64_t* __restrict__ toff,
                         const uint64_t* __restrict__ tmask, const uint64_t* __restrict__ lt,
                         const int64_t* rowoff, int64_t* out) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nq) return;
  const int pq = probs ? probs[i] : prob;
  const int16_t* k = q + i * d;
  uint64_t h = 0;
  for (int t = 0; t < d; ++t) h += (uint64_t)(int64_t)k[t] * z[t];
  const uint64_t base = (uint64_t)toff[pq], mask = tmask[pq];
  uint64_t pos = slot_first(h, base, mask);
  int64_t res = -1;
  while (true) {
    const uint64_t v = lt[pos];
    if (v == 0) break;
    const int64_t m = lslot_idx(v);
    if (lslot_fp_eq(v, h)) {
      int acc = 0;
      for (int t = 0; t < d; ++t) acc |= (int)keys[m * d + t] ^ (int)k[t];
      if (acc == 0) {
        res = probs ? m : m - rowoff[pq];
        break;
      }
    }
    pos = slot_next(pos, base, mask);
  }
  out[i] = res;
}

inline unsigned grid_for(int64_t n) { return (unsigned)std::max<int64_t>(1, ceil_div(n, kBlock)); }

template <typename T>
ss_status grow(T** p, int64_t* cap, int64_t need, int64_t keep, int mult, hipStream_t stream) {
  if (need <= *cap) return SS_OK;
  int64_t ncap = std::max<int64_t>(need, *cap * 2);
  T* q = nullptr;
  SS_TRY(dalloc(&q, (size_t)ncap * mult));
  if (keep > 0 && *p) SS_HIP(hipMemcpyAsync(q, *p, (size_t)keep * mult * sizeof(T), hipMemcpyDeviceToDevice, stream));
  SS_HIP(hipStreamSynchronize(stream));
  dfree(*p);
  *p = q;
  *cap = ncap;
  return SS_OK;
}

uint64_t next_pow2(uint64_t x) {
  uint64_t p = 1;
  while (p < x) p <<= 1;
  return p;
}

int bits_for(uint64_t range) {   // bits to hold 0..range
  int b = 0;
  while (b < 64 && (range >> b) != 0) ++b;
  return b;
}

// App. A count for |F| forcing frequencies, s support points, level N (capped)
double app_a_count(int64_t n_f, int s, int N) {
  const int half = (s - 1) / 2;
  auto comb = [](int n, int k) -> double {
    if (n == -1 && k == -1) return 1;
    if (n < 0 || k < 0 || k > n) return 0;
    double c = 1;
    for (int q = 1; q <= k; ++q) c = c * (n - k + q) / q;
    return c;
  };
  double tot = 0;
  for (int n = 0; n <= N; ++n)
    for (int t = 0; t <= std::min(n, half); ++t) tot += std::ldexp(1.0, t) * comb(half, t) * comb(n - 1, t - 1);
  return tot * (double)n_f;
}

// Owns scratch device allocations of one build; frees them on every exit path.
struct Scratch {
  hipStream_t stream = nullptr;
  std::vector<void**> slots;
  std::vector<void*> retired;   // no longer used by the host, maybe still by queued work
  explicit Scratch(hipStream_t s) : stream(s) {}
  // p's block (whatever p points to when the scratch ends) is freed then; p must outlive the
  // scratch, so it is declared before it
  template <typename T>
  void hold(T*& p) {
    slots.push_back((void**)&p);
  }
  // p goes back to the pool at the next release_retired(), which follows a stream sync
  template <typename T>
  void retire(T*& p) {
    if (p) retired.push_back((void*)p);
    p = nullptr;
  }
  void release_retired() {
    for (void* q : retired) pool_free(q);
    retired.clear();
  }
  ~Scratch() {
    (void)hipStreamSynchronize(stream);   // queued work may still use the blocks (error paths)
    release_retired();
    for (void** s : slots)
      if (*s) {
        pool_free(*s);
        *s = nullptr;
      }
  }
};

// Rows of at least this many coordinates are copied a wavefront per row (contiguous loads and
// stores across the lanes) rather than a thread per row.
constexpr int kWideD = 32;

// Slots per key when a region is sized: a load factor of at most 1/4 keeps linear-probe
// sequences short (a lookup costs a cache line per probe; the lanes of a wave wait for the
// longest sequence among them).  A region is grown when it would pass a load of 1/2.
constexpr int kSlotsPerKey = 4;

// Lay out per-problem table regions of the given capacities and insert keys [0, n).
ss_status layout_table(StampImpl* st, const std::vector<uint64_t>& cap, int64_t n, const uint64_t* hash,
                       const int32_t* pid, hipStream_t stream) {
  const int np = st->n_prob;
  std::vector<uint64_t> om(2 * (size_t)np);   // region offsets, then region masks
  uint64_t total = 0;
  for (int p = 0; p < np; ++p) {
    om[p] = total;
    om[np + p] = cap[p] - 1;
    total += cap[p];
  }
  if (total >= (uint64_t(1) << 40)) return fail(SS_ERANGE, "hash table too large");
  if (st->d_table) {   // queued work (the last k_append) may still write the old table
    SS_HIP(hipStreamSynchronize(stream));
    dfree(st->d_table);
  }
  SS_TRY(dalloc(&st->d_table, total));
  if (!st->d_toff) {   // offsets and masks in one block (d_tmask is a view into it)
    SS_TRY(dalloc(&st->d_toff, 2 * (size_t)np));
    st->d_tmask = reinterpret_cast<uint64_t*>(st->d_toff + np);
  }
  SS_HIP(hipMemsetAsync(st->d_table, 0, total * 8, stream));
  SS_HIP(h2d(st->d_toff, om.data(), om.size() * 8, stream));
  st->n_slots = total;
  st->tcap = cap;
  if (n > 0) k_insert_main<<<grid_for(n), kBlock, 0, stream>>>(n, hash, pid, st->d_toff, st->d_tmask, st->d_table);
  return SS_OK;
}

}  // namespace

// ---------------------------------------------------------------- canonical a
ss_status canonical_a(int32_t d, int32_t n_a, const int16_t* freqs, const double* coef,
                      bool drop_zero_coef, ATable* out) {
  if (n_a <= 0 || !freqs) return fail(SS_EINVAL, "supp(a) must be a non-empty list");
  // the given entries (e < n_a) and their negations (e >= n_a, conjugate coefficients), sorted
  // lexicographically: each key is packed big-endian into 64-bit words of four offset-binary
  // coordinates, so comparing words compares keys
  const int n2 = 2 * n_a, nw = (d + 3) / 4;
  thread_local std::vector<uint64_t> W;
  thread_local std::vector<int> idx;
  thread_local std::vector<double2> C;
  W.assign((size_t)n2 * nw, 0);
  C.resize(n2);
  idx.resize(n2);
  double scale = 0;
  for (int i = 0; i < n_a; ++i) {
    const double2 c = coef ? make_double2(coef[2 * i], coef[2 * i + 1]) : make_double2(1.0, 0.0);
    if (!std::isfinite(c.x) || !std::isfinite(c.y)) return fail(SS_EINVAL, "a_hat is not finite");
    scale = std::max(scale, cabs2d(c.x, c.y));
    C[i] = c;
    C[n_a + i] = make_double2(c.x, -c.y);
    for (int t = 0; t < d; ++t) {
      const int v = freqs[(int64_t)i * d + t];
      if (v == -32768) return fail(SS_ERANGE, "a frequency coordinate -32768 has no int16 negation");
      const int sh = 48 - 16 * (t & 3);
      W[(size_t)i * nw + t / 4] |= (uint64_t)(uint16_t)(v + 32768) << sh;
      W[(size_t)(n_a + i) * nw + t / 4] |= (uint64_t)(uint16_t)(-v + 32768) << sh;
    }
  }
  const uint64_t* Wp = W.data();
  auto cmp = [&](int x, int y) {   // -1, 0, 1 on keys only
    const uint64_t* a = Wp + (size_t)x * nw;
    const uint64_t* b = Wp + (size_t)y * nw;
    for (int q = 0; q < nw; ++q)
      if (a[q] != b[q]) return a[q] < b[q] ? -1 : 1;
    return 0;
  };
  // sort the given entries; negation reverses lexicographic order, so the derived entries in
  // ascending order are the negations of the given ones from the largest down; merge the two
  // (on equal keys the given entry first)
  thread_local std::vector<int> sg;
  sg.resize(n_a);
  for (int i = 0; i < n_a; ++i) sg[i] = i;
  std::sort(sg.begin(), sg.end(), [&](int x, int y) {
    const int c = cmp(x, y);
    return c != 0 ? c < 0 : x < y;
  });
  for (int i = 0, k = n_a - 1, o = 0; i < n_a || k >= 0;) {
    if (k < 0 || (i < n_a && cmp(sg[i], n_a + sg[k]) <= 0))
      idx[o++] = sg[i++];
    else
      idx[o++] = n_a + sg[k--];
  }
  out->d = d;
  out->keys.clear();
  out->coef.clear();
  out->zero = -1;
  for (int g0 = 0; g0 < n2;) {
    int g1 = g0 + 1;
    while (g1 < n2 && cmp(idx[g0], idx[g1]) == 0) ++g1;
    int n_given = 0;
    for (int q = g0; q < g1; ++q) n_given += idx[q] < n_a;
    if (n_given > 1) return fail(SS_EINVAL, "duplicate frequency in supp(a)");
    const int e = idx[g0];
    const double2 c = C[e];   // the given coefficient if there is one, else the conjugate of -w's
    if (coef)
      for (int q = g0 + 1; q < g1; ++q) {
        const double2 o = C[idx[q]];
        if (cabs2d(o.x - c.x, o.y - c.y) > 1e-14 * scale)
          return fail(SS_EINVAL, "coefficients at w and -w are not complex conjugates (a must be real)");
      }
    const int16_t* src = freqs + (int64_t)(e < n_a ? e : e - n_a) * d;
    const int sign = e < n_a ? 1 : -1;
    bool is_zero = true;
    for (int t = 0; t < d; ++t) is_zero &= src[t] == 0;
    double2 cv = c;
    if (is_zero && coef) {
      if (std::fabs(c.y) > 1e-14 * scale || c.x <= 0) return fail(SS_EINVAL, "a_0 must be real and positive");
      cv.y = 0;
    }
    g0 = g1;
    if (coef && drop_zero_coef && !is_zero && cv.x == 0 && cv.y == 0) continue;
    if (is_zero) out->zero = out->size();
    for (int t = 0; t < d; ++t) out->keys.push_back((int16_t)(sign * src[t]));
    out->coef.push_back(cv);
  }
  if (out->zero < 0) return fail(SS_EINVAL, "0 must be in supp(a) (a_0 > 0 for a positive coefficient)");
  if (out->size() > kMaxA) return fail(SS_ERANGE, "|supp(a)| after closing under negation exceeds 127");
  return SS_OK;
}

// ---------------------------------------------------------------- build
ss_status build_stamp_impl(int32_t n_prob, int32_t d, const int32_t* n_a, const int16_t* a_freqs,
                           const int32_t* n_f, const int16_t* f_freqs, const int32_t* level,
                           hipStream_t stream, StampImpl** out) {
  *out = nullptr;
  if (n_prob < 1 || n_prob > kMaxProblems) return fail(SS_EINVAL, "n_prob must be in [1, 16383]");
  if (d < 1 || d > 1024) return fail(SS_EINVAL, "d must be in [1, 1024]");
  if (!n_a || !a_freqs || !n_f || !f_freqs || !level) return fail(SS_EINVAL, "null argument");
  StampImpl* st = new StampImpl();
  std::unique_ptr<StampImpl, void (*)(StampImpl*)> guard(st, free_stamp_impl);
  st->d = d;
  st->n_prob = n_prob;
  st->level.assign(level, level + n_prob);
  st->a_off.assign(n_prob + 1, 0);

  // ---- host: canonical a-tables, validation
  const std::vector<uint64_t> z = hash_coefs(d);
  const std::vector<uint64_t> lz = lattice_z(d);
  std::vector<int16_t> wkeys;
  std::vector<uint64_t> ahash, whash, alat;
  std::vector<int64_t> anorm;
  std::vector<int32_t> woff(n_prob + 1, 0), f_off(n_prob + 1, 0), s_of(n_prob);
  int max_level = 0, smax1 = 1;
  int64_t a_pos = 0;
  // coordinate ranges of the stamped keys: S^n holds f + n w for every f in F and w in supp(a)
  // (0 in supp(a) gives every shorter sum), so coordinate t spans exactly
  // [min_f f_t + n min_w w_t, max_f f_t + n max_w w_t] over the batch
  std::vector<int64_t> kmin(d, INT64_MAX), kmax(d, INT64_MIN);
  std::vector<int> fidx;
  ATable at;   // reused across problems
  for (int p = 0; p < n_prob; ++p) {
    if (level[p] < 0 || level[p] > 255) return fail(SS_EINVAL, "level must be in [0, 255]");
    if (n_a[p] < 1) return fail(SS_EINVAL, "every problem needs a non-empty supp(a)");
    if (n_f[p] < 1) return fail(SS_EINVAL, "every problem needs at least one forcing frequency");
    max_level = std::max(max_level, level[p]);
    SS_TRY(canonical_a(d, n_a[p], a_freqs + a_pos * d, nullptr, false, &at));
    a_pos += n_a[p];
    st->a_zero.push_back(at.zero);
    s_of[p] = at.size();
    for (int j = 0; j < at.size(); ++j) {
      const int16_t* kj = at.key(j);
      st->a_keys.insert(st->a_keys.end(), kj, kj + d);
      uint64_t h = 0;
      int64_t nn = 0;
      for (int t = 0; t < d; ++t) {
        h += (uint64_t)(int64_t)kj[t] * z[t];
        nn += (int64_t)kj[t] * kj[t];
      }
      ahash.push_back(h);
      anorm.push_back(nn);
      alat.push_back(lat_of_key(kj, lz.data(), d));
      if (j != at.zero) {
        wkeys.insert(wkeys.end(), kj, kj + d);
        whash.push_back(h);
      }
    }
    st->a_off[p + 1] = st->a_off[p] + at.size();
    for (int t = 0; t < d; ++t) {
      int64_t wlo = 0, whi = 0, flo = INT64_MAX, fhi = INT64_MIN;
      for (int j = 0; j < at.size(); ++j) {
        wlo = std::min<int64_t>(wlo, at.key(j)[t]);
        whi = std::max<int64_t>(whi, at.key(j)[t]);
      }
      for (int i = f_off[p]; i < f_off[p] + n_f[p]; ++i) {
        flo = std::min<int64_t>(flo, f_freqs[(int64_t)i * d + t]);
        fhi = std::max<int64_t>(fhi, f_freqs[(int64_t)i * d + t]);
      }
      kmin[t] = std::min(kmin[t], flo + (int64_t)level[p] * wlo);
      kmax[t] = std::max(kmax[t], fhi + (int64_t)level[p] * whi);
    }
    woff[p + 1] = woff[p] + at.size() - 1;
    smax1 = std::max<int>(smax1, at.size() - 1);
    f_off[p + 1] = f_off[p] + n_f[p];
    fidx.resize(n_f[p]);
    for (int i = 0; i < n_f[p]; ++i) fidx[i] = f_off[p] + i;
    const int16_t* fk = f_freqs;
    auto fless = [&](int x, int y) {
      return std::lexicographical_compare(fk + (int64_t)x * d, fk + (int64_t)(x + 1) * d, fk + (int64_t)y * d,
                                          fk + (int64_t)(y + 1) * d);
    };
    std::sort(fidx.begin(), fidx.end(), fless);
    for (int i = 1; i < n_f[p]; ++i)
      if (!fless(fidx[i - 1], fidx[i])) return fail(SS_EINVAL, "duplicate forcing frequency within a problem");
  }
  const int64_t nF = f_off[n_prob];
  for (int t = 0; t < d; ++t)
    if (kmin[t] < INT16_MIN || kmax[t] > INT16_MAX)
      return fail(SS_ERANGE, "a stamped frequency coordinate leaves the int16 range");
  SS_HIP(hipGetDevice(&st->device));

  // ---- device a-tables (kept by the stamp), one transfer
  {
    Upload up;
    up.add(&st->d_latz, lz.data(), d);
    up.add(&st->d_alat, alat.data(), alat.size());
    up.add(&st->d_akeys, st->a_keys.data(), st->a_keys.size());
    up.add(&st->d_ahash, ahash.data(), ahash.size());
    up.add(&st->d_anorm, anorm.data(), anorm.size());
    up.add(&st->d_aoff, st->a_off.data(), n_prob + 1);
    up.add(&st->d_azero, st->a_zero.data(), n_prob);
    up.add(&st->d_coef, z.data(), d);
    SS_TRY(up.commit(&st->d_upload, stream));
  }

  // ---- build scratch: every pointer the scratch frees is declared before it, so each is still
  // alive when the scratch's destructor reads it
  int16_t* wk = nullptr;
  uint64_t* wh = nullptr;
  int32_t *wo = nullptr, *plev = nullptr;
  int16_t* ukeys = nullptr;
  uint64_t* uhash = nullptr;
  int32_t* upid = nullptr;
  uint8_t* ulast = nullptr;
  uint8_t* d_full = nullptr;
  int64_t* uroot = nullptr;
  uint32_t *cpos = nullptr, *flag = nullptr, *idx = nullptr, *ccnt = nullptr, *coff = nullptr;
  uint64_t* cand = nullptr;
  uint64_t* wsrc = nullptr;              // large d: source words of a level's new rows
  const bool wide = d >= kWideD;
  int64_t *d_fstart = nullptr, *d_fcount = nullptr, *d_cnt = nullptr;
  void* tmp = nullptr;
  void* d_in = nullptr;   // wk, wh, wo and plev are views into it
  Field* d_fields = nullptr;
  uint32_t *perm = nullptr, *perm2 = nullptr;
  uint64_t *k64 = nullptr, *k64b = nullptr;
  uint64_t* wq = nullptr;   // a later pass's words in unsorted order, gathered through the permutation
  int2* d_pr = nullptr;
  int32_t* d_tie = nullptr;
  int64_t* d_lstart = nullptr;
  Scratch sc(stream);
  sc.hold(d_in);
  sc.hold(ukeys); sc.hold(uhash); sc.hold(upid); sc.hold(uroot);
  sc.hold(ulast); sc.hold(d_full);
  sc.hold(cpos); sc.hold(flag); sc.hold(idx); sc.hold(tmp); sc.hold(ccnt); sc.hold(coff); sc.hold(cand); sc.hold(wsrc);
  sc.hold(d_fstart); sc.hold(d_cnt);
  sc.hold(d_fields); sc.hold(perm); sc.hold(perm2); sc.hold(k64); sc.hold(k64b); sc.hold(wq);
  sc.hold(d_pr); sc.hold(d_tie); sc.hold(d_lstart);
  {
    Upload up;
    up.add(&wk, wkeys.data(), wkeys.size());
    up.add(&wh, whash.data(), whash.size());
    up.add(&wo, woff.data(), n_prob + 1);
    up.add(&plev, level, n_prob);
    SS_TRY(up.commit(&d_in, stream));
  }
  SS_TRY(dalloc(&d_fstart, 2 * (size_t)n_prob));   // the level's frontier starts, then its counts
  d_fcount = d_fstart + n_prob;
  SS_TRY(dalloc(&d_cnt, n_prob));
  SS_TRY(dalloc(&d_full, n_prob));
  SS_HIP(hipMemsetAsync(d_full, 0, n_prob, stream));

  // ---- level 0: F
  // The rows of every level fit the App. A count of the whole build (a bound on |S^N| for any a):
  // when that is moderate the key arrays are allocated once at its size, else they grow per level
  // for the worst case of the level (every candidate new).
  double row_bound_d = 0;
  for (int p = 0; p < n_prob; ++p) row_bound_d += app_a_count(n_f[p], s_of[p], level[p]);
  const int64_t row_bound = row_bound_d <= (double)(int64_t(1) << 27) ? std::max<int64_t>((int64_t)row_bound_d, nF)
                                                                        : INT64_MAX;
  int64_t kcap = row_bound != INT64_MAX ? row_bound : std::max<int64_t>(nF * 4, 1024);
  int64_t kcap_h = kcap, kcap_p = kcap, kcap_r = kcap, kcap_t = kcap;
  SS_TRY(dalloc(&ukeys, (size_t)kcap * d));
  SS_TRY(dalloc(&uhash, kcap));
  SS_TRY(dalloc(&upid, kcap));
  SS_TRY(dalloc(&ulast, kcap));
  SS_TRY(dalloc(&uroot, kcap));
  {
    std::vector<int32_t> fpid(nF);
    for (int p = 0; p < n_prob; ++p)
      for (int i = f_off[p]; i < f_off[p + 1]; ++i) fpid[i] = p;
    SS_HIP(h2d(ukeys, f_freqs, (size_t)nF * d * 2, stream));
    SS_HIP(h2d(upid, fpid.data(), nF * 4, stream));
    SS_HIP(hipMemsetAsync(ulast, 0, nF, stream));
    k_iota_i64<<<grid_for(nF), kBlock, 0, stream>>>(nF, uroot);
    k_hash_keys<<<grid_for(nF), kBlock, 0, stream>>>(nF, d, ukeys, st->d_coef, uhash);
  }
  // per-problem regions sized from the App. A count (grown below if coincidences are rarer than it assumes)
  std::vector<uint64_t> cap(n_prob);
  for (int p = 0; p < n_prob; ++p) {
    const double bound = app_a_count(n_f[p], s_of[p], level[p]);
    const double first = (double)n_f[p] * s_of[p];
    const double want = bound <= (double)(1 << 22) ? bound : first;
    cap[p] = next_pow2((uint64_t)std::max(64.0, kSlotsPerKey * want));
  }
  SS_TRY(layout_table(st, cap, nF, uhash, upid, stream));

  std::vector<int64_t> cnt(n_prob), front(2 * (size_t)n_prob);   // front: starts, then counts
  int64_t* fstart = front.data();
  int64_t* fcount = front.data() + n_prob;
  for (int p = 0; p < n_prob; ++p) {
    cnt[p] = n_f[p];
    fstart[p] = f_off[p];
    fcount[p] = n_f[p];
  }
  int64_t total = nF, f0 = 0, f1 = nF, ccap = 0, fcap = 0;
  std::vector<int64_t> lstart{0};   // first unsorted row of each level
  size_t tmp_bytes = 0;
  std::vector<uint8_t> full(n_prob, 0), redo(n_prob, 0);   // host copy of d_full; problems completed again
  for (int n = 1; n <= max_level; ++n) {
    const int64_t n_front = f1 - f0;
    if (n_front == 0) break;
    const int64_t n_cand = n_front * smax1;
    const int64_t need = std::min(total + n_cand, row_bound);   // worst case: every candidate is new
    if (need > (int64_t(1) << 31)) return fail(SS_ERANGE, "stamping sets exceed 2^31 keys in one batch");
    SS_TRY(grow(&ukeys, &kcap, need, total, d, stream));
    SS_TRY(grow(&uhash, &kcap_h, need, total, 1, stream));
    SS_TRY(grow(&upid, &kcap_p, need, total, 1, stream));
    SS_TRY(grow(&ulast, &kcap_t, need, total, 1, stream));
    SS_TRY(grow(&uroot, &kcap_r, need, total, 1, stream));
    // slots in use after this level: at most the worst case (every candidate new) and at most
    // the App. A count, which bounds |S^n| for any a (the count of coefficient vectors over the
    // +-w pairs with L1 norm <= n, per forcing frequency)
    bool relayout = false;
    for (int p = 0; p < n_prob; ++p) {
      const int64_t worst = cnt[p] + (level[p] >= n ? fcount[p] * (s_of[p] - 1) : 0);
      const double bound = app_a_count(n_f[p], s_of[p], std::min(n, level[p]));
      const int64_t need_p = bound < (double)worst ? (int64_t)std::ceil(bound) : worst;
      if ((uint64_t)need_p * 2 > cap[p]) {
        cap[p] = next_pow2((uint64_t)need_p * kSlotsPerKey);
        relayout = true;
      }
    }
    if (relayout) SS_TRY(layout_table(st, cap, total, uhash, upid, stream));
    if (n_cand > ccap) {   // the last level's k_append may still read them
      sc.retire(cpos);
      sc.retire(flag);
      sc.retire(idx);
      sc.retire(cand);
      sc.retire(wsrc);
      ccap = n_cand;
      SS_TRY(dalloc(&cpos, ccap));
      SS_TRY(dalloc(&flag, ccap));
      SS_TRY(dalloc(&idx, ccap));
      SS_TRY(dalloc(&cand, ccap));
      if (wide) SS_TRY(dalloc(&wsrc, ccap));
    }
    if (n_front + 1 > fcap) {
      sc.retire(ccnt);
      sc.retire(coff);
      fcap = n_front + 1;
      SS_TRY(dalloc(&ccnt, fcap));
      SS_TRY(dalloc(&coff, fcap));
    }
    ExpandArgs ea{n_cand, coff + n_front, cand, d, ukeys, uhash, upid, wk, wh, wo, st->d_toff, st->d_tmask,
                  st->d_table, cpos};
    const unsigned cg = grid_for(n_cand);
    SS_HIP(h2d(d_fstart, front.data(), front.size() * 8, stream));
    std::vector<int64_t> added(n_prob);
    auto scan_u32 = [&](const uint32_t* in, uint32_t* out, int64_t n_items) -> ss_status {
      size_t need_tmp = 0;
      SS_HIP(hipcub::DeviceScan::ExclusiveSum(nullptr, need_tmp, in, out, n_items, stream));
      if (need_tmp > tmp_bytes) {
        sc.retire(tmp);   // an earlier scan of this level may still be queued on it
        SS_HIP(pool_alloc((void**)&tmp, need_tmp));
        tmp_bytes = need_tmp;
      }
      SS_HIP(hipcub::DeviceScan::ExclusiveSum(tmp, tmp_bytes, in, out, n_items, stream));
      return SS_OK;
    };
    // the level's candidates, densely listed from the current generation modes
    auto list_candidates = [&]() -> ss_status {
      k_cand_count<<<grid_for(n_front + 1), kBlock, 0, stream>>>(n_front, f0, upid, wo, plev, n, d_full, ulast,
                                                                 ccnt);
      SS_TRY(scan_u32(ccnt, coff, n_front + 1));
      k_cand_fill<<<grid_for(n_front), kBlock, 0, stream>>>(n_front, f0, upid, d_full, ulast, coff, cand);
      return SS_OK;
    };
    // winners, their positions and the new keys per problem of the listed candidates
    auto count_level = [&]() -> ss_status {
      k_winners<<<cg, kBlock, 0, stream>>>(n_cand, coff + n_front, cand, cpos, upid, st->d_toff, st->d_table, flag);
      SS_TRY(scan_u32(flag, idx, n_cand));
      k_level_counts<<<grid_for(n_prob), kBlock, 0, stream>>>(n_prob, f0, d_fstart, d_fcount, coff, idx, flag,
                                                              d_cnt);
      Readback rb(stream);
      SS_TRY(rb.add(added.data(), d_cnt, n_prob * 8));
      SS_TRY(rb.sync());
      sc.release_retired();
      return SS_OK;
    };
    SS_TRY(list_candidates());
    k_expand<<<cg, kBlock, 0, stream>>>(ea);
    SS_TRY(count_level());
    // a problem generating once per key that found fewer new keys than the App. A count met a
    // coincidence: complete the level with every candidate, and keep doing so
    bool again = false;
    for (int p = 0; p < n_prob; ++p) {
      redo[p] = 0;
      if (full[p] || level[p] < n) continue;
      const int64_t bound = std::llround(app_a_count(n_f[p], s_of[p], n)) -
                            std::llround(app_a_count(n_f[p], s_of[p], n - 1));
      if (added[p] != bound) {
        full[p] = redo[p] = 1;
        again = true;
      }
    }
    if (again) {
      // every candidate of those problems: the list is made again (candidates already inserted
      // find their own or an equal smaller candidate's slot, so repeating them changes nothing)
      SS_HIP(h2d(d_full, full.data(), n_prob, stream));
      SS_TRY(list_candidates());
      k_expand<<<cg, kBlock, 0, stream>>>(ea);
      SS_TRY(count_level());
    }
    k_append<<<cg, kBlock, 0, stream>>>(ea, flag, idx, total, ukeys, uhash, upid, uroot, ulast, wide ? wsrc : nullptr);
    if (wide) {
      int64_t n_new = 0;
      for (int p = 0; p < n_prob; ++p) n_new += added[p];
      if (n_new > 0)
        k_append_keys_wide<<<(unsigned)std::min<int64_t>(kWideGrid, ceil_div(n_new * 64, kBlock)), kBlock, 0,
                             stream>>>(n_new, total, d, wsrc, upid, wo, wk, ukeys);
    }
    f0 = total;
    lstart.push_back(total);
    for (int p = 0; p < n_prob; ++p) {
      fstart[p] = total;
      fcount[p] = added[p];
      cnt[p] += added[p];
      total += added[p];
    }
    f1 = total;
  }
  sc.retire(cpos);   // the last k_append may still read them
  sc.retire(flag);
  sc.retire(idx);
  sc.retire(cand);
  sc.retire(ccnt);
  sc.retire(coff);
  dfree(tmp);        // its last user, a scan, is behind the last sync
  tmp_bytes = 0;

  // ---- canonical order: LSD radix sort over packed, range-biased coordinates, then problem id
  st->total = total;
  std::vector<int32_t> mn(d), mx(d);
  for (int t = 0; t < d; ++t) {
    mn[t] = (int32_t)kmin[t];
    mx[t] = (int32_t)kmax[t];
  }
  // words of <= 64 bits, filled from the least significant coordinate up; the problem id on top
  std::vector<Field> fields;
  std::vector<std::pair<int, int>> passes;   // [first field, end field), bits
  std::vector<int> pass_bits;
  {
    int used = 0, first = 0;
    auto add = [&](int t, int lo, int bits) {
      if (bits == 0) return;
      if (used + bits > 64) {
        passes.emplace_back(first, (int)fields.size());
        pass_bits.push_back(used);
        first = (int)fields.size();
        used = 0;
      }
      fields.push_back(Field{t, lo, used, 0});
      used += bits;
    };
    for (int t = d - 1; t >= 0; --t) add(t, mn[t], bits_for((uint64_t)(mx[t] - mn[t])));
    add(-1, 0, bits_for((uint64_t)(n_prob - 1)));
    if (used > 0) {
      passes.emplace_back(first, (int)fields.size());
      pass_bits.push_back(used);
    }
  }
  // With two words or more, one word packed from the most significant side first:
  // the problem id on top, then coordinates 0, 1, ... while they fit.  If no two keys share it,
  // sorting by it alone gives the canonical order and the LSD passes are skipped.
  const int nf = (int)fields.size();
  int top_bits = 0;
  if (passes.size() >= 2) {
    std::vector<std::pair<int, int>> items{{-1, bits_for((uint64_t)(n_prob - 1))}};   // (t, bits)
    int used = items[0].second;
    for (int t = 0; t < d; ++t) {
      const int b = bits_for((uint64_t)(mx[t] - mn[t]));
      if (used + b > 64) break;
      items.emplace_back(t, b);
      used += b;
    }
    int shift = used;
    for (const auto& it : items) {
      shift -= it.second;
      if (it.second > 0) fields.push_back(Field{it.first, it.first >= 0 ? mn[it.first] : 0, shift, 0});
    }
    top_bits = used;
  }
  SS_TRY(dalloc(&d_fields, std::max<size_t>(fields.size(), 1)));
  if (!fields.empty())
    SS_HIP(h2d(d_fields, fields.data(), fields.size() * sizeof(Field), stream));

  SS_TRY(dalloc(&perm, total));
  SS_TRY(dalloc(&perm2, total));
  SS_TRY(dalloc(&k64, total));
  SS_TRY(dalloc(&k64b, total));
  k_iota_u32<<<grid_for(total), kBlock, 0, stream>>>(total, perm);
  if (!passes.empty()) {
    sc.retire(tmp);   // the level scans' scratch: back to the pool once the stream has passed them
    SS_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, tmp_bytes, k64, k64b, perm, perm2, total, 0, 64, stream));
    SS_HIP(pool_alloc((void**)&tmp, tmp_bytes));
  }
  bool done = false;
  // long rows: every pass's words (and the most-significant word) formed in one read of the keys
  // (the per-pass form would read a row's cache lines once per pass), when they fit 2 GiB
  const int np_ = (int)passes.size();
  const int nw_ = np_ + (top_bits > 0 ? 1 : 0);
  const bool all_words = np_ > 1 && wide && (int64_t)nw_ * total * 8 <= (int64_t(1) << 31);
  if (all_words) {
    std::vector<int2> pr(nw_);
    for (int q = 0; q < np_; ++q) pr[q] = make_int2(passes[q].first, passes[q].second);
    if (top_bits > 0) pr[np_] = make_int2(nf, (int)fields.size());
    SS_TRY(dalloc(&d_pr, nw_));
    SS_HIP(h2d(d_pr, pr.data(), nw_ * sizeof(int2), stream));
    SS_TRY(dalloc(&wq, (size_t)nw_ * total));
    k_digits_all<<<(unsigned)ceil_div((int64_t)nw_ * total, kBlock), kBlock, 0, stream>>>(total, nw_, d, ukeys, upid,
                                                                                           d_fields, d_pr, wq);
  }
  if (top_bits > 0) {
    SS_TRY(dalloc(&d_tie, 1));
    SS_HIP(hipMemsetAsync(d_tie, 0, 4, stream));
    const uint64_t* kin = k64;
    if (all_words)
      kin = wq + (int64_t)np_ * total;
    else
      k_digits<<<grid_for(total), kBlock, 0, stream>>>(total, d, ukeys, upid, nullptr, d_fields, nf,
                                                       (int)fields.size(), k64);
    size_t tb = tmp_bytes;
    SS_HIP(hipcub::DeviceRadixSort::SortPairs(tmp, tb, kin, k64b, perm, perm2, total, 0, top_bits, stream));
    k_adjacent_ties<<<grid_for(total), kBlock, 0, stream>>>(total, k64b, d_tie);
    int32_t tie = 1;
    Readback rb(stream);
    SS_TRY(rb.add(&tie, d_tie, 4));
    SS_TRY(rb.sync());
    if (!tie) {
      std::swap(perm, perm2);
      done = true;
    } else {
      k_iota_u32<<<grid_for(total), kBlock, 0, stream>>>(total, perm);
    }
  }
  if (!all_words && passes.size() > 1 && !done) SS_TRY(dalloc(&wq, total));
  for (size_t q = 0; q < passes.size() && !done; ++q) {
    const uint64_t* kin = k64;
    if (all_words) {
      if (q == 0) kin = wq;
      else k_gather_u64<<<grid_for(total), kBlock, 0, stream>>>(total, perm, wq + q * total, k64);
    } else if (q == 0) {
      k_digits<<<grid_for(total), kBlock, 0, stream>>>(total, d, ukeys, upid, nullptr, d_fields, passes[q].first,
                                                       passes[q].second, k64);
    } else {
      k_digits<<<grid_for(total), kBlock, 0, stream>>>(total, d, ukeys, upid, nullptr, d_fields, passes[q].first,
                                                       passes[q].second, wq);
      k_gather_u64<<<grid_for(total), kBlock, 0, stream>>>(total, perm, wq, k64);
    }
    size_t tb = tmp_bytes;
    SS_HIP(hipcub::DeviceRadixSort::SortPairs(tmp, tb, kin, k64b, perm, perm2, total, 0, pass_bits[q], stream));
    std::swap(perm, perm2);
  }

  // ---- final arrays in canonical order; re-point the hash table at them
  SS_TRY(dalloc(&st->d_keys, (size_t)total * d));
  SS_TRY(dalloc(&st->d_hash, total));
  SS_TRY(dalloc(&st->d_lat, total));
  SS_TRY(dalloc(&st->d_pid, total));
  SS_TRY(dalloc(&st->d_lev, total));
  SS_TRY(dalloc(&st->d_norm, total));
  SS_TRY(dalloc(&st->d_root, total));
  SS_TRY(dalloc(&st->d_rowoff, n_prob + 2));   // row offsets, then the largest |k|^2 (read back together)
  uint32_t* inv = perm2;
  unsigned long long* d_maxn = reinterpret_cast<unsigned long long*>(st->d_rowoff + n_prob + 1);
  SS_HIP(hipMemsetAsync(d_maxn, 0, 8, stream));
  // the problem id sits at the top of the words the last sort ordered (k64b)
  const int pid_bits = bits_for((uint64_t)(n_prob - 1));
  const int pid_shift = (done ? top_bits : (passes.empty() ? 0 : pass_bits.back())) - pid_bits;
  SS_TRY(dalloc(&d_lstart, lstart.size()));
  SS_HIP(h2d(d_lstart, lstart.data(), lstart.size() * sizeof(int64_t), stream));
  if (wide)
    k_permute_rows_wide<<<(unsigned)std::min<int64_t>(kWideGrid, ceil_div(total * 64, kBlock)), kBlock, 0, stream>>>(
        total, d, perm, ukeys, k64b, pid_shift, pid_bits, d_lstart, (int)lstart.size(), st->d_coef, st->d_latz,
        st->d_keys, st->d_hash, st->d_lat, st->d_pid, st->d_lev, st->d_norm, inv, d_maxn);
  else
    k_permute_rows<<<xcd_grid(ceil_div(total, kBlock)), kBlock, 0, stream>>>(total, d, perm, ukeys, k64b, pid_shift, pid_bits, d_lstart,
                                                           (int)lstart.size(), st->d_coef, st->d_latz, st->d_keys,
                                                           st->d_hash, st->d_lat, st->d_pid, st->d_lev, st->d_norm,
                                                           inv, d_maxn);
  k_root_out<<<xcd_grid(ceil_div(total, kBlock)), kBlock, 0, stream>>>(total, perm, uroot, inv, st->d_root);
  // the forcing frequencies are the first nF unsorted keys, in the order given
  st->n_f = nF;
  SS_TRY(dalloc(&st->d_fslot, nF));
  SS_HIP(hipMemcpyAsync(st->d_fslot, inv, nF * 4, hipMemcpyDeviceToDevice, stream));
  {
    // regions sized for the build's worst case are re-laid out for the final counts;
    // otherwise the slots are re-pointed at the canonical rows
    std::vector<uint64_t> tight(n_prob);
    bool shrink = false;
    for (int p = 0; p < n_prob; ++p) {
      tight[p] = next_pow2((uint64_t)std::max<int64_t>(64, kSlotsPerKey * cnt[p]));
      shrink |= tight[p] < cap[p];
    }
    if (shrink) SS_TRY(layout_table(st, tight, total, st->d_hash, st->d_pid, stream));
    // the lookup table takes over the build table's slots
    k_lookup_table<<<(unsigned)ceil_div((int64_t)st->n_slots, kBlock), kBlock, 0, stream>>>(
        st->n_slots, st->d_table, shrink ? nullptr : inv);
    st->d_ltable = st->d_table;
    st->d_table = nullptr;
  }
  k_rowoff<<<grid_for(total), kBlock, 0, stream>>>(total, n_prob, st->d_pid, st->d_rowoff);
  st->row_off.assign(n_prob + 2, 0);
  {
    Readback rb(stream);
    SS_TRY(rb.add(st->row_off.data(), st->d_rowoff, (n_prob + 2) * 8));
    SS_TRY(rb.sync());
  }
  st->max_norm = st->row_off[n_prob + 1];
  st->row_off.pop_back();
  for (int p = 0; p < n_prob; ++p)
    if (st->row_off[p + 1] - st->row_off[p] > kMaxRowsPerProblem)
      return fail(SS_ERANGE, "a stamping set exceeds 4194303 keys");
  *out = guard.release();
  return SS_OK;
}

void free_stamp_impl(StampImpl* st) {
  if (!st) return;
  dfree(st->d_fslot);
  dfree(st->d_upload);   // the a-table arrays are views into it
  dfree(st->d_keys);
  dfree(st->d_lev);
  dfree(st->d_norm);
  dfree(st->d_hash);
  dfree(st->d_pid);
  dfree(st->d_root);
  dfree(st->d_rowoff);
  dfree(st->d_lat);
  dfree(st->d_table);
  dfree(st->d_ltable);
  dfree(st->d_toff);   // d_tmask is a view into it
  delete st;
}

ss_status stamp_lookup_impl(const StampImpl* st, int32_t prob, int64_t nq, const int16_t* q,
                            int64_t* slot_out, hipStream_t stream, const int32_t* probs) {
  if (!probs && (prob < 0 || prob >= st->n_prob)) return fail(SS_EINVAL, "problem index out of range");
  if (nq < 0 || (nq > 0 && (!q || !slot_out))) return fail(SS_EINVAL, "bad query arrays");
  if (probs)
    for (int64_t i = 0; i < nq; ++i)
      if (probs[i] < 0 || probs[i] >= st->n_prob) return fail(SS_EINVAL, "problem index out of range");
  if (nq == 0) return SS_OK;
  int16_t* dq = nullptr;
  int64_t* dout = nullptr;
  int32_t* dp = nullptr;
  Scratch sc(stream);
  sc.hold(dq); sc.hold(dout); sc.hold(dp);
  SS_TRY(dalloc(&dq, (size_t)nq * st->d));
  SS_TRY(dalloc(&dout, nq));
  if (probs) {
    SS_TRY(dalloc(&dp, nq));
    SS_HIP(h2d(dp, probs, nq * 4, stream));
  }
  SS_HIP(h2d(dq, q, (size_t)nq * st->d * 2, stream));
  k_lookup<<<grid_for(nq), kBlock, 0, stream>>>(nq, st->d, dq, prob, dp, st->d_coef, st->d_keys, st->d_toff,
                                                 st->d_tmask, st->d_ltable, st->d_rowoff, dout);
  Readback rb(stream);
  SS_TRY(rb.add(slot_out, dout, nq * 8));
  return rb.sync();
}

ss_status stamp_forcing_impl(const StampImpl* st, const double* f_hat, void* f, hipStream_t stream) {
  if (!f || (st->n_f > 0 && !f_hat)) return fail(SS_EINVAL, "null argument");
  double2* dv = nullptr;
  Scratch sc(stream);
  sc.hold(dv);
  SS_TRY(dalloc(&dv, st->n_f));
  SS_HIP(h2d(dv, f_hat, st->n_f * 16, stream));
  double2* df = static_cast<double2*>(f);
  k_zero_c128<<<grid_for(st->total), kBlock, 0, stream>>>(st->total, df);
  k_scatter_f<<<grid_for(st->n_f), kBlock, 0, stream>>>(st->n_f, st->d_fslot, dv, df);
  return SS_OK;   // Scratch synchronises the stream before releasing the staging block
}

}  // namespace ss
