// Operator construction: the neighbour map of the truncated Galerkin operator
// (Sec. 9, Eq. FiniteGalerkinOperator) and its execution layout.
//
// Row k of L_N has an entry for every w_j in supp(a) with k - w_j in S^N
// (terms with l outside S^N are dropped by the truncation).  The entry value
// 4 pi^2 (k . (k - w_j)) a_j is never stored: with
//     k . (k - w) = (|k|^2 + |k - w|^2 - |w|^2) / 2
// it is rebuilt in the matvec from three exact integer squared norms, so a
// stored entry is just (column, j) packed in 32 bits and the operator is
// independent of d once built.
//
// Layout.  The canonical CSR (rows and columns in canonical slot order,
// entries in a-table order) is kept for export.  The matvec runs on a SELL-64
// layout in an execution order that groups each problem's rows by connected
// class (the independent blocks of Sec. 6, proof of Prop. SolutionSupport),
// then by decreasing row length, so a 64-row slice (one wavefront) holds rows
// of similar length and gathers stay inside one class.  Each problem's rows
// are padded to a multiple of 64.
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <cmath>
#include <memory>

#include "ss_internal.h"

namespace ss {

namespace {

inline unsigned grid_for(int64_t n) { return (unsigned)std::max<int64_t>(1, ceil_div(n, kBlock)); }

struct NbrArgs {
  int64_t total;
  int32_t d;
  int32_t smax;
  int32_t rows_per_wave;          // floor(64 / smax), at least 1
  const int16_t* keys;
  const uint64_t* hash;
  const int32_t* pid;
  const int64_t* rowoff;
  const int16_t* akeys;
  const uint64_t* ahash;
  const int32_t* aoff;
  const int32_t* azero;
  const int64_t* toff;
  const uint64_t* tmask;
  const uint64_t* table;
  uint32_t* buf;       // [smax x total] compact row entries (entry q of row r at q * total + r): local canonical column | j << kColBits
  int64_t* rowlen;     // [total]
  const uint64_t* lat;   // [total] lattice value of every key (lattice lookups)
  const uint64_t* alat;  // [sum s] lattice value of every a-table entry
};

// One lane per (row, a-table index): look up k - w_j; a ballot over the row's lanes compacts the
// hits to the front of the row's buffer in j order.  A table of more than 64 entries takes one wave
// per row, its lanes covering j = 0..63, then 64..127.
template <bool LAT>
__global__ __launch_bounds__(kBlock) void k_neighbors(NbrArgs a) {
  const int lane = threadIdx.x & 63;
  const int64_t n_blocks = ceil_div(ceil_div(a.total, a.rows_per_wave), kBlock / 64);
  const int64_t wave = (xcd_block(n_blocks) * kBlock + threadIdx.x) >> 6;
  const int width = a.smax < 64 ? a.smax : 64;   // lanes per row
  const int rl = lane / width, jl = lane % width;
  const int64_t r = wave * a.rows_per_wave + rl;
  const bool live = rl < a.rows_per_wave && r < a.total;
  const int p = live ? a.pid[r] : 0;
  const int j0 = live ? a.aoff[p] : 0, s = live ? a.aoff[p + 1] - j0 : 0;
  int found = 0;   // entries of this row found in earlier chunks
  for (int jb = 0; jb < a.smax; jb += 64) {
    const int j = jb + jl;
    int64_t col = -1;
    if (live && j < s) {
      if (j == a.azero[p]) {
        col = r;
      } else {
        const int d = a.d;
        const int16_t* k = a.keys + r * d;
        const int16_t* w = a.akeys + (int64_t)(j0 + j) * d;
        const uint64_t h = a.hash[r] - a.ahash[j0 + j];
        const uint64_t lt = LAT ? lat_sub(a.lat[r], a.alat[j0 + j]) : 0;
        const uint64_t base = (uint64_t)a.toff[p], mask = a.tmask[p];
        uint64_t pos = slot_first(h, base, mask);
        while (true) {
          const uint64_t v = a.table[pos];
          if (v == 0) break;
          if (lslot_fp_eq(v, h)) {
            const int64_t m = lslot_idx(v);
            if (LAT ? a.lat[m] == lt : key_eq_shift(a.keys + m * d, k, w, -1, d)) {
              col = m;
              break;
            }
          }
          pos = slot_next(pos, base, mask);
        }
      }
    }
    const uint64_t hits = __ballot(col >= 0);
    const uint64_t seg = width >= 64 ? hits : (hits >> (rl * width)) & ((1ull << width) - 1);
    if (live && col >= 0) {
      const int q = found + __popcll(seg & ((1ull << jl) - 1));
      a.buf[q * a.total + r] = (uint32_t)(col - a.rowoff[p]) | ((uint32_t)j << kColBits);
    }
    found += __popcll(seg);
  }
  if (live && jl == 0) a.rowlen[r] = found;
}

constexpr int kNbrGroup = 8;   // lookup-table words per probe group (64 bytes)

// One lane per row, for dimensions up to DMAX: the row's key and hash stay in registers while
// the lane looks up k - w_j for the upper half of the a-table (see below).  A lookup reads the
// aligned group of G slots that holds its first probe position and scans it from there (linear
// probing stays within the group for nearly every lookup at the table's load factor), so the
// lanes of a wave finish together instead of waiting for the longest probe sequence among them;
// only a lookup that runs past its group continues slot by slot.  A candidate c matches when
// c + w = k coordinatewise (exact in int).  A wave whose rows all belong to one problem reads
// that problem's a-table from LDS.  The CSR built from the table equals k_neighbors'.
template <int DMAX, bool EVEN>
__device__ __forceinline__ bool key_is_shift(const int16_t* __restrict__ cp, const int* kr, const int16_t* w, int d) {
  int acc = 0;
  if (EVEN) {
#pragma unroll
    for (int t2 = 0; t2 < DMAX / 2; ++t2)
      if (2 * t2 < d) {
        const uint32_t v = reinterpret_cast<const uint32_t*>(cp)[t2];
        acc |= ((int)(int16_t)(v & 0xffff) + (int)w[2 * t2]) ^ kr[2 * t2];
        acc |= ((int)(int16_t)(v >> 16) + (int)w[2 * t2 + 1]) ^ kr[2 * t2 + 1];
      }
  } else {
#pragma unroll
    for (int t = 0; t < DMAX; ++t)
      if (t < d) acc |= ((int)cp[t] + (int)w[t]) ^ kr[t];
  }
  return acc == 0;
}

// The neighbour relation is symmetric (the a-table is closed under negation and sorted, so
// w_{s-1-j} = -w_j and w_z = 0 at z = (s-1)/2): a row looks up k - w_j only for j > z, writes
// that entry and, when l = k - w_j is present, the mirror entry (l, s-1-j) = k into l's row.
// Entries go to a dense j-major table (entry j of row r at j * n + r; absent = all ones); the
// lower half of it is cleared beforehand, the upper half and the diagonal are written here.  An
// entry is `local column | j << kColBits` (u32), or the local column alone (u16) when every problem has
// fewer than 65535 keys (j is then the table row the entry sits in).
template <typename E>
__device__ inline E dense_entry(int64_t col, int j) {
  if (sizeof(E) == 2) return (E)col;
  return (E)((uint32_t)col | ((uint32_t)j << kColBits));
}

template <int DMAX, bool EVEN, bool UNI, int G, typename E, bool LAT>
__device__ __forceinline__ void nbr_row(const NbrArgs& a, int64_t r, int p, const int16_t* wtab,
                                        const uint64_t* htab) {
  const int d = a.d;
  int kr[DMAX];
  const int16_t* kp = a.keys + r * d;
  if (LAT) {   // candidates are matched by lattice value: the row's key is not needed
  } else if (EVEN) {
#pragma unroll
    for (int t2 = 0; t2 < DMAX / 2; ++t2) {
      const uint32_t v = 2 * t2 < d ? reinterpret_cast<const uint32_t*>(kp)[t2] : 0u;
      kr[2 * t2] = (int16_t)(v & 0xffff);
      kr[2 * t2 + 1] = (int16_t)(v >> 16);
    }
  } else {
#pragma unroll
    for (int t = 0; t < DMAX; ++t) kr[t] = t < d ? kp[t] : 0;
  }
  const int j0 = a.aoff[p], s = a.aoff[p + 1] - j0, z = a.azero[p];
  const int64_t ro = a.rowoff[p];
  const uint64_t hr = a.hash[r], base = (uint64_t)a.toff[p], mask = a.tmask[p];
  const uint64_t lr = LAT ? a.lat[r] : 0;
  const uint64_t* table = a.table + base;   // lookup table: one word per slot
  E* D = reinterpret_cast<E*>(a.buf);
  constexpr E kNone = (E)~(E)0;
  const int64_t T = a.total;
  D[(int64_t)z * T + r] = dense_entry<E>(r - ro, z);
  for (int j = z + 1; j < s; ++j) {
    int64_t m = -1;
    {
      // (the LDS tables hold the upper half, entries z + 1 .. s - 1)
      const int16_t* w = UNI ? wtab + (j - z - 1) * d : a.akeys + (int64_t)(j0 + j) * d;
      const uint64_t h = hr - (UNI ? htab[j - z - 1] : a.ahash[j0 + j]);
      const uint64_t lt = LAT ? lat_sub(lr, a.alat[j0 + j]) : 0;
      const uint64_t pos = h >> slot_shift(mask);
      const uint64_t g0 = pos & ~(uint64_t)(G - 1);   // regions are multiples of 64 slots: aligned
      uint64_t sv[G];
#pragma unroll
      for (int i = 0; i < G; i += 2) {
        const ulonglong2 two = *reinterpret_cast<const ulonglong2*>(table + g0 + i);
        sv[i] = two.x;
        sv[i + 1] = two.y;
      }
      bool stop = false;         // an empty slot ends the probe sequence
      int64_t cand = -1;         // first slot (local) in probe order whose fingerprint matches
      uint64_t cv = 0;
#pragma unroll
      for (int i = 0; i < G; ++i)
        if ((uint64_t)i >= pos - g0 && !stop && cand < 0) {
          if (sv[i] == 0) {
            stop = true;
          } else if (lslot_fp_eq(sv[i], h)) {
            cand = (int64_t)g0 + i;
            cv = sv[i];
          }
        }
      uint64_t next = g0 + G;    // where a probe sequence that left the group resumes
      if (cand >= 0) {
        const int64_t c = lslot_idx(cv);
        if (LAT ? a.lat[c] == lt : key_is_shift<DMAX, EVEN>(a.keys + c * d, kr, w, d)) {
          m = c;
          stop = true;
        } else {
          next = (uint64_t)cand + 1;   // a fingerprint collision: keep probing after it
          stop = false;
        }
      }
      if (!stop) {
        uint64_t pp = next & mask;
        while (true) {
          const uint64_t v = table[pp];
          if (v == 0) break;
          if (lslot_fp_eq(v, h)) {
            const int64_t c = lslot_idx(v);
            if (LAT ? a.lat[c] == lt : key_is_shift<DMAX, EVEN>(a.keys + c * d, kr, w, d)) {
              m = c;
              break;
            }
          }
          pp = (pp + 1) & mask;
        }
      }
    }
    D[(int64_t)j * T + r] = m >= 0 ? dense_entry<E>(m - ro, j) : kNone;
    if (m >= 0) D[(int64_t)(s - 1 - j) * T + m] = dense_entry<E>(r - ro, s - 1 - j);
  }
}

// The neighbour table as the later kernels read it, row r's slots u at u * total + r (reads of a
// slot are coalesced over consecutive rows):
//   kDense16  slot u = a-table index j, local canonical column or 0xffff (absent);
//   kDense32  slot u = j, `column | j << kColBits` or all ones (absent);
//   kCompact  slots u < rowlen[r], present entries in j order, `column | j << kColBits`.
enum NbrKind { kDense16 = 0, kDense32 = 1, kCompact = 2 };

// row r's entries are read kDenseChunk slots at a time, every load of a chunk in flight
constexpr int kDenseChunk = 8;

template <int K>
struct NbrView {
  static constexpr int kKind = K;
  const void* D;
  int64_t total;
  const int32_t* aoff;
  const int64_t* rowlen;
  __device__ int slots(int p, int64_t r) const {
    return K == kCompact ? (int)rowlen[r] : aoff[p + 1] - aoff[p];
  }
  // slot u of row r: true and (column, j) when an entry is present
  __device__ bool load(int64_t r, int u, uint32_t& v) const {
    if (K == kDense16) {
      const uint16_t x = reinterpret_cast<const uint16_t*>(D)[(int64_t)u * total + r];
      v = (uint32_t)x | ((uint32_t)u << kColBits);
      return x != 0xffffu;
    }
    v = reinterpret_cast<const uint32_t*>(D)[(int64_t)u * total + r];
    return K == kCompact || v != 0xffffffffu;
  }
};

// entries per problem: one block per problem sums the row lengths of its rows (rows of a
// problem are contiguous), in a fixed order
__global__ __launch_bounds__(kBlock) void k_problem_nnz(const int64_t* __restrict__ rowoff,
                                                        const int64_t* __restrict__ rowlen, int64_t* __restrict__ nnz_p) {
  const int p = blockIdx.x;
  const int64_t r0 = rowoff[p], r1 = rowoff[p + 1];
  int64_t c = 0;
  for (int64_t r = r0 + threadIdx.x; r < r1; r += kBlock) c += rowlen[r];
  for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off, 64);
  __shared__ int64_t part[kBlock / 64];
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t t = 0;
    for (int q = 0; q < kBlock / 64; ++q) t += part[q];
    nnz_p[p] = t;
  }
}

template <int DMAX, bool EVEN, typename E, bool LAT>
__global__ __launch_bounds__(kBlock) void k_neighbors_row(NbrArgs a) {
  // the upper half of a mirrored table: at most (kMaxA - 1) / 2 entries
  __shared__ int16_t s_w[kBlock / 64][(kMaxA / 2) * DMAX];
  __shared__ uint64_t s_h[kBlock / 64][kMaxA / 2];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t r = xcd_block(ceil_div(a.total, kBlock)) * kBlock + threadIdx.x;
  const bool live = r < a.total;
  const int p = live ? a.pid[r] : -1;
  const int pu = __builtin_amdgcn_readfirstlane(p);
  const bool uni = pu >= 0 && __all(!live || p == pu);
  if (uni) {
    const int j1 = a.aoff[pu] + a.azero[pu] + 1, nh = a.aoff[pu + 1] - j1;
    if (!LAT)   // (lattice matches need no key)
      for (int i = lane; i < nh * a.d; i += 64) s_w[wv][i] = a.akeys[(int64_t)j1 * a.d + i];
    for (int i = lane; i < nh; i += 64) s_h[wv][i] = a.ahash[j1 + i];
  }
  __syncthreads();
  if (!live) return;
  constexpr int G = kNbrGroup;
  if (uni)
    nbr_row<DMAX, EVEN, true, G, E, LAT>(a, r, p, s_w[wv], s_h[wv]);
  else
    nbr_row<DMAX, EVEN, false, G, E, LAT>(a, r, p, nullptr, nullptr);
}

// one pass of min-label propagation over the neighbour relation (thread per canonical row); with
// COUNT the pass also writes every row's entry count; FIRST the pass reads the initial labels from
// `init` and writes every row's label (the later passes update `label` in place)
template <int K, bool COUNT, bool FIRST>
__global__ void k_cc_prop(NbrView<K> v, const int32_t* __restrict__ pid, const int64_t* __restrict__ rowoff,
                          const int64_t* init, int64_t* label, int32_t* changed, int64_t* __restrict__ rowlen) {
  const int64_t total = v.total;
  const int64_t r = xcd_block(ceil_div(total, kBlock)) * kBlock + threadIdx.x;
  if (r >= total) return;
  const int64_t* src = FIRST ? init : label;
  const int p = pid[r];
  const int64_t base = rowoff[p];
  const int64_t own = src[r];
  int64_t l = own;
  const int n = v.slots(p, r);
  int cnt = 0;
  for (int u0 = 0; u0 < n; u0 += kDenseChunk) {   // entries, then labels, a chunk at a time
    uint32_t c[kDenseChunk];
    bool ok[kDenseChunk];
    int64_t lc[kDenseChunk];
#pragma unroll
    for (int u = 0; u < kDenseChunk; ++u) {
      ok[u] = u0 + u < n && v.load(r, u0 + u, c[u]);
      c[u] &= kColMask;
      cnt += ok[u] ? 1 : 0;
    }
#pragma unroll
    for (int u = 0; u < kDenseChunk; ++u) lc[u] = ok[u] ? src[base + c[u]] : own;
#pragma unroll
    for (int u = 0; u < kDenseChunk; ++u) l = lc[u] < l ? lc[u] : l;
  }
  if (COUNT) rowlen[r] = cnt;
  if (FIRST || l < own) label[r] = l;
  if (l < own) *changed = 1;
}

__global__ void k_cc_jump(int64_t total, int64_t* label) {
  const int64_t r = xcd_tid();
  if (r >= total) return;
  label[r] = label[label[r]];
}

// one wavefront per class (a run [cq[k], cq[k+1]) of the sorted rows): the class id is the
// smallest canonical slot of the class, written to every member
__global__ void k_class_min(int64_t n_cls, int64_t total, const int64_t* __restrict__ cq,
                            const uint32_t* __restrict__ order, const int32_t* __restrict__ pid,
                            const int64_t* __restrict__ rowoff, int32_t* __restrict__ comp) {
  const int64_t k = xcd_tid() >> 6;
  const int lane = threadIdx.x & 63;
  if (k >= n_cls) return;
  const int64_t q0 = cq[k], q1 = k + 1 < n_cls ? cq[k + 1] : total;
  const int64_t base = rowoff[pid[order[q0]]];
  int64_t m = INT64_MAX;
  for (int64_t q = q0 + lane; q < q1; q += 64) {
    const int64_t r = order[q];
    m = r < m ? r : m;
  }
  for (int off = 32; off > 0; off >>= 1) {
    const int64_t o = __shfl_xor(m, off, 64);
    m = o < m ? o : m;
  }
  for (int64_t q = q0 + lane; q < q1; q += 64) comp[order[q]] = (int32_t)(m - base);
}

// sort key (problem, class, kMaxA - row length) packed with `lb` bits per local index (32-bit keys
// when the fields fit, which halves the key traffic of every sort pass); the rows come in
// canonical order and the radix sort is stable, so the canonical slot breaks ties
template <typename K>
__global__ void k_exec_keys(int64_t total, int lb, const int32_t* __restrict__ pid,
                            const int64_t* __restrict__ rowoff, const int64_t* __restrict__ label,
                            const int64_t* __restrict__ rowlen, K* __restrict__ key,
                            uint32_t* __restrict__ val) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= total) return;
  const int p = pid[r];
  const uint64_t cls = (uint64_t)(label[r] - rowoff[p]);
  key[r] = (K)(((((uint64_t)p << lb) | cls) << kJBits) | (uint64_t)(kMaxA - rowlen[r]));
  val[r] = (uint32_t)r;
}

__global__ void k_fill_i64(int64_t n, int64_t* p, int64_t v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// sorted position q -> execution row: start of its class in the execution layout + offset in the class
__global__ void k_exec_map(int64_t total, const uint32_t* __restrict__ order, const uint32_t* __restrict__ cflag,
                           const uint32_t* __restrict__ cidx, const int64_t* __restrict__ cq0,
                           const int64_t* __restrict__ ce0, int64_t* __restrict__ canon2exec,
                           int64_t* __restrict__ exec2canon) {
  const int64_t q = xcd_tid();
  if (q >= total) return;
  const int64_t r = order[q];
  const int64_t k = (int64_t)cidx[q] + cflag[q] - 1;
  const int64_t e = ce0[k] + (q - cq0[k]);
  canon2exec[r] = e;
  exec2canon[e] = r;
}

// width (in entries) of each 64-row slice: one wavefront per slice, one lane per row
__global__ void k_slice_width(int64_t n_slices, const int64_t* __restrict__ exec2canon,
                              const int64_t* __restrict__ rowlen, uint32_t* __restrict__ width) {
  const int64_t g = xcd_tid();
  const int64_t sl = g >> 6;
  if (sl >= n_slices) return;
  const int64_t r = exec2canon[g];
  int w = r >= 0 ? (int)rowlen[r] : 0;
  for (int off = 32; off > 0; off >>= 1) {
    const int o = __shfl_xor(w, off, 64);
    w = o > w ? o : w;
  }
  if ((g & 63) == 0) width[sl] = (uint32_t)(w * kSlice);
  if (g == 0) width[n_slices] = 0;   // the scan's last element: the total
}

// 1 where a position of `order` (sorted rows) starts a new class: first row of a problem,
// or a class change; flag[n] = 0 (the scan's last element: the class count)
__global__ void k_class_start_flags(int64_t n, const uint32_t* __restrict__ order, const int64_t* __restrict__ label,
                                    const int32_t* __restrict__ pid, uint32_t* __restrict__ flag) {
  const int64_t q = xcd_tid();
  if (q >= n) return;
  const int64_t r = order[q];
  uint32_t f = 1;
  if (q > 0) {
    const int64_t rp = order[q - 1];
    f = (pid[rp] != pid[r] || label[rp] != label[r]) ? 1u : 0u;
  }
  flag[q] = f;
  if (q == 0) flag[n] = 0;
}

__global__ void k_compact_starts(int64_t n, const uint32_t* __restrict__ flag, const uint32_t* __restrict__ idx,
                                 int64_t* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n && flag[e]) out[idx[e]] = e;
}

// SELL-64 entries from the neighbour table, a thread per canonical row (its slots read coalesced
// with the neighbouring rows'): the row's entries go, in j order, to its execution row
// e = canon2exec[r] (lane e % 64 of slice e / 64, entry q at sptr + q * 64 + lane) with their
// columns mapped to local execution rows, and null entries pad it to the slice width.  Threads
// t < n_exec also pad the execution rows that hold no canonical row.
template <int K, typename NormT>
__global__ void k_sell_fill(NbrView<K> v, int64_t n_exec, const int64_t* __restrict__ exec2canon,
                            const int64_t* __restrict__ canon2exec, const int32_t* __restrict__ pid,
                            const int64_t* __restrict__ rowoff, const int64_t* __restrict__ eoff,
                            const int64_t* __restrict__ norm, const uint32_t* __restrict__ sptr,
                            uint32_t* __restrict__ sent, NormT* __restrict__ norm_exec, int64_t n_threads) {
  const int64_t t = xcd_block(ceil_div(n_threads, kBlock)) * kBlock + threadIdx.x;
  if (t >= n_threads) return;
  const uint32_t null_ent = (uint32_t)kNullJ << kColBits;
  if (t < n_exec && exec2canon[t] < 0) {   // a padding row
    const int64_t sl = t / kSlice;
    const int lane = (int)(t % kSlice);
    const uint32_t base = sptr[sl], w = (sptr[sl + 1] - base) / kSlice;
    for (uint32_t q = 0; q < w; ++q) sent[base + q * kSlice + lane] = null_ent;
    norm_exec[t] = 0;
  }
  const int64_t r = t;
  if (r >= v.total) return;
  const int p = pid[r];
  const int64_t e = canon2exec[r];
  const int64_t sl = e / kSlice;
  const int lane = (int)(e % kSlice);
  const uint32_t base = sptr[sl], w = (sptr[sl + 1] - base) / kSlice;
  const int64_t ro = rowoff[p], eo = eoff[p];
  const int n = v.slots(p, r);
  uint32_t q = 0;
  for (int u0 = 0; u0 < n; u0 += kDenseChunk) {
    uint32_t ent[kDenseChunk];
    bool ok[kDenseChunk];
    int64_t col[kDenseChunk];
#pragma unroll
    for (int u = 0; u < kDenseChunk; ++u) ok[u] = u0 + u < n && v.load(r, u0 + u, ent[u]);
#pragma unroll
    for (int u = 0; u < kDenseChunk; ++u) col[u] = ok[u] ? canon2exec[ro + (ent[u] & kColMask)] - eo : 0;
#pragma unroll
    for (int u = 0; u < kDenseChunk; ++u)
      if (ok[u]) sent[base + (q++) * kSlice + lane] = (uint32_t)col[u] | (ent[u] & ~kColMask);
  }
  for (; q < w; ++q) sent[base + q * kSlice + lane] = null_ent;
  norm_exec[e] = (NormT)norm[r];
}

}  // namespace

OpDev OpImpl::dev() const {
  OpDev o;
  o.sent = d_sent;
  o.sptr = d_sptr;
  o.norm = d_norm;
  o.eoff = d_eoff;
  o.work = d_work;
  o.wrange = d_wrange;
  o.A64 = d_A64;
  o.A32 = d_A32;
  o.nu = d_nu;
  o.a0 = d_a0;
  o.n_work = (int32_t)work.size();
  o.n_prob = n_prob;
  return o;
}

ss_status build_op_impl(const StampImpl* st, const int32_t* n_a, const int16_t* a_freqs,
                        const double* a_hat, uint32_t flags, hipStream_t stream, OpImpl** out) {
  *out = nullptr;
  if (!st || !n_a || !a_freqs || !a_hat) return fail(SS_EINVAL, "null argument");
  const int32_t n_prob = st->n_prob, d = st->d;
  OpImpl* op = new OpImpl();
  std::unique_ptr<OpImpl, void (*)(OpImpl*)> guard(op, free_op_impl);
  op->n_prob = n_prob;
  op->d = d;
  op->total = st->total;
  op->row_off = st->row_off;
  op->wide_norm = st->max_norm >= (int64_t(1) << 30);

  // ---- coefficient tables (host), matched to the stamp's a-tables
  const double two_pi2 = 2.0 * M_PI * M_PI;
  // host staging reused across builds of a thread (fresh pages would be faulted in every time)
  thread_local std::vector<double2> A64;
  thread_local std::vector<float2> A32;
  thread_local std::vector<int64_t> nu;
  A64.assign((size_t)n_prob * kTab, make_double2(0, 0));
  A32.assign((size_t)n_prob * kTab, make_float2(0, 0));
  nu.assign((size_t)n_prob * kTab, 0);
  std::vector<double> a0(n_prob);
  int smax = 1;
  int64_t pos = 0;
  ATable at;   // reused across problems
  for (int p = 0; p < n_prob; ++p) {
    SS_TRY(canonical_a(d, n_a[p], a_freqs + pos * d, a_hat + 2 * pos, false, &at));
    pos += n_a[p];
    const int s = st->a_off[p + 1] - st->a_off[p];
    const bool same = at.size() == s && std::equal(at.keys.begin(), at.keys.end(),
                                                   st->a_keys.begin() + (int64_t)st->a_off[p] * d);
    if (!same) return fail(SS_EINVAL, "supp(a) differs from the one the stamping set was built with");
    smax = std::max(smax, s);
    double l1 = 0;
    for (int j = 0; j < s; ++j) {
      const double2 c = at.coef[j];
      A64[(size_t)p * kTab + j] = make_double2(two_pi2 * c.x, two_pi2 * c.y);
      A32[(size_t)p * kTab + j] = make_float2((float)(two_pi2 * c.x), (float)(two_pi2 * c.y));
      int64_t nn = 0;
      for (int t = 0; t < d; ++t) nn += (int64_t)at.key(j)[t] * at.key(j)[t];
      nu[(size_t)p * kTab + j] = nn;
      if (j != at.zero) l1 += cabs2d(c.x, c.y);
    }
    a0[p] = at.coef[at.zero].x;
    op->a0_host.push_back(a0[p]);
    if (!(flags & SS_SKIP_L1_CHECK) && !(l1 < a0[p]))
      return fail(SS_ENOTPD, "l1 positivity certificate failed: a_0 <= sum |a_w| (pass SS_SKIP_L1_CHECK "
                             "if a is known to be positive)");
  }

  const int64_t total = st->total;
  SS_HIP(hipGetDevice(&op->device));
  struct Tmp {
    hipStream_t s;
    std::vector<void*> p;
    ~Tmp() {
      (void)hipStreamSynchronize(s);   // queued work may still use the blocks (error paths)
      for (void* q : p)
        if (q) pool_free(q);
    }
  } tmpmem{stream, {}};
  auto track = [&](void* q) { tmpmem.p.push_back(q); };

  // ---- neighbour map: for d <= 64, half the lookups into a dense j-major table (the other
  // half mirrored); above, one lane per (row, j) with rows compacted in j order
  int64_t max_rows = 1;
  for (int p = 0; p < n_prob; ++p) max_rows = std::max(max_rows, st->row_off[p + 1] - st->row_off[p]);
  const bool narrow = max_rows < 65535;   // 16-bit dense entries (0xffff = absent)
  // the mirrored half needs w_{s-1-j} = -w_j with w_z = 0 at z = (s-1)/2 in every a-table
  // lattice matches read no key, so the row-per-lane kernel then serves any d
  const bool lat = (flags & SS_EXACT_LOOKUP) == 0;
  bool dense = d <= 64 || lat;
  for (int p = 0; dense && p < n_prob; ++p) {
    const int s = st->a_off[p + 1] - st->a_off[p];
    const int16_t* ak = st->a_keys.data() + (int64_t)st->a_off[p] * d;
    dense = st->a_zero[p] * 2 == s - 1;
    for (int j = 0; dense && j < s; ++j)
      for (int t = 0; t < d; ++t) dense &= ak[(int64_t)j * d + t] == -ak[(int64_t)(s - 1 - j) * d + t];
  }
  uint32_t* nbr = nullptr;
  int64_t* rowlen = nullptr;
  SS_TRY(dalloc(&nbr, dense && narrow ? ceil_div((int64_t)total * smax, 2) : (int64_t)total * smax));
  track(nbr);
  SS_TRY(dalloc(&rowlen, total + 1));
  track(rowlen);
  const int rpw = smax <= 64 ? 64 / smax : 1;
  NbrArgs na{total, d, smax, rpw, st->d_keys, st->d_hash, st->d_pid, st->d_rowoff, st->d_akeys, st->d_ahash,
             st->d_aoff, st->d_azero, st->d_toff, st->d_tmask, st->d_ltable, nbr, rowlen, st->d_lat, st->d_alat};
  if (dense) {
    int zmax = 0;
    for (int p = 0; p < n_prob; ++p) zmax = std::max(zmax, st->a_zero[p]);
    SS_HIP(hipMemsetAsync(nbr, 0xff, (size_t)zmax * total * (narrow ? 2 : 4), stream));   // the mirrored half
    const unsigned g = xcd_grid(ceil_div(total, kBlock));
    const bool even = d % 2 == 0;
    auto launch = [&](auto entry) {
      using E = decltype(entry);
      if (lat)
        k_neighbors_row<8, true, E, true><<<g, kBlock, 0, stream>>>(na);   // no key is read: any d
      else if (d <= 8)
        even ? k_neighbors_row<8, true, E, false><<<g, kBlock, 0, stream>>>(na) : k_neighbors_row<8, false, E, false><<<g, kBlock, 0, stream>>>(na);
      else if (d <= 16)
        even ? k_neighbors_row<16, true, E, false><<<g, kBlock, 0, stream>>>(na) : k_neighbors_row<16, false, E, false><<<g, kBlock, 0, stream>>>(na);
      else if (d <= 32)
        even ? k_neighbors_row<32, true, E, false><<<g, kBlock, 0, stream>>>(na) : k_neighbors_row<32, false, E, false><<<g, kBlock, 0, stream>>>(na);
      else
        even ? k_neighbors_row<64, true, E, false><<<g, kBlock, 0, stream>>>(na) : k_neighbors_row<64, false, E, false><<<g, kBlock, 0, stream>>>(na);
    };
    if (narrow) launch(uint16_t{});
    else launch(uint32_t{});
  } else {
    if (lat)
      k_neighbors<true><<<xcd_grid(ceil_div(ceil_div(total, rpw), kBlock / 64)), kBlock, 0, stream>>>(na);
    else
      k_neighbors<false><<<xcd_grid(ceil_div(ceil_div(total, rpw), kBlock / 64)), kBlock, 0, stream>>>(na);
  }
  const int kind = dense ? (narrow ? kDense16 : kDense32) : kCompact;
  // the neighbour table in the view of `kind`, passed to f
  auto with_view = [&](auto f) {
    if (kind == kDense16) f(NbrView<kDense16>{nbr, total, st->d_aoff, rowlen});
    else if (kind == kDense32) f(NbrView<kDense32>{nbr, total, st->d_aoff, rowlen});
    else f(NbrView<kCompact>{nbr, total, st->d_aoff, rowlen});
  };

  // ---- connected classes: labels start at each key's root forcing key (so classes that no
  // coincidence merged are final at once); min-propagation with pointer jumping settles merges.
  // The class id (smallest canonical slot of the class) is taken after the execution sort,
  // which makes every class a contiguous run
  int64_t* label = nullptr;
  int32_t* changed = nullptr;
  SS_TRY(dalloc(&label, total));
  track(label);
  SS_TRY(dalloc(&changed, 1));
  track(changed);
  for (int it = 0; it < 100000; ++it) {
    int32_t h = 0;
    SS_HIP(hipMemsetAsync(changed, 0, 4, stream));
    with_view([&](auto v) {
      constexpr int K = decltype(v)::kKind;
      const unsigned g = xcd_grid(ceil_div(total, kBlock));
      // the first pass starts from the roots and also counts the entries of every row
      if (K != kCompact && it == 0)
        k_cc_prop<K, true, true><<<g, kBlock, 0, stream>>>(v, st->d_pid, st->d_rowoff, st->d_root, label, changed, rowlen);
      else if (it == 0)
        k_cc_prop<K, false, true><<<g, kBlock, 0, stream>>>(v, st->d_pid, st->d_rowoff, st->d_root, label, changed, rowlen);
      else
        k_cc_prop<K, false, false><<<g, kBlock, 0, stream>>>(v, st->d_pid, st->d_rowoff, nullptr, label, changed, rowlen);
    });
    k_cc_jump<<<xcd_grid(ceil_div(total, kBlock)), kBlock, 0, stream>>>(total, label);
    Readback rb(stream);
    SS_TRY(rb.add(&h, changed, 4));
    SS_TRY(rb.sync());
    if (!h) break;
  }
  // entries per problem (read back with the slice offsets below)
  int64_t* d_nnzp = nullptr;
  SS_TRY(dalloc(&d_nnzp, n_prob));
  track(d_nnzp);
  k_problem_nnz<<<n_prob, kBlock, 0, stream>>>(st->d_rowoff, rowlen, d_nnzp);

  // ---- execution order: (problem, class, -row length, canonical slot); a class whose
  // padding to a slice boundary costs at most 1/8 of its rows is padded, so the slices of
  // large classes never straddle two classes (their matvec windows stay one class wide)
  uint64_t *ek = nullptr, *ek2 = nullptr;
  uint32_t *ev = nullptr, *ev2 = nullptr;
  SS_TRY(dalloc(&ek, total));
  track(ek);
  SS_TRY(dalloc(&ek2, total));
  track(ek2);
  SS_TRY(dalloc(&ev, total));
  track(ev);
  SS_TRY(dalloc(&ev2, total));
  track(ev2);
  int lb = 1;
  while ((int64_t(1) << lb) < max_rows) ++lb;
  int pb = 0;
  while ((1 << pb) < n_prob) ++pb;
  const int key_bits = pb + lb + kJBits;   // <= 14 + 22 + 7
  auto exec_sort = [&](auto* k1, auto* k2) -> ss_status {
    k_exec_keys<<<grid_for(total), kBlock, 0, stream>>>(total, lb, st->d_pid, st->d_rowoff, label, rowlen, k1, ev);
    size_t tb = 0;
    SS_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, tb, k1, k2, ev, ev2, total, 0, key_bits, stream));
    void* t = nullptr;
    SS_HIP(pool_alloc((void**)&t, tb));
    track(t);
    SS_HIP(hipcub::DeviceRadixSort::SortPairs(t, tb, k1, k2, ev, ev2, total, 0, key_bits, stream));
    return SS_OK;
  };
  if (key_bits <= 32) SS_TRY(exec_sort(reinterpret_cast<uint32_t*>(ek), reinterpret_cast<uint32_t*>(ek2)));
  else SS_TRY(exec_sort(ek, ek2));
  // class starts in sorted order
  uint32_t *cflag = nullptr, *cidx = nullptr;
  SS_TRY(dalloc(&cflag, total + 1));
  track(cflag);
  SS_TRY(dalloc(&cidx, total + 1));
  track(cidx);
  k_class_start_flags<<<xcd_grid(ceil_div(total, kBlock)), kBlock, 0, stream>>>(total, ev2, label, st->d_pid, cflag);
  std::vector<int64_t> cq;   // sorted position of every class start
  {
    size_t tb = 0;
    SS_HIP(hipcub::DeviceScan::ExclusiveSum(nullptr, tb, cflag, cidx, total + 1, stream));
    void* t = nullptr;
    SS_HIP(pool_alloc((void**)&t, tb));
    track(t);
    SS_HIP(hipcub::DeviceScan::ExclusiveSum(t, tb, cflag, cidx, total + 1, stream));
    uint32_t n_cls = 0;
    Readback rb(stream);
    SS_TRY(rb.add(&n_cls, cidx + total, 4));
    SS_TRY(rb.sync());
    int64_t* d_cq = nullptr;
    SS_TRY(dalloc(&d_cq, std::max<uint32_t>(n_cls, 1)));
    track(d_cq);
    k_compact_starts<<<grid_for(total), kBlock, 0, stream>>>(total, cflag, cidx, d_cq);
    SS_TRY(dalloc(&op->d_comp, total));
    if (n_cls)
      k_class_min<<<xcd_grid(ceil_div((int64_t)n_cls * 64, kBlock)), kBlock, 0, stream>>>(
          n_cls, total, d_cq, ev2, st->d_pid, st->d_rowoff, op->d_comp);
    cq.resize(n_cls);
    SS_TRY(rb.add(cq.data(), d_cq, n_cls * 8));
    SS_TRY(rb.sync());
  }
  op->comps.assign(n_prob, 0);
  for (int64_t q : cq) {
    const int p = (int)(std::upper_bound(st->row_off.begin(), st->row_off.end(), q) - st->row_off.begin()) - 1;
    op->comps[p] += 1;
  }
  op->n_components = (int64_t)cq.size();
  // exec layout of every class (host), per problem
  const int64_t n_cls = (int64_t)cq.size();
  std::vector<int64_t> ce0(n_cls);                       // global exec row of each class start
  std::vector<std::vector<int64_t>> cbounds(n_prob);     // local class starts + problem end
  op->eoff.assign(n_prob + 1, 0);
  op->cls_e0.clear();
  op->cls_n.clear();
  {
    size_t k = 0;
    for (int p = 0; p < n_prob; ++p) {
      const int64_t q1 = st->row_off[p + 1];
      int64_t cur = 0;
      while (k < cq.size() && cq[k] < q1) {
        const int64_t size = (k + 1 < cq.size() ? std::min(cq[k + 1], q1) : q1) - cq[k];
        const int64_t pad = (kSlice - size % kSlice) % kSlice;
        ce0[k] = op->eoff[p] + cur;
        op->cls_e0.push_back(ce0[k]);
        op->cls_n.push_back(size);
        cbounds[p].push_back(cur);
        cur += size + (pad * 8 <= size ? pad : 0);
        ++k;
      }
      const int64_t rows = ceil_div(cur, kSlice) * kSlice;
      cbounds[p].push_back(rows);
      op->eoff[p + 1] = op->eoff[p] + rows;
    }
  }
  op->n_exec = op->eoff[n_prob];
  op->n_slices = op->n_exec / kSlice;
  if (op->n_slices * (int64_t)kMaxA * kSlice >= (int64_t(1) << 32))
    return fail(SS_ERANGE, "batch too large for 32-bit SELL offsets (split it)");
  // problem offsets (kept) and the class starts of the execution map, one transfer
  int64_t *d_cq0 = nullptr, *d_ce0 = nullptr;
  {
    Upload up;
    up.add(&op->d_eoff, op->eoff.data(), n_prob + 1);
    up.add(&d_cq0, cq.data(), n_cls);
    up.add(&d_ce0, ce0.data(), n_cls);
    SS_TRY(up.commit(&op->d_upload[0], stream));
  }
  SS_TRY(dalloc(&op->d_exec2canon, op->n_exec));
  SS_TRY(dalloc(&op->d_canon2exec, total));
  k_fill_i64<<<grid_for(op->n_exec), kBlock, 0, stream>>>(op->n_exec, op->d_exec2canon, -1);
  k_exec_map<<<xcd_grid(ceil_div(total, kBlock)), kBlock, 0, stream>>>(total, ev2, cflag, cidx, d_cq0, d_ce0, op->d_canon2exec,
                                                      op->d_exec2canon);

  // ---- SELL-64 slices
  uint32_t* width = nullptr;
  SS_TRY(dalloc(&width, op->n_slices + 1));
  track(width);
  SS_TRY(dalloc(&op->d_sptr, op->n_slices + 1));
  k_slice_width<<<xcd_grid(ceil_div(op->n_slices * kSlice, kBlock)), kBlock, 0, stream>>>(op->n_slices, op->d_exec2canon, rowlen,
                                                                        width);
  {
    size_t tb = 0;
    SS_HIP(hipcub::DeviceScan::ExclusiveSum(nullptr, tb, width, op->d_sptr, op->n_slices + 1, stream));
    void* t = nullptr;
    SS_HIP(pool_alloc((void**)&t, tb));
    track(t);
    SS_HIP(hipcub::DeviceScan::ExclusiveSum(t, tb, width, op->d_sptr, op->n_slices + 1, stream));
  }
  thread_local std::vector<uint32_t> sptr_h;   // slice entry offsets, for sizing solve units
  sptr_h.resize(op->n_slices + 1);
  op->nnz_p.resize(n_prob);
  {
    Readback rb(stream);
    SS_TRY(rb.add(sptr_h.data(), op->d_sptr, (op->n_slices + 1) * 4));
    SS_TRY(rb.add(op->nnz_p.data(), d_nnzp, n_prob * 8));
    SS_TRY(rb.sync());
  }
  op->nnz = 0;
  for (int p = 0; p < n_prob; ++p) op->nnz += op->nnz_p[p];
  const uint32_t n_sell = sptr_h[op->n_slices];
  op->n_sell = n_sell;
  int64_t ncomp_total = 0;
  for (int p = 0; p < n_prob; ++p) ncomp_total += op->comps[p];
  op->n_components = ncomp_total;
  SS_TRY(dalloc(&op->d_sent, std::max<int64_t>(n_sell, 1)));
  const int64_t n_fill = std::max(total, op->n_exec);   // canonical rows, and padding execution rows
  if (op->wide_norm) {
    int64_t* ne = nullptr;
    SS_TRY(dalloc(&ne, op->n_exec));
    op->d_norm = ne;
    with_view([&](auto v) {
      k_sell_fill<<<xcd_grid(ceil_div(n_fill, kBlock)), kBlock, 0, stream>>>(
          v, op->n_exec, op->d_exec2canon, op->d_canon2exec, st->d_pid, st->d_rowoff, op->d_eoff, st->d_norm,
          op->d_sptr, op->d_sent, ne, n_fill);
    });
  } else {
    int32_t* ne = nullptr;
    SS_TRY(dalloc(&ne, op->n_exec));
    op->d_norm = ne;
    with_view([&](auto v) {
      k_sell_fill<<<xcd_grid(ceil_div(n_fill, kBlock)), kBlock, 0, stream>>>(
          v, op->n_exec, op->d_exec2canon, op->d_canon2exec, st->d_pid, st->d_rowoff, op->d_eoff, st->d_norm,
          op->d_sptr, op->d_sent, ne, n_fill);
    });
  }

  // ---- work items: runs of slices of one problem whose rows' classes fit an LDS window
  // (the matvec stages x and |k|^2 of the window once per block); a class larger than the
  // window gets items of four slices that gather from global memory
  op->wrange.resize(n_prob);
  op->max_window = 0;
  for (int p = 0; p < n_prob; ++p) {
    const int64_t e0 = op->eoff[p], e1 = op->eoff[p + 1];
    // class boundaries of this problem, local rows (a class owns the padding rows after it)
    const std::vector<int64_t>& cb = cbounds[p];
    auto class_of = [&](int64_t row) {   // index k with cb[k] <= row < cb[k+1]
      return (int64_t)(std::upper_bound(cb.begin(), cb.end(), row) - cb.begin()) - 1;
    };
    const int ns = (int)((e1 - e0) / kSlice);
    op->wrange[p].x = (int)op->work.size();
    int sl = 0;
    while (sl < ns) {
      const int64_t w0 = cb[class_of((int64_t)sl * kSlice)];
      int64_t w1 = cb[class_of((int64_t)(sl + 1) * kSlice - 1) + 1];
      if (w1 - w0 > kWinRows) {   // too large for LDS: global gathers
        const int n = std::min(kSolveWaves, ns - sl);
        op->work.push_back(make_int4(p, (int)(e0 / kSlice) + sl, n, 0));
        sl += n;
        continue;
      }
      int n = 1;
      while (sl + n < ns && n < kMaxItemSlices) {
        const int64_t nw1 = cb[class_of((int64_t)(sl + n + 1) * kSlice - 1) + 1];
        if (nw1 - w0 > kWinRows) break;
        w1 = nw1;
        ++n;
      }
      op->work.push_back(make_int4(p, (int)(e0 / kSlice) + sl, n | (int)((w1 - w0) << 16), (int)w0));
      op->max_window = std::max<int64_t>(op->max_window, w1 - w0);
      sl += n;
    }
    op->wrange[p].y = (int)op->work.size();
  }
  // ---- solve units: greedy runs ending on the furthest class boundary that is also a slice
  // boundary within kWinRows rows, preferring runs whose entries fit the LDS entry cache
  op->urange.assign(n_prob, make_int2(-1, -1));
  for (int p = 0; p < n_prob; ++p) {
    const std::vector<int64_t>& cb = cbounds[p];
    const int64_t rows = cb.back();
    const int64_t sl0 = op->eoff[p] / kSlice;
    const size_t u0 = op->units.size();
    int64_t start = 0;
    bool ok = true;
    while (start < rows) {
      auto entries = [&](int64_t end) {
        return (int64_t)sptr_h[sl0 + end / kSlice] - (int64_t)sptr_h[sl0 + start / kSlice];
      };
      // candidates: boundaries in (start, start + kWinRows], scanned from the far end
      auto it = std::upper_bound(cb.begin(), cb.end(), start + kWinRows);
      int64_t cut = -1, cut_cached = -1;
      while (it != cb.begin()) {
        --it;
        if (*it <= start) break;
        if (*it % kSlice != 0) continue;
        if (cut < 0) cut = *it;
        if (entries(*it) <= kUnitEntries) {
          cut_cached = *it;
          break;
        }
      }
      if (cut_cached >= 0) cut = cut_cached;
      if (cut < 0) {
        ok = false;
        break;
      }
      op->units.push_back(make_int4(p, (int)(sl0 + start / kSlice), (int)((cut - start) / kSlice), (int)start));
      start = cut;
    }
    if (ok && op->units.size() > u0) {
      op->urange[p] = make_int2((int)u0, (int)op->units.size());
    } else {
      op->units.resize(u0);
    }
  }
  op->unit_entries.resize(op->units.size());
  op->unit_ebase.resize(op->units.size());
  for (size_t i = 0; i < op->units.size(); ++i) {
    const int4 un = op->units[i];
    op->unit_entries[i] = (int32_t)(sptr_h[un.y + un.z] - sptr_h[un.y]);
    op->unit_ebase[i] = sptr_h[un.y];
  }
  {   // the operator's launch tables and coefficient tables, one transfer
    Upload up;
    if (!op->units.empty()) up.add(&op->d_units, op->units.data(), op->units.size());
    up.add(&op->d_work, op->work.data(), op->work.size());
    up.add(&op->d_wrange, op->wrange.data(), n_prob);
    up.add(&op->d_A64, A64.data(), A64.size());
    up.add(&op->d_A32, A32.data(), A32.size());
    up.add(&op->d_nu, nu.data(), nu.size());
    up.add(&op->d_a0, a0.data(), n_prob);
    SS_TRY(up.commit(&op->d_upload[1], stream));
  }
  SS_HIP(hipStreamSynchronize(stream));
  *out = guard.release();
  return SS_OK;
}

void free_op_impl(OpImpl* op) {
  if (!op) return;
  dfree(op->d_comp);
  dfree(op->d_exec2canon);
  dfree(op->d_canon2exec);
  dfree(op->d_sent);
  dfree(op->d_sptr);
  if (op->d_norm) pool_free(op->d_norm);
  op->d_norm = nullptr;
  dfree(op->d_upload[0]);   // d_eoff is a view into it
  dfree(op->d_upload[1]);   // d_units, d_work, d_wrange, d_A64, d_A32, d_nu and d_a0 are views into it
  if (op->ws.base) pool_free(op->ws.base);
  if (op->h_pinned) (void)hipHostFree(op->h_pinned);
  free_apply_cache(op);
  delete op;
}

}  // namespace ss
