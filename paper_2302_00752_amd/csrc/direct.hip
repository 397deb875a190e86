// Dense direct solve of the truncated Galerkin system, one connected class at a time: the
// paper's own solver (Alg. 1, steps 4-5: assemble L_N densely, solve directly), restricted to
// the independent blocks the classes of Sec. 6 split it into.
//
// Each class block is Hermitian positive definite on the nonzero frequencies (the operator is
// Hermitian, and coercive by Prop. ExistenceUniquenessStability); the zero frequency has an
// all-zero row and column, and is given the identity instead (u_0 = 0).  The block is factored
// by a tiled left-looking Cholesky, L L^H, in FP64:
//   for every tile column j:  A_ij -= sum_{s<j} L_is L_js^H   (i >= j; FP64 MFMA, split over s)
//                             L_jj = chol(A_jj);  L_ij = A_ij L_jj^{-H}   (i > j)
// then L y = f and L^H u = y by tile substitution.  Storage: per class the lower triangle of
// 32 x 32 complex tiles, each tile column-major and contiguous (16 KB), row-major over tiles:
// tile (i, j), j <= i, is number i (i + 1) / 2 + j.  The factored diagonal tiles go to a
// separate array, so a step that factors A_jj never writes a tile other blocks still read.
#include <hipcub/hipcub.hpp>

#include <cmath>

#include "ss_internal.h"

namespace ss {

namespace {

constexpr int kT = 32;                        // tile rows and columns (complex entries)
constexpr int kTE = kT * kT;                  // entries per tile
constexpr int kLdT = kT + 1;                  // LDS row stride of a staged tile
constexpr int kDnBlock = 256;
constexpr int kDnWaves = kDnBlock / 64;
constexpr int64_t kDirectMaxRows = 8192;      // the substitution keeps one class vector in LDS
constexpr int64_t kDirectBudget = int64_t(6) << 30;   // factor storage per chunk of classes

typedef double d4_t __attribute__((ext_vector_type(4)));

struct DClass {
  int64_t e0;      // first global execution row
  int64_t eb;      // first execution row of the class's problem (SELL columns are problem-local)
  int64_t tbase;   // first lower tile in the chunk's tile array
  int64_t dbase;   // first factored diagonal tile
  int32_t n;       // rows
  int32_t nt;      // tile rows (n rounded up to kT, over kT)
  int32_t prob;
  int32_t pad;
};

__host__ __device__ inline int64_t tri(int64_t i) { return i * (i + 1) / 2; }

// block index -> (class, tile row).  With at least 8 classes every class keeps all of its blocks
// on one XCD (block b runs on XCD b mod 8), so the L tiles a step rereads stay in that L2.
__device__ inline bool dn_map(int nc, int per, bool xcd, int& c, int& t) {
  const int64_t b = blockIdx.x;
  if (xcd) {
    const int64_t k = b >> 3;
    c = (int)((b & 7) + 8 * (k / per));
    t = (int)(k % per);
  } else {
    c = (int)(b / per);
    t = (int)(b % per);
  }
  return c < nc;
}

// ---- assembly: row i of a class writes its entries (i, l) with l <= i; padding rows of the last
// tile and the zero frequency get a unit diagonal.  Every entry is 4 pi^2 (k . l) a_{k-l},
// formed as (|k|^2 + |l|^2 - |k-l|^2) 2 pi^2 a_{k-l} in the integer type of the norms.
template <typename NormT>
__global__ __launch_bounds__(kDnBlock) void k_dn_assemble(int nc, const DClass* __restrict__ cls,
                                                           const uint32_t* __restrict__ sent,
                                                           const uint32_t* __restrict__ sptr,
                                                           const NormT* __restrict__ norm,
                                                           const double2* __restrict__ A64,
                                                           const int64_t* __restrict__ nu, double2* __restrict__ W,
                                                           int* __restrict__ err) {
  const int c = blockIdx.y;
  if (c >= nc) return;
  const DClass C = cls[c];
  const int i = blockIdx.x * kDnBlock + threadIdx.x;
  if (i >= C.nt * kT) return;
  double2* tiles = W + C.tbase * kTE;
  const int64_t ti = i / kT;
  double2* diag = tiles + (tri(ti) + ti) * kTE + (i % kT) * kT + (i % kT);
  if (i >= C.n) {
    *diag = make_double2(1.0, 0.0);
    return;
  }
  const int64_t e = C.e0 + i;
  const NormT nk = norm[e];
  if (nk == 0) {
    *diag = make_double2(1.0, 0.0);
    return;
  }
  const int64_t sl = e / kSlice;
  const int lane = (int)(e % kSlice);
  const uint32_t base = sptr[sl];
  const uint32_t width = (sptr[sl + 1] - base) / kSlice;
  const double2* At = A64 + (int64_t)C.prob * 64;
  const int64_t* nut = nu + (int64_t)C.prob * 64;
  for (uint32_t q = 0; q < width; ++q) {
    const uint32_t ent = sent[base + q * kSlice + lane];
    const uint32_t j = ent >> kColBits;
    if (j == (uint32_t)kNullJ) continue;
    const int64_t ge = C.eb + (int64_t)(ent & kColMask);
    const int64_t l = ge - C.e0;
    if (l < 0 || l >= C.n) {
      err[1] = 1;   // a column outside the class: the class layout is inconsistent
      continue;
    }
    if (l > i) continue;
    const NormT I = nk + norm[ge] - (NormT)nut[j];
    const double fi = (double)I;
    const double2 a = At[j];
    const int64_t tj = l / kT;
    tiles[(tri(ti) + tj) * kTE + (l % kT) * kT + (i % kT)] = make_double2(fi * a.x, fi * a.y);
  }
}

// ---- trailing products of tile column j: A_ij -= sum_{s<j} L_is L_js^H, i >= j.  Wave w takes
// s = w, w + 4, ...; each wave holds the whole 32 x 32 product as 2 x 2 quadrants of 16 x 16 FP64
// MFMA accumulators (real and imaginary part each), and the four partial products are summed in
// LDS in a fixed order.  MFMA 16x16x4 operands: lane = row + 16 k for A (16 x 4) and column + 16 k
// for B (4 x 16); the result holds (4 v + lane / 16, lane mod 16) in item v.
__global__ __launch_bounds__(kDnBlock) void k_dn_update(int nc, int per, int j, bool xcd,
                                                         const DClass* __restrict__ cls, double2* __restrict__ W) {
  int c, t;
  if (!dn_map(nc, per, xcd, c, t)) return;
  const DClass C = cls[c];
  const int i = j + t;
  if (j >= C.nt || i >= C.nt) return;
  double2* tiles = W + C.tbase * kTE;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int lr = lane & 15, lk = lane >> 4;
  d4_t acc_re[2][2], acc_im[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      acc_re[a][b] = d4_t{0, 0, 0, 0};
      acc_im[a][b] = d4_t{0, 0, 0, 0};
    }
  for (int s = wave; s < j; s += kDnWaves) {
    const double2* P = tiles + (tri(i) + s) * kTE;
    const double2* Q = tiles + (tri(j) + s) * kTE;
#pragma unroll 2
    for (int kc = 0; kc < kT / 4; ++kc) {
      const int col = 4 * kc + lk;
      double2 p[2], q[2];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        p[h] = P[col * kT + 16 * h + lr];
        q[h] = Q[col * kT + 16 * h + lr];
      }
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          // (P Q^H)_re = Pre Qre^T + Pim Qim^T,  (P Q^H)_im = Pim Qre^T - Pre Qim^T
          acc_re[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(p[a].x, q[b].x, acc_re[a][b], 0, 0, 0);
          acc_re[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(p[a].y, q[b].y, acc_re[a][b], 0, 0, 0);
          acc_im[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(p[a].y, q[b].x, acc_im[a][b], 0, 0, 0);
          acc_im[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(-p[a].x, q[b].y, acc_im[a][b], 0, 0, 0);
        }
    }
  }
  // partial products of waves 1..3 through LDS, summed by wave 0's layout owner in wave order
  __shared__ double2 red[kDnWaves - 1][kTE];
  if (wave > 0) {
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int r = 16 * a + 4 * v + lk, cc = 16 * b + lr;
          red[wave - 1][cc * kT + r] = make_double2(acc_re[a][b][v], acc_im[a][b][v]);
        }
  }
  __syncthreads();
  if (wave == 0) {
    double2* A = tiles + (tri(i) + j) * kTE;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int r = 16 * a + 4 * v + lk, cc = 16 * b + lr;
          double sr = acc_re[a][b][v], si = acc_im[a][b][v];
#pragma unroll
          for (int w = 0; w < kDnWaves - 1; ++w) {
            const double2 o = red[w][cc * kT + r];
            sr += o.x;
            si += o.y;
          }
          double2 x = A[cc * kT + r];
          x.x -= sr;
          x.y -= si;
          A[cc * kT + r] = x;
        }
  }
}

// In-LDS Cholesky of the lower triangle of a 32 x 32 tile (stride kLdT), as L D L^H with the
// unit-lower columns kept unscaled and divided by the pivot on the fly, then scaled to L = L1
// D^{1/2}.  One barrier per column.  A pivot that is not positive and finite sets *bad and is
// replaced by 1, so the factor stays finite.
__device__ void tile_chol(double2* sA, double* sd, int* bad) {
  const int tid = threadIdx.x;
  for (int c = 0; c < kT; ++c) {
    __syncthreads();
    double piv = sA[c * kLdT + c].x;
    if (!(piv > 0.0) || !(piv < INFINITY)) {
      if (tid == 0) *bad = 1;
      piv = 1.0;
      if (tid == 0) sA[c * kLdT + c] = make_double2(1.0, 0.0);
    }
    const double ip = 1.0 / piv;
    for (int idx = tid; idx < kTE; idx += kDnBlock) {
      const int r = idx & (kT - 1), q = idx >> 5;   // element (r, q), column q
      if (q > c && r >= q) {
        const double2 arc = sA[c * kLdT + r], aqc = sA[c * kLdT + q];
        // A_rq -= A_rc conj(A_qc) / piv
        const double tr = arc.x * aqc.x + arc.y * aqc.y, ti = arc.y * aqc.x - arc.x * aqc.y;
        double2 v = sA[q * kLdT + r];
        v.x -= tr * ip;
        v.y -= ti * ip;
        sA[q * kLdT + r] = v;
      }
    }
  }
  __syncthreads();
  if (tid < kT) sd[tid] = sA[tid * kLdT + tid].x;
  __syncthreads();
  for (int idx = tid; idx < kTE; idx += kDnBlock) {
    const int r = idx & (kT - 1), q = idx >> 5;
    if (r >= q) {
      const double d = sd[q];
      double2 v = sA[q * kLdT + r];
      if (r == q) {
        v = make_double2(sqrt(d), 0.0);
      } else {
        const double s = 1.0 / sqrt(d);
        v = make_double2(v.x * s, v.y * s);
      }
      sA[q * kLdT + r] = v;
    }
  }
  __syncthreads();
}

// ---- tile column j: factor the updated A_jj (every block, redundantly, in LDS); block i == j
// stores L_jj, block i > j solves L_ij L_jj^H = A_ij in place
__global__ __launch_bounds__(kDnBlock) void k_dn_panel(int nc, int per, int j, bool xcd,
                                                        const DClass* __restrict__ cls, double2* __restrict__ W,
                                                        double2* __restrict__ D, int* __restrict__ err) {
  int c, t;
  if (!dn_map(nc, per, xcd, c, t)) return;
  const DClass C = cls[c];
  const int i = j + t;
  if (j >= C.nt || i >= C.nt) return;
  double2* tiles = W + C.tbase * kTE;
  __shared__ double2 sL[kT * kLdT];
  __shared__ double2 sX[kT * kLdT];
  __shared__ double s_piv[kT];
  __shared__ int s_bad;
  const int tid = threadIdx.x;
  if (tid == 0) s_bad = 0;
  const double2* Ajj = tiles + (tri(j) + j) * kTE;
  for (int idx = tid; idx < kTE; idx += kDnBlock) {
    const int r = idx & (kT - 1), q = idx >> 5;
    sL[q * kLdT + r] = Ajj[idx];
  }
  tile_chol(sL, s_piv, &s_bad);
  if (i == j) {
    double2* Lj = D + (C.dbase + j) * kTE;
    for (int idx = tid; idx < kTE; idx += kDnBlock) {
      const int r = idx & (kT - 1), q = idx >> 5;
      Lj[idx] = r >= q ? sL[q * kLdT + r] : make_double2(0.0, 0.0);
    }
    if (tid == 0 && s_bad) err[0] = 1;
    return;
  }
  double2* Aij = tiles + (tri(i) + j) * kTE;
  for (int idx = tid; idx < kTE; idx += kDnBlock) {
    const int r = idx & (kT - 1), q = idx >> 5;
    sX[q * kLdT + r] = Aij[idx];
  }
  // X L^H = A, column by column: x_rc = a_rc / L_cc, then a_rq -= x_rc conj(L_qc) for q > c
  for (int cc = 0; cc < kT; ++cc) {
    __syncthreads();
    const double il = 1.0 / sL[cc * kLdT + cc].x;
    for (int idx = tid; idx < kTE; idx += kDnBlock) {
      const int r = idx & (kT - 1), q = idx >> 5;
      if (q > cc) {
        const double2 a = sX[cc * kLdT + r], l = sL[cc * kLdT + q];
        const double xr = a.x * il, xi = a.y * il;
        double2 v = sX[q * kLdT + r];
        v.x -= xr * l.x + xi * l.y;
        v.y -= xi * l.x - xr * l.y;
        sX[q * kLdT + r] = v;
      }
    }
  }
  __syncthreads();
  for (int idx = tid; idx < kTE; idx += kDnBlock) {
    const int r = idx & (kT - 1), q = idx >> 5;
    const double il = 1.0 / sL[q * kLdT + q].x;
    const double2 v = sX[q * kLdT + r];
    Aij[idx] = make_double2(v.x * il, v.y * il);
  }
}

// ---- L y = f, then L^H u = y, one block per class, the class vector in LDS.  The diagonal
// tile substitution runs on one wavefront (lane = tile row); the off-diagonal tile products are
// spread over the block.
template <typename NormT>
__global__ __launch_bounds__(kDnBlock) void k_dn_subst(int nc, const DClass* __restrict__ cls,
                                                        const NormT* __restrict__ norm,
                                                        const double2* __restrict__ W,
                                                        const double2* __restrict__ D,
                                                        const int64_t* __restrict__ exec2canon,
                                                        const double2* __restrict__ f, double2* __restrict__ u) {
  const int c = blockIdx.x;
  if (c >= nc) return;
  const DClass C = cls[c];
  extern __shared__ __align__(16) double2 s_dn[];
  double2* sT = s_dn;                 // staged diagonal factor, stride kLdT
  double2* v = s_dn + kT * kLdT;      // the class vector, nt * kT entries
  const double2* tiles = W + C.tbase * kTE;
  const int tid = threadIdx.x;
  const int np = C.nt * kT;
  for (int r = tid; r < np; r += kDnBlock) {
    double2 x = make_double2(0.0, 0.0);
    if (r < C.n) {
      const int64_t g = exec2canon[C.e0 + r];
      if (g >= 0 && norm[C.e0 + r] != 0) x = f[g];   // u_0 = 0 whatever f_0 holds
    }
    v[r] = x;
  }
  // forward: L y = f
  for (int s = 0; s < C.nt; ++s) {
    __syncthreads();
    const double2* Ls = D + (C.dbase + s) * kTE;
    for (int idx = tid; idx < kTE; idx += kDnBlock) sT[(idx >> 5) * kLdT + (idx & (kT - 1))] = Ls[idx];
    __syncthreads();
    if (tid < 64) {
      const int r = tid & (kT - 1);
      double2 b = v[s * kT + r];
      for (int cc = 0; cc < kT; ++cc) {
        const double bx = __shfl(b.x, cc, 64), by = __shfl(b.y, cc, 64);
        const double il = 1.0 / sT[cc * kLdT + cc].x;
        const double yx = bx * il, yy = by * il;
        if (r == cc) b = make_double2(yx, yy);
        else if (r > cc) {
          const double2 l = sT[cc * kLdT + r];
          b.x -= l.x * yx - l.y * yy;
          b.y -= l.x * yy + l.y * yx;
        }
      }
      if (tid < kT) v[s * kT + r] = b;
    }
    __syncthreads();
    for (int R = (s + 1) * kT + tid; R < np; R += kDnBlock) {
      const int ti = R / kT, r = R % kT;
      const double2* L = tiles + (tri(ti) + s) * kTE;
      double sx = 0, sy = 0;
#pragma unroll 8
      for (int cc = 0; cc < kT; ++cc) {
        const double2 l = L[cc * kT + r], y = v[s * kT + cc];
        sx += l.x * y.x - l.y * y.y;
        sy += l.x * y.y + l.y * y.x;
      }
      double2 x = v[R];
      x.x -= sx;
      x.y -= sy;
      v[R] = x;
    }
  }
  // backward: L^H u = y
  for (int s = C.nt - 1; s >= 0; --s) {
    __syncthreads();
    const double2* Ls = D + (C.dbase + s) * kTE;
    for (int idx = tid; idx < kTE; idx += kDnBlock) sT[(idx >> 5) * kLdT + (idx & (kT - 1))] = Ls[idx];
    __syncthreads();
    if (tid < 64) {
      const int r = tid & (kT - 1);
      double2 b = v[s * kT + r];
      for (int cc = kT - 1; cc >= 0; --cc) {
        const double bx = __shfl(b.x, cc, 64), by = __shfl(b.y, cc, 64);
        const double il = 1.0 / sT[cc * kLdT + cc].x;
        const double ux = bx * il, uy = by * il;
        if (r == cc) b = make_double2(ux, uy);
        else if (r < cc) {
          // (L^H)_{r,cc} = conj(L_{cc,r})
          const double2 l = sT[r * kLdT + cc];
          b.x -= l.x * ux + l.y * uy;
          b.y -= l.x * uy - l.y * ux;
        }
      }
      if (tid < kT) v[s * kT + r] = b;
    }
    __syncthreads();
    for (int R = tid; R < s * kT; R += kDnBlock) {
      const int ti = R / kT, r = R % kT;
      const double2* L = tiles + (tri(s) + ti) * kTE;   // tile (s, ti), its column r
      double sx = 0, sy = 0;
#pragma unroll 8
      for (int cc = 0; cc < kT; ++cc) {
        const double2 l = L[r * kT + cc], y = v[s * kT + cc];
        sx += l.x * y.x + l.y * y.y;
        sy += l.x * y.y - l.y * y.x;
      }
      double2 x = v[R];
      x.x -= sx;
      x.y -= sy;
      v[R] = x;
    }
  }
  __syncthreads();
  for (int r = tid; r < C.n; r += kDnBlock) {
    const int64_t g = exec2canon[C.e0 + r];
    if (g >= 0) u[g] = v[r];
  }
}

}  // namespace

ss_status direct_solve_impl(const OpImpl* op, const void* f_dev, void* u_dev, hipStream_t s,
                            DirectStats* stats) {
  if (!op || !f_dev || !u_dev) return fail(SS_EINVAL, "null argument");
  const int64_t n_cls = (int64_t)op->cls_n.size();
  int64_t max_n = 0;
  for (int64_t k = 0; k < n_cls; ++k) max_n = std::max(max_n, op->cls_n[k]);
  if (max_n > kDirectMaxRows)
    return fail(SS_ERANGE, "a class has more than 8192 rows: too large for the dense direct solve");
  // the problem of every class, from the execution offsets
  std::vector<int32_t> cprob(n_cls);
  for (int64_t k = 0; k < n_cls; ++k)
    cprob[k] = (int32_t)(std::upper_bound(op->eoff.begin(), op->eoff.end(), op->cls_e0[k]) - op->eoff.begin()) - 1;
  if (stats) *stats = DirectStats{};
  const OpDev od = op->dev();
  int k0 = 0;
  ss_status result = SS_OK;
  while (k0 < n_cls) {
    // a chunk of consecutive classes whose tiles fit the budget (at least one class)
    std::vector<DClass> ch;
    int64_t tiles = 0, dtiles = 0;
    int max_nt = 0;
    int64_t k = k0;
    for (; k < n_cls && (int64_t)ch.size() < 65535; ++k) {
      const int nt = (int)ceil_div(op->cls_n[k], kT);
      const int64_t need = (tri(nt) + nt) * kTE * (int64_t)sizeof(double2);
      if (!ch.empty() && (tiles + dtiles) * kTE * (int64_t)sizeof(double2) + need > kDirectBudget) break;
      DClass dc;
      dc.e0 = op->cls_e0[k];
      dc.eb = op->eoff[cprob[k]];
      dc.tbase = tiles;
      dc.dbase = dtiles;
      dc.n = (int32_t)op->cls_n[k];
      dc.nt = nt;
      dc.prob = cprob[k];
      dc.pad = 0;
      tiles += tri(nt);
      dtiles += nt;
      max_nt = std::max(max_nt, nt);
      ch.push_back(dc);
    }
    k0 = (int)k;
    const int nc = (int)ch.size();
    double2 *W = nullptr, *Dg = nullptr;
    DClass* dcls = nullptr;
    int* err = nullptr;
    SS_TRY(dalloc(&W, (size_t)std::max<int64_t>(tiles, 1) * kTE));
    SS_TRY(dalloc(&Dg, (size_t)std::max<int64_t>(dtiles, 1) * kTE));
    SS_TRY(dalloc((char**)&dcls, (size_t)nc * sizeof(DClass)));
    SS_TRY(dalloc(&err, 2));
    struct Release {
      hipStream_t s;
      void* p[4];
      ~Release() {
        (void)hipStreamSynchronize(s);
        for (void* b : p) pool_free(b);
      }
    } rel{s, {W, Dg, dcls, err}};
    SS_HIP(h2d(dcls, ch.data(), (size_t)nc * sizeof(DClass), s));
    SS_HIP(hipMemsetAsync(W, 0, (size_t)tiles * kTE * sizeof(double2), s));
    SS_HIP(hipMemsetAsync(err, 0, 2 * sizeof(int), s));
    const dim3 ag((unsigned)ceil_div((int64_t)max_nt * kT, kDnBlock), (unsigned)nc);
    if (op->wide_norm)
      k_dn_assemble<int64_t><<<ag, kDnBlock, 0, s>>>(nc, dcls, od.sent, od.sptr, (const int64_t*)od.norm, od.A64,
                                                      od.nu, W, err);
    else
      k_dn_assemble<int32_t><<<ag, kDnBlock, 0, s>>>(nc, dcls, od.sent, od.sptr, (const int32_t*)od.norm, od.A64,
                                                      od.nu, W, err);
    SS_HIP(hipGetLastError());
    const bool xcd = nc >= 8;
    hipEvent_t f0 = nullptr, f1 = nullptr;
    if (stats) {
      SS_HIP(hipEventCreate(&f0));
      SS_HIP(hipEventCreate(&f1));
      SS_HIP(hipEventRecord(f0, s));
    }
    for (int j = 0; j < max_nt; ++j) {
      const int per = max_nt - j;
      const int64_t nb = xcd ? 8 * ceil_div(nc, 8) * (int64_t)per : (int64_t)nc * per;
      if (j > 0) k_dn_update<<<(unsigned)nb, kDnBlock, 0, s>>>(nc, per, j, xcd, dcls, W);
      k_dn_panel<<<(unsigned)nb, kDnBlock, 0, s>>>(nc, per, j, xcd, dcls, W, Dg, err);
    }
    SS_HIP(hipGetLastError());
    if (stats) SS_HIP(hipEventRecord(f1, s));
    const size_t lds = (size_t)(kT * kLdT + max_nt * kT) * sizeof(double2);
    if (op->wide_norm)
      k_dn_subst<int64_t><<<(unsigned)nc, kDnBlock, lds, s>>>(nc, dcls, (const int64_t*)od.norm, W, Dg,
                                                              op->d_exec2canon, static_cast<const double2*>(f_dev),
                                                              static_cast<double2*>(u_dev));
    else
      k_dn_subst<int32_t><<<(unsigned)nc, kDnBlock, lds, s>>>(nc, dcls, (const int32_t*)od.norm, W, Dg,
                                                              op->d_exec2canon, static_cast<const double2*>(f_dev),
                                                              static_cast<double2*>(u_dev));
    SS_HIP(hipGetLastError());
    int h_err[2] = {0, 0};
    SS_HIP(hipMemcpyAsync(h_err, err, sizeof(h_err), hipMemcpyDeviceToHost, s));
    SS_HIP(hipStreamSynchronize(s));
    if (stats) {
      float ms = 0;
      SS_HIP(hipEventElapsedTime(&ms, f0, f1));
      stats->factor_ms += ms;
      (void)hipEventDestroy(f0);
      (void)hipEventDestroy(f1);
      stats->chunks += 1;
      stats->tiles += tiles;
    }
    if (h_err[1]) return fail(SS_EDEVICE, "dense assembly found a column outside its class");
    if (h_err[0] && result == SS_OK)
      result = fail(SS_ENOTPD, "a pivot of the dense Cholesky factorisation was not positive");
  }
  return result;
}

}  // namespace ss
