// Dense direct solve of the truncated Galerkin system, one connected class at a time: the
// paper's own solver (Alg. 1, steps 4-5: assemble L_N densely, solve directly), restricted to
// the independent blocks the classes of Sec. 6 split it into.
//
// Each class block is Hermitian positive definite on the nonzero frequencies (the operator is
// Hermitian, and coercive by Prop. ExistenceUniquenessStability); the zero frequency has an
// all-zero row and column, and is given the identity instead (u_0 = 0).  The block is factored
// by a tiled left-looking Cholesky, L L^H, in FP64 or FP32, the launch of tile column j doing
//   below the diagonal:  A_ij -= sum_{s<j} L_is L_js^H;  L_ij = A_ij M_j^H              (i > j)
//   the next diagonal:   A_jj -= sum_{s<j} L_js L_js^H;  L_jj = chol(A_jj);  M_j = L_jj^{-1}
// (the products on MFMA, split over s across the waves of a block), then L y = f and L^H u = y by
// tile substitution, the diagonal blocks applied as products with M_j.  With an FP32 factor the
// substitutions are steps of iterative refinement, u += solve(f - L u), the residual and u in
// FP64.  Storage: per class the lower triangle of 32 x 32 complex tiles, each tile column-major
// and contiguous (16 KB in FP64), row-major over tiles: tile (i, j), j <= i, is number
// i (i + 1) / 2 + j.  The inverses M_j go to an array of their own; the diagonal tiles keep the
// updated A_jj.
#include <algorithm>
#include <cmath>
#include <vector>

#include "ss_internal.h"

namespace ss {

namespace {

constexpr int kT = 32;                        // tile rows and columns (complex entries)
constexpr int kTE = kT * kT;                  // entries per tile
constexpr int kLdT = kT + 1;                  // LDS row stride of a staged tile
constexpr int kDnBlock = 256;
constexpr int kDnWaves = kDnBlock / 64;
constexpr int64_t kDirectMaxRows = 32768;     // rows of one class (4.3 GB of FP32, 8.6 GB of FP64 tiles)
constexpr size_t kSubstLds = 150 * 1024;     // LDS the substitution may take for the class vector
constexpr int64_t kDirectBudget = int64_t(16) << 30;  // factor storage per chunk of classes

typedef double d4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));

// Arithmetic of one factorisation precision: complex type, MFMA accumulator, the 16x16x4 MFMA
// and the row its result item v holds in lane (column + 16 k): 4 v + k in FP64, 4 k + v in FP32
// (measured layouts of the two instructions on gfx950).
template <typename T> struct Prec;
template <> struct Prec<double> {
  typedef double2 C;
  typedef d4_t A4;
  __device__ static A4 mma(double a, double b, A4 c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
  __device__ static int row(int v, int k) { return 4 * v + k; }
  __host__ __device__ static C mk(double x, double y) { return make_double2(x, y); }
};
template <> struct Prec<float> {
  typedef float2 C;
  typedef f4_t A4;
  __device__ static A4 mma(float a, float b, A4 c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
  __device__ static int row(int v, int k) { return 4 * k + v; }
  __host__ __device__ static C mk(float x, float y) { return make_float2(x, y); }
};

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

// ---- assembly: row i of a class writes its entries (i, l) with l <= i; padding rows of the last
// tile and the zero frequency get a unit diagonal.  Every entry is 4 pi^2 (k . l) a_{k-l},
// formed as (|k|^2 + |l|^2 - |k-l|^2) 2 pi^2 a_{k-l} in the integer type of the norms, in FP64, and
// stored in the factorisation precision T.
template <typename NormT, typename T>
__global__ __launch_bounds__(kDnBlock) void k_dn_assemble(int nc, const DClass* __restrict__ cls,
                                                           const uint32_t* __restrict__ sent,
                                                           const uint32_t* __restrict__ sptr,
                                                           const NormT* __restrict__ norm,
                                                           const double2* __restrict__ A64,
                                                           const int64_t* __restrict__ nu, typename Prec<T>::C* __restrict__ W,
                                                           int* __restrict__ err) {
  const int c = blockIdx.y;
  if (c >= nc) return;
  const DClass C = cls[c];
  const int i = blockIdx.x * kDnBlock + threadIdx.x;
  if (i >= C.nt * kT) return;
  typedef typename Prec<T>::C C2;
  C2* tiles = W + C.tbase * kTE;
  const int64_t ti = i / kT;
  C2* diag = tiles + (tri(ti) + ti) * kTE + (i % kT) * kT + (i % kT);
  if (i >= C.n) {
    *diag = Prec<T>::mk(1, 0);
    return;
  }
  const int64_t e = C.e0 + i;
  const NormT nk = norm[e];
  if (nk == 0) {
    *diag = Prec<T>::mk(1, 0);
    return;
  }
  const int64_t sl = e / kSlice;
  const int lane = (int)(e % kSlice);
  const uint32_t base = sptr[sl];
  const uint32_t width = (sptr[sl + 1] - base) / kSlice;
  const double2* At = A64 + (int64_t)C.prob * kTab;
  const int64_t* nut = nu + (int64_t)C.prob * kTab;
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
    tiles[(tri(ti) + tj) * kTE + (l % kT) * kT + (i % kT)] = Prec<T>::mk((T)(fi * a.x), (T)(fi * a.y));
  }
}

// ---- split-K tile products.  The wave w of a block accumulates sum_{s = w, w+4, ... < ns}
// P_s Q_s^H, P_s and Q_s the tiles s of two tile rows of L (consecutive tiles, kTE apart), as
// 2 x 2 quadrants of 16 x 16 MFMA accumulators (FP64 or FP32), real and imaginary part each:
//   (P Q^H)_re = Pre Qre^T + Pim Qim^T,   (P Q^H)_im = Pim Qre^T - Pre Qim^T.
// MFMA 16x16x4 operands: lane = row + 16 k for A (16 x 4) and column + 16 k for B (4 x 16); the
// result holds (Prec::row(v, lane / 16), lane mod 16) in item v.  Operands come in groups of
// k-steps, the next groups loaded while the current one is multiplied.
template <typename T>
struct Acc {
  typename Prec<T>::A4 re[2][2], im[2][2];
};

template <typename T>
__device__ inline void acc_zero(Acc<T>& A) {
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      A.re[a][b] = typename Prec<T>::A4{0, 0, 0, 0};
      A.im[a][b] = typename Prec<T>::A4{0, 0, 0, 0};
    }
}

constexpr int kGroup = 2;   // k-steps of 4 per operand group

template <typename T>
struct Group {
  typename Prec<T>::C p[kGroup][2], q[kGroup][2];
};

template <typename T>
__device__ inline void load_group(const typename Prec<T>::C* __restrict__ P, const typename Prec<T>::C* __restrict__ Q,
                                  int kc0, int lr, int lk, Group<T>& g) {
#pragma unroll
  for (int u = 0; u < kGroup; ++u) {
    const int col = 4 * (kc0 + u) + lk;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      g.p[u][h] = P[col * kT + 16 * h + lr];
      g.q[u][h] = Q[col * kT + 16 * h + lr];
    }
  }
}

// eight independent accumulators between the two products that feed each one
template <typename T>
__device__ inline void mma_group(const Group<T>& g, Acc<T>& A) {
#pragma unroll
  for (int u = 0; u < kGroup; ++u) {
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        A.re[a][b] = Prec<T>::mma(g.p[u][a].x, g.q[u][b].x, A.re[a][b]);
        A.im[a][b] = Prec<T>::mma(g.p[u][a].y, g.q[u][b].x, A.im[a][b]);
      }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        A.re[a][b] = Prec<T>::mma(g.p[u][a].y, g.q[u][b].y, A.re[a][b]);
        A.im[a][b] = Prec<T>::mma(-g.p[u][a].x, g.q[u][b].y, A.im[a][b]);
      }
  }
}

template <typename T>
__device__ void split_k(const typename Prec<T>::C* __restrict__ Prow, const typename Prec<T>::C* __restrict__ Qrow,
                        int ns, Acc<T>& A) {
  constexpr int kPer = (kT / 4) / kGroup;   // groups per tile
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int lr = lane & 15, lk = lane >> 4;
  const int cnt = ns > wave ? (ns - wave + kDnWaves - 1) / kDnWaves : 0;
  const int G = kPer * cnt;
  if (G == 0) return;
  auto load = [&](int g, Group<T>& dst) {
    const int64_t s = wave + (int64_t)(g / kPer) * kDnWaves;
    load_group(Prow + s * kTE, Qrow + s * kTE, (g % kPer) * kGroup, lr, lk, dst);
  };
  // two groups in flight ahead of the one being multiplied, three buffers in rotation: the loop
  // body is straight-line code (addresses past the last group are clamped to it), so each wait
  // covers only the group about to be multiplied
  Group<T> b0, b1, b2;
  load(0, b0);
  load(min(1, G - 1), b1);
  int g = 0;
  for (; g + 3 <= G; g += 3) {
    load(min(g + 2, G - 1), b2);
    mma_group(b0, A);
    load(min(g + 3, G - 1), b0);
    mma_group(b1, A);
    load(min(g + 4, G - 1), b1);
    mma_group(b2, A);
  }
  if (g < G) mma_group(b0, A);
  if (g + 1 < G) mma_group(b1, A);
}

// C = A - (sum of the four waves' products), summed in wave order through one LDS tile `buf`,
// into LDS (element (r, c) at c * ld + r)
template <typename T>
__device__ void reduce_into(Acc<T>& A, const typename Prec<T>::C* __restrict__ Ag, typename Prec<T>::C* buf,
                            typename Prec<T>::C* C, int ld) {
  typedef typename Prec<T>::C C2;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int lr = lane & 15, lk = lane >> 4;
  for (int w = 1; w < kDnWaves; ++w) {
    if (wave == w) {
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int r = 16 * a + Prec<T>::row(v, lk), cc = 16 * b + lr;
            buf[cc * kT + r] = Prec<T>::mk(A.re[a][b][v], A.im[a][b][v]);
          }
    }
    __syncthreads();
    if (wave == 0) {
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int r = 16 * a + Prec<T>::row(v, lk), cc = 16 * b + lr;
            const C2 o = buf[cc * kT + r];
            A.re[a][b][v] += o.x;
            A.im[a][b][v] += o.y;
          }
    }
    __syncthreads();
  }
  if (wave == 0) {
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int r = 16 * a + Prec<T>::row(v, lk), cc = 16 * b + lr;
          const C2 x = Ag[cc * kT + r];
          C[cc * ld + r] = Prec<T>::mk(x.x - A.re[a][b][v], x.y - A.im[a][b][v]);
        }
  }
  __syncthreads();
}

// In-LDS Cholesky of the lower triangle of a 32 x 32 tile (stride kLdT), as L D L^H with the
// unit-lower columns kept unscaled and divided by the pivot on the fly, then scaled to L = L1
// D^{1/2}.  One barrier per column.  A pivot that is not positive and finite sets *bad and is
// replaced by 1, so the factor stays finite.
template <typename T>
__device__ void tile_chol(typename Prec<T>::C* sA, T* sd, int* bad) {
  typedef typename Prec<T>::C C2;
  const int tid = threadIdx.x;
  for (int c = 0; c < kT; ++c) {
    __syncthreads();
    T piv = sA[c * kLdT + c].x;
    if (!(piv > (T)0) || !(piv < (T)INFINITY)) {
      if (tid == 0) *bad = 1;
      piv = 1;
      if (tid == 0) sA[c * kLdT + c] = Prec<T>::mk(1, 0);
    }
    const T ip = (T)1 / piv;
    for (int idx = tid; idx < kTE; idx += kDnBlock) {
      const int r = idx & (kT - 1), q = idx >> 5;   // element (r, q), column q
      if (q > c && r >= q) {
        const C2 arc = sA[c * kLdT + r], aqc = sA[c * kLdT + q];
        // A_rq -= A_rc conj(A_qc) / piv
        const T tr = arc.x * aqc.x + arc.y * aqc.y, ti = arc.y * aqc.x - arc.x * aqc.y;
        C2 v = sA[q * kLdT + r];
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
      const T d = sd[q];
      C2 v = sA[q * kLdT + r];
      if (r == q) {
        v = Prec<T>::mk(sqrt(d), 0);
      } else {
        const T s = (T)1 / sqrt(d);
        v = Prec<T>::mk(v.x * s, v.y * s);
      }
      sA[q * kLdT + r] = v;
    }
  }
  __syncthreads();
}

// Factor the updated diagonal tile in sD (stride kLdT), invert the factor into sM (stride kLdT),
// write M = L^{-1} (lower, column-major) to Mout.  *s_bad must be 0 on entry.
template <typename T>
__device__ void diag_tail(typename Prec<T>::C* sD, typename Prec<T>::C* sM, T* piv, int* s_bad,
                          typename Prec<T>::C* __restrict__ Mout, int* __restrict__ err) {
  typedef typename Prec<T>::C C2;
  const int tid = threadIdx.x;
  tile_chol<T>(sD, piv, s_bad);
  // one column per thread: M_rc = (delta_rc - sum_{c<=m<r} L_rm M_mc) / L_rr
  if (tid < kT) {
    const int cc = tid;
    for (int r = 0; r < kT; ++r) {
      if (r < cc) {
        sM[cc * kLdT + r] = Prec<T>::mk(0, 0);
        continue;
      }
      T xr = r == cc ? 1 : 0, xi = 0;
      for (int m = cc; m < r; ++m) {
        const C2 l = sD[m * kLdT + r], x = sM[cc * kLdT + m];
        xr -= l.x * x.x - l.y * x.y;
        xi -= l.x * x.y + l.y * x.x;
      }
      const T il = (T)1 / sD[r * kLdT + r].x;
      sM[cc * kLdT + r] = Prec<T>::mk(xr * il, xi * il);
    }
  }
  __syncthreads();
  for (int idx = tid; idx < kTE; idx += kDnBlock) Mout[idx] = sM[(idx >> 5) * kLdT + (idx & (kT - 1))];
  if (tid == 0 && *s_bad) err[0] = 1;
}

// ---- tile column j, diagonal only: A_jj -= sum_{s<j} L_js L_js^H, L_jj = chol(A_jj), M_j =
// L_jj^{-1}; one block per class (used for j = 0; later diagonals are done by k_dn_offdiag)
template <typename T>
__global__ __launch_bounds__(kDnBlock) void k_dn_diag(int nc, int j, const DClass* __restrict__ cls,
                                                       const typename Prec<T>::C* __restrict__ W,
                                                       typename Prec<T>::C* __restrict__ Minv, int* __restrict__ err) {
  typedef typename Prec<T>::C C2;
  const int c = blockIdx.x;
  if (c >= nc) return;
  const DClass C = cls[c];
  if (j >= C.nt) return;
  const C2* tiles = W + C.tbase * kTE;
  __shared__ C2 buf[kT * kLdT];
  __shared__ C2 sD[kT * kLdT];
  __shared__ T s_piv[kT];
  __shared__ int s_bad;
  if (threadIdx.x == 0) s_bad = 0;
  const C2* Arow = tiles + tri(j) * kTE;
  Acc<T> A;
  acc_zero(A);
  split_k<T>(Arow, Arow, j, A);
  reduce_into<T>(A, Arow + (int64_t)j * kTE, buf, sD, kLdT);
  diag_tail<T>(sD, buf, s_piv, &s_bad, Minv + (C.dbase + j) * kTE, err);
}

// ---- tile column j, below the diagonal: A_ij -= sum_{s<j} L_is L_js^H, then L_ij = A_ij M_j^H
// (the triangular solve L_ij L_jj^H = A_ij as a product with the inverse), both on MFMA.  The
// block of i = j + 1 then does the next diagonal: A_{j+1,j+1} -= sum_{s<=j} L_{j+1,s} L_{j+1,s}^H
// (the s = j term from the tile it just computed, in LDS), its factor and inverse M_{j+1}.  Blocks
// go out tile row by tile row, so those come first.
template <typename T>
__global__ __launch_bounds__(kDnBlock) void k_dn_offdiag(int nc, int per, int j, bool xcd,
                                                          const DClass* __restrict__ cls,
                                                          typename Prec<T>::C* __restrict__ W,
                                                          typename Prec<T>::C* __restrict__ Minv,
                                                          int* __restrict__ err) {
  typedef typename Prec<T>::C C2;
  typedef typename Prec<T>::A4 A4;
  const int64_t b = blockIdx.x;
  int c, t;
  if (xcd) {
    const int64_t k = b >> 3, nc8 = (nc + 7) / 8;
    t = (int)(k / nc8);
    c = (int)((b & 7) + 8 * (k % nc8));
  } else {
    t = (int)(b / nc);
    c = (int)(b % nc);
  }
  if (c >= nc || t >= per) return;
  const DClass C = cls[c];
  const int i = j + 1 + t;
  if (i >= C.nt) return;
  C2* tiles = W + C.tbase * kTE;
  __shared__ C2 buf[kT * kLdT];
  __shared__ C2 sC[kT * kLdT];
  __shared__ C2 sX[kTE];
  __shared__ T s_piv[kT];
  __shared__ int s_bad;
  if (threadIdx.x == 0) s_bad = 0;
  Acc<T> A;
  acc_zero(A);
  split_k<T>(tiles + tri(i) * kTE, tiles + tri(j) * kTE, j, A);
  C2* Aij = tiles + (tri(i) + j) * kTE;
  reduce_into<T>(A, Aij, buf, sC, kLdT);
  // X = C M^H: wave (a, b) computes quadrant (a, b); A operand C from LDS, B operand M from HBM
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int lr = lane & 15, lk = lane >> 4;
  const int qa = wave >> 1, qb = wave & 1;
  const C2* M = Minv + (C.dbase + j) * kTE;
  A4 xr = {0, 0, 0, 0}, xi = {0, 0, 0, 0};
#pragma unroll
  for (int kc = 0; kc < kT / 4; ++kc) {
    const int col = 4 * kc + lk;
    const C2 p = sC[col * kLdT + 16 * qa + lr];
    const C2 q = M[col * kT + 16 * qb + lr];
    xr = Prec<T>::mma(p.x, q.x, xr);
    xi = Prec<T>::mma(p.y, q.x, xi);
    xr = Prec<T>::mma(p.y, q.y, xr);
    xi = Prec<T>::mma(-p.x, q.y, xi);
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int r = 16 * qa + Prec<T>::row(v, lk), cc = 16 * qb + lr;
    Aij[cc * kT + r] = Prec<T>::mk(xr[v], xi[v]);
    sX[cc * kT + r] = Prec<T>::mk(xr[v], xi[v]);
  }
  if (t != 0) return;
  __syncthreads();
  // next diagonal: the tiles s < j of row i from HBM, s = j (X) from LDS split over the waves by k
  acc_zero(A);
  split_k<T>(tiles + tri(i) * kTE, tiles + tri(i) * kTE, j, A);
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int col = 4 * (2 * wave + u) + lk;
    C2 p[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) p[h] = sX[col * kT + 16 * h + lr];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int bb = 0; bb < 2; ++bb) {
        A.re[a][bb] = Prec<T>::mma(p[a].x, p[bb].x, A.re[a][bb]);
        A.im[a][bb] = Prec<T>::mma(p[a].y, p[bb].x, A.im[a][bb]);
        A.re[a][bb] = Prec<T>::mma(p[a].y, p[bb].y, A.re[a][bb]);
        A.im[a][bb] = Prec<T>::mma(-p[a].x, p[bb].y, A.im[a][bb]);
      }
  }
  reduce_into<T>(A, tiles + (tri(i) + i) * kTE, buf, sC, kLdT);
  diag_tail<T>(sC, buf, s_piv, &s_bad, Minv + (C.dbase + i) * kTE, err);
}

// ---- L y = b, then L^H d = y, one block per class, the class vector in LDS in the factorisation
// precision.  The diagonal blocks are products with M_s (one thread per row); the off-diagonal
// tile products are spread over the block (the vector in device memory when the class is too large
// for LDS).  One refinement step: b = r (execution order, FP64;
// the zero frequency's row gives 0), then x += d in FP64.  A class whose residual ratio is already
// at most tol2 takes no step, so each class's iterate does not depend on the others'.
template <typename NormT, typename T>
__global__ __launch_bounds__(kDnBlock) void k_dn_subst(int nc, const DClass* __restrict__ cls,
                                                        const NormT* __restrict__ norm,
                                                        const typename Prec<T>::C* __restrict__ W,
                                                        const typename Prec<T>::C* __restrict__ Minv,
                                                        const double2* __restrict__ r, double2* __restrict__ x,
                                                        const double* __restrict__ ratio, double tol2,
                                                        typename Prec<T>::C* __restrict__ gv) {
  typedef typename Prec<T>::C C2;
  const int c = blockIdx.x;
  if (c >= nc) return;
  if (ratio && ratio[c] <= tol2) return;
  const DClass C = cls[c];
  extern __shared__ __align__(16) char s_raw[];
  C2* sT = reinterpret_cast<C2*>(s_raw);   // staged inverse diagonal factor, stride kLdT
  // the class vector, nt * kT entries: in LDS, or for classes too large for it in device memory
  // (at the class's diagonal-tile offset; the block's barriers order its accesses there as well)
  C2* v = gv ? gv + C.dbase * kT : sT + kT * kLdT;
  const C2* tiles = W + C.tbase * kTE;
  const int tid = threadIdx.x;
  const int np = C.nt * kT;
  for (int i = tid; i < np; i += kDnBlock) {
    C2 b = Prec<T>::mk(0, 0);
    if (i < C.n && norm[C.e0 + i] != 0) {
      const double2 rv = r[C.e0 + i];
      b = Prec<T>::mk((T)rv.x, (T)rv.y);
    }
    v[i] = b;
  }
  // forward: L y = b
  for (int s = 0; s < C.nt; ++s) {
    __syncthreads();
    const C2* Ms = Minv + (C.dbase + s) * kTE;
    for (int idx = tid; idx < kTE; idx += kDnBlock) sT[(idx >> 5) * kLdT + (idx & (kT - 1))] = Ms[idx];
    __syncthreads();
    C2 y = Prec<T>::mk(0, 0);
    if (tid < kT) {   // y_s = M_s b_s
      for (int cc = 0; cc < kT; ++cc) {
        const C2 m = sT[cc * kLdT + tid], xv = v[s * kT + cc];
        y.x += m.x * xv.x - m.y * xv.y;
        y.y += m.x * xv.y + m.y * xv.x;
      }
    }
    __syncthreads();
    if (tid < kT) v[s * kT + tid] = y;
    __syncthreads();
    for (int R = (s + 1) * kT + tid; R < np; R += kDnBlock) {
      const int ti = R / kT, rr = R % kT;
      const C2* L = tiles + (tri(ti) + s) * kTE;
      T sx = 0, sy = 0;
#pragma unroll 8
      for (int cc = 0; cc < kT; ++cc) {
        const C2 l = L[cc * kT + rr], yv = v[s * kT + cc];
        sx += l.x * yv.x - l.y * yv.y;
        sy += l.x * yv.y + l.y * yv.x;
      }
      C2 xv = v[R];
      xv.x -= sx;
      xv.y -= sy;
      v[R] = xv;
    }
  }
  // backward: L^H d = y
  for (int s = C.nt - 1; s >= 0; --s) {
    __syncthreads();
    const C2* Ms = Minv + (C.dbase + s) * kTE;
    for (int idx = tid; idx < kTE; idx += kDnBlock) sT[(idx >> 5) * kLdT + (idx & (kT - 1))] = Ms[idx];
    __syncthreads();
    C2 y = Prec<T>::mk(0, 0);
    if (tid < kT) {   // d_s = M_s^H b_s, (M^H)_{r,c} = conj(M_{c,r})
      for (int cc = 0; cc < kT; ++cc) {
        const C2 m = sT[tid * kLdT + cc], xv = v[s * kT + cc];
        y.x += m.x * xv.x + m.y * xv.y;
        y.y += m.x * xv.y - m.y * xv.x;
      }
    }
    __syncthreads();
    if (tid < kT) v[s * kT + tid] = y;
    __syncthreads();
    for (int R = tid; R < s * kT; R += kDnBlock) {
      const int ti = R / kT, rr = R % kT;
      const C2* L = tiles + (tri(s) + ti) * kTE;   // tile (s, ti), its column rr
      T sx = 0, sy = 0;
#pragma unroll 8
      for (int cc = 0; cc < kT; ++cc) {
        const C2 l = L[rr * kT + cc], yv = v[s * kT + cc];
        sx += l.x * yv.x + l.y * yv.y;
        sy += l.x * yv.y - l.y * yv.x;
      }
      C2 xv = v[R];
      xv.x -= sx;
      xv.y -= sy;
      v[R] = xv;
    }
  }
  __syncthreads();
  for (int i = tid; i < C.n; i += kDnBlock) {
    const C2 d = v[i];
    double2 xv = x[C.e0 + i];
    xv.x += (double)d.x;
    xv.y += (double)d.y;
    x[C.e0 + i] = xv;
  }
}

// f in execution order (0 on padding rows); x = 0
__global__ void k_dn_start(int64_t n_exec, const int64_t* __restrict__ exec2canon, const double2* __restrict__ f,
                           double2* __restrict__ fe, double2* __restrict__ x) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n_exec) return;
  const int64_t g = exec2canon[e];
  fe[e] = g >= 0 ? f[g] : make_double2(0.0, 0.0);
  x[e] = make_double2(0.0, 0.0);
}

// r = f - y over each class's rows (the zero frequency's row left out), and per class |r|^2 / |f|^2
// in a fixed order (0 for f = 0)
template <typename NormT>
__global__ __launch_bounds__(kDnBlock) void k_dn_resid(int nc, const DClass* __restrict__ cls,
                                                        const NormT* __restrict__ norm,
                                                        const double2* __restrict__ fe, const double2* __restrict__ y,
                                                        double2* __restrict__ r, double* __restrict__ ratio) {
  const int c = blockIdx.x;
  if (c >= nc) return;
  const DClass C = cls[c];
  double rr = 0, ff = 0;
  for (int i = threadIdx.x; i < C.n; i += kDnBlock) {
    const int64_t e = C.e0 + i;
    double2 rv = make_double2(0.0, 0.0);
    if (norm[e] != 0) {
      const double2 fv = fe[e], yv = y[e];
      rv = make_double2(fv.x - yv.x, fv.y - yv.y);
      ff += fv.x * fv.x + fv.y * fv.y;
    }
    r[e] = rv;
    rr += rv.x * rv.x + rv.y * rv.y;
  }
  __shared__ double s0[kDnBlock], s1[kDnBlock];
  s0[threadIdx.x] = rr;
  s1[threadIdx.x] = ff;
  __syncthreads();
  for (int h = kDnBlock / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) {
      s0[threadIdx.x] += s0[threadIdx.x + h];
      s1[threadIdx.x] += s1[threadIdx.x + h];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) ratio[c] = s1[0] > 0 ? s0[0] / s1[0] : 0.0;
}

__global__ void k_dn_scatter(int64_t n_exec, const int64_t* __restrict__ exec2canon, const double2* __restrict__ x,
                             double2* __restrict__ u) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n_exec) return;
  const int64_t g = exec2canon[e];
  if (g >= 0) u[g] = x[e];
}

constexpr int kMaxRefine = 30;

}  // namespace

namespace {

// One chunk of classes: assemble, factor in precision T, then refinement steps (x += solve(f - L x)
// with the FP64 residual) until every class of the chunk has |r_c| <= tol |f_c| (one step when
// tol <= 0).  x and fe are execution-order FP64 vectors of the whole operator.
template <typename T>
ss_status run_chunk(const OpImpl* op, const std::vector<DClass>& ch, int64_t tiles, int64_t dtiles, int max_nt,
                    double tol, const double2* fe, double2* x, double2* r, double2* y, hipStream_t s,
                    DirectStats* stats, bool* not_pd, int* steps, double* worst) {
  typedef typename Prec<T>::C C2;
  const OpDev od = op->dev();
  const int nc = (int)ch.size();
  C2 *W = nullptr, *Dg = nullptr;   // lower tiles; inverses of the diagonal factors
  DClass* dcls = nullptr;
  int* err = nullptr;
  double* ratio = nullptr;
  struct Release {   // every block this chunk allocated, returned on every exit path
    hipStream_t s;
    std::vector<void*> p;
    ~Release() {
      (void)hipStreamSynchronize(s);
      for (void* b : p) pool_free(b);
    }
  } rel{s, {}};
  SS_TRY(dalloc(&W, (size_t)std::max<int64_t>(tiles, 1) * kTE));
  rel.p.push_back(W);
  SS_TRY(dalloc(&Dg, (size_t)std::max<int64_t>(dtiles, 1) * kTE));
  rel.p.push_back(Dg);
  SS_TRY(dalloc((char**)&dcls, (size_t)nc * sizeof(DClass)));
  rel.p.push_back(dcls);
  SS_TRY(dalloc(&err, 2));
  rel.p.push_back(err);
  SS_TRY(dalloc(&ratio, (size_t)nc));
  rel.p.push_back(ratio);
  SS_HIP(h2d(dcls, ch.data(), (size_t)nc * sizeof(DClass), s));
  SS_HIP(hipMemsetAsync(W, 0, (size_t)tiles * kTE * sizeof(C2), s));
  SS_HIP(hipMemsetAsync(err, 0, 2 * sizeof(int), s));
  const dim3 ag((unsigned)ceil_div((int64_t)max_nt * kT, kDnBlock), (unsigned)nc);
  if (op->wide_norm)
    k_dn_assemble<int64_t, T><<<ag, kDnBlock, 0, s>>>(nc, dcls, od.sent, od.sptr, (const int64_t*)od.norm, od.A64,
                                                       od.nu, W, err);
  else
    k_dn_assemble<int32_t, T><<<ag, kDnBlock, 0, s>>>(nc, dcls, od.sent, od.sptr, (const int32_t*)od.norm, od.A64,
                                                       od.nu, W, err);
  SS_HIP(hipGetLastError());
  const bool xcd = nc >= 8;
  hipEvent_t f0 = nullptr, f1 = nullptr;
  if (stats) {
    SS_HIP(hipEventCreate(&f0));
    SS_HIP(hipEventCreate(&f1));
    SS_HIP(hipEventRecord(f0, s));
  }
  k_dn_diag<T><<<(unsigned)nc, kDnBlock, 0, s>>>(nc, 0, dcls, W, Dg, err);
  for (int j = 0; j + 1 < max_nt; ++j) {
    const int per = max_nt - j - 1;
    const int64_t nb = xcd ? 8 * ceil_div(nc, 8) * (int64_t)per : (int64_t)nc * per;
    k_dn_offdiag<T><<<(unsigned)nb, kDnBlock, 0, s>>>(nc, per, j, xcd, dcls, W, Dg, err);
  }
  SS_HIP(hipGetLastError());
  if (stats) SS_HIP(hipEventRecord(f1, s));
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
  if (h_err[0]) *not_pd = true;
  size_t lds = (size_t)(kT * kLdT + max_nt * kT) * sizeof(C2);
  C2* gv = nullptr;
  if (lds > kSubstLds) {
    SS_TRY(dalloc(&gv, (size_t)dtiles * kT));
    rel.p.push_back(gv);
    lds = (size_t)kT * kLdT * sizeof(C2);
  }
  const double tol2 = tol * tol;
  std::vector<double> h_ratio(nc);
  const double2* rhs = fe;   // the first step solves with f itself (x = 0)
  const double* gate = nullptr;
  int step = 0;
  for (;;) {
    if (op->wide_norm)
      k_dn_subst<int64_t, T><<<(unsigned)nc, kDnBlock, lds, s>>>(nc, dcls, (const int64_t*)od.norm, W, Dg, rhs, x,
                                                                  gate, tol2, gv);
    else
      k_dn_subst<int32_t, T><<<(unsigned)nc, kDnBlock, lds, s>>>(nc, dcls, (const int32_t*)od.norm, W, Dg, rhs, x,
                                                                  gate, tol2, gv);
    SS_HIP(hipGetLastError());
    ++step;
    SS_TRY(apply_impl(op, SS_FP64, x, y, s));
    if (op->wide_norm)
      k_dn_resid<int64_t><<<(unsigned)nc, kDnBlock, 0, s>>>(nc, dcls, (const int64_t*)od.norm, fe, y, r, ratio);
    else
      k_dn_resid<int32_t><<<(unsigned)nc, kDnBlock, 0, s>>>(nc, dcls, (const int32_t*)od.norm, fe, y, r, ratio);
    SS_HIP(hipGetLastError());
    SS_HIP(hipMemcpyAsync(h_ratio.data(), ratio, (size_t)nc * sizeof(double), hipMemcpyDeviceToHost, s));
    SS_HIP(hipStreamSynchronize(s));
    double w = 0;
    for (double v : h_ratio) w = std::max(w, v);
    if (tol <= 0 || w <= tol2 || step >= kMaxRefine || *not_pd) {
      *steps = std::max(*steps, step);
      *worst = std::max(*worst, std::sqrt(w));
      return SS_OK;
    }
    rhs = r;
    gate = ratio;
  }
}

}  // namespace

ss_status direct_solve_impl(const OpImpl* op, const void* f_dev, void* u_dev, ss_precision prec, double tol,
                            hipStream_t s, DirectStats* stats) {
  if (!op || !f_dev || !u_dev) return fail(SS_EINVAL, "null argument");
  if (prec != SS_FP64 && prec != SS_FP32_REFINE) return fail(SS_EINVAL, "unknown precision");
  if (!(tol == tol)) return fail(SS_EINVAL, "tol is not a number");
  const int64_t n_cls = (int64_t)op->cls_n.size();
  int64_t max_n = 0;
  for (int64_t k = 0; k < n_cls; ++k) max_n = std::max(max_n, op->cls_n[k]);
  if (max_n > kDirectMaxRows)
    return fail(SS_ERANGE, "a class has more than 32768 rows: too large for the dense direct solve");
  // the problem of every class, from the execution offsets
  std::vector<int32_t> cprob(n_cls);
  for (int64_t k = 0; k < n_cls; ++k)
    cprob[k] = (int32_t)(std::upper_bound(op->eoff.begin(), op->eoff.end(), op->cls_e0[k]) - op->eoff.begin()) - 1;
  if (stats) *stats = DirectStats{};
  const size_t cbytes = prec == SS_FP64 ? sizeof(double2) : sizeof(float2);
  // chunks of consecutive classes of about equal storage, each within the budget (a chunk holds
  // one class at least), so no chunk is left with a few classes that cannot fill the device
  auto class_bytes = [&](int64_t k) {
    const int64_t nt = ceil_div(op->cls_n[k], kT);
    return (tri(nt) + nt) * kTE * (int64_t)cbytes;
  };
  int64_t total_bytes = 0;
  for (int64_t k = 0; k < n_cls; ++k) total_bytes += class_bytes(k);
  const int64_t n_chunks = std::max<int64_t>(1, ceil_div(total_bytes, kDirectBudget));
  const int64_t target = ceil_div(total_bytes, n_chunks);
  // execution-order FP64 vectors of the whole operator: f, x, residual, L x
  const int64_t ne = op->n_exec;
  double2* vec = nullptr;
  SS_TRY(dalloc(&vec, (size_t)ne * 4));
  struct Release {
    hipStream_t s;
    void* p;
    ~Release() {
      (void)hipStreamSynchronize(s);
      pool_free(p);
    }
  } rel{s, vec};
  double2 *fe = vec, *x = vec + ne, *r = vec + 2 * ne, *y = vec + 3 * ne;
  k_dn_start<<<(unsigned)std::max<int64_t>(1, ceil_div(ne, kDnBlock)), kDnBlock, 0, s>>>(
      ne, op->d_exec2canon, static_cast<const double2*>(f_dev), fe, x);
  SS_HIP(hipGetLastError());
  bool not_pd = false;
  int steps = 0;
  double worst = 0;
  int64_t k0 = 0;
  while (k0 < n_cls) {
    std::vector<DClass> ch;
    int64_t tiles = 0, dtiles = 0;
    int max_nt = 0;
    int64_t k = k0;
    for (; k < n_cls && (int64_t)ch.size() < 65535; ++k) {
      const int nt = (int)ceil_div(op->cls_n[k], kT);
      const int64_t need = class_bytes(k), have = (tiles + dtiles) * kTE * (int64_t)cbytes;
      if (!ch.empty() && (have + need > kDirectBudget || have >= target)) break;
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
    k0 = k;
    if (prec == SS_FP64)
      SS_TRY(run_chunk<double>(op, ch, tiles, dtiles, max_nt, tol, fe, x, r, y, s, stats, &not_pd, &steps, &worst));
    else
      SS_TRY(run_chunk<float>(op, ch, tiles, dtiles, max_nt, tol, fe, x, r, y, s, stats, &not_pd, &steps, &worst));
  }
  k_dn_scatter<<<(unsigned)std::max<int64_t>(1, ceil_div(ne, kDnBlock)), kDnBlock, 0, s>>>(
      ne, op->d_exec2canon, x, static_cast<double2*>(u_dev));
  SS_HIP(hipGetLastError());
  SS_HIP(hipStreamSynchronize(s));
  if (stats) {
    stats->refine_steps = steps;
    stats->rel_residual = worst;
  }
  if (not_pd) return fail(SS_ENOTPD, "a pivot of the dense Cholesky factorisation was not positive");
  if (tol > 0 && worst > tol) return fail(SS_ENOCONV, "refinement did not reach tol within 30 steps");
  return SS_OK;
}

}  // namespace ss
