// Advection-diffusion-reaction extension (Remark ADR, Eq. ADR): -div(a grad u) + b . grad u + c u = f.
// The operator gains, per neighbour pair (k, l = k - w_j), the advection and reaction terms
//   2 pi i (l . b_j) + c_j
// beside the diffusion term 2 pi^2 (|k|^2 + |l|^2 - |w_j|^2) a_j.  The stamp and the operator are
// built by the diffusion path on the union of the supports (closed under negation, with 0), with
// a_j = 0 where w_j is not in supp(a); this module stores the whole complex FP64 coefficient of every
// SELL entry (the matvec streams it), the diagonal, and a batched Jacobi-preconditioned
// BiCGSTAB (the operator is not Hermitian, so CG does not apply) in FP64 with per-problem scalars
// and fixed-order per-problem reductions.  With c_0 > 0 the zero frequency is an ordinary unknown.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>

#include "ss_internal.h"

namespace ss {

namespace {

constexpr int kAdrBlock = 256;

inline unsigned adr_grid(int64_t n) { return (unsigned)std::max<int64_t>(1, ceil_div(n, kAdrBlock)); }

// problem of every execution row
__global__ void k_adr_pid(int64_t n_exec, int n_prob, const int64_t* __restrict__ eoff, int32_t* __restrict__ pid) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n_exec) return;
  int lo = 0, hi = n_prob - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (eoff[mid] <= e) lo = mid;
    else hi = mid - 1;
  }
  pid[e] = lo;
}

// E[q] = 2 pi^2 (|k|^2 + |l|^2 - |w_j|^2) a_j + 2 pi i (l . b_j) + c_j, the whole coefficient of
// every stored entry q of row e (l the key of the entry's column), and the diagonal D[e] = the
// coefficient of the entry with w_j = 0.  Padding rows get D = 1.
template <typename NormT>
__global__ void k_adr_coef(int64_t n_exec, int d, const int32_t* __restrict__ pid, const int64_t* __restrict__ eoff,
                           const int64_t* __restrict__ exec2canon, const int16_t* __restrict__ keys,
                           const uint32_t* __restrict__ sent, const uint32_t* __restrict__ sptr,
                           const NormT* __restrict__ norm, const double2* __restrict__ A64,
                           const int64_t* __restrict__ nu, const double2* __restrict__ Bt,
                           const double2* __restrict__ Ct, const int32_t* __restrict__ zero_j,
                           double2* __restrict__ E, uint32_t* __restrict__ col, double2* __restrict__ D) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n_exec) return;
  const int64_t sl = e / kSlice;
  const int lane = (int)(e % kSlice);
  const uint32_t base = sptr[sl];
  const uint32_t width = (sptr[sl + 1] - base) / kSlice;
  if (exec2canon[e] < 0) {
    D[e] = make_double2(1.0, 0.0);
    for (uint32_t q = 0; q < width; ++q) {
      E[base + q * kSlice + lane] = make_double2(0.0, 0.0);
      col[base + q * kSlice + lane] = (uint32_t)e;
    }
    return;
  }
  const int p = pid[e];
  const NormT nk = norm[e];
  const double2* Bp = Bt + (int64_t)p * kTab * d;
  const double2* Cp = Ct + (int64_t)p * kTab;
  const int zj = zero_j[p];
  double2 diag = make_double2(0.0, 0.0);
  for (uint32_t q = 0; q < width; ++q) {
    const uint32_t ent = sent[base + q * kSlice + lane];
    const uint32_t j = ent >> kColBits;
    double2 v = make_double2(0.0, 0.0);
    if (j != (uint32_t)kNullJ) {
      const int64_t ge = eoff[p] + (int64_t)(ent & kColMask);
      const int16_t* l = keys + exec2canon[ge] * d;
      const double2* b = Bp + (int64_t)j * d;
      double sr = 0, si = 0;   // l . b_j
      for (int t = 0; t < d; ++t) {
        const double lt = (double)l[t];
        sr += lt * b[t].x;
        si += lt * b[t].y;
      }
      const double tp = 2.0 * M_PI;
      const NormT I = nk + norm[ge] - (NormT)nu[(int64_t)p * kTab + j];
      const double2 a = A64[(int64_t)p * kTab + j];
      v = make_double2((double)I * a.x + (Cp[j].x - tp * si), (double)I * a.y + (Cp[j].y + tp * sr));
      if ((int)j == zj) diag = v;
    }
    E[base + q * kSlice + lane] = v;
    // a padding entry keeps coefficient 0 and points at its own row
    col[base + q * kSlice + lane] = j != (uint32_t)kNullJ ? (uint32_t)(eoff[p] + (int64_t)(ent & kColMask)) : (uint32_t)e;
  }
  D[e] = diag;
}

// problem of every SELL slice (problems start on slice boundaries)
__global__ void k_adr_spid(int64_t n_slices, int n_prob, const int64_t* __restrict__ eoff, int32_t* __restrict__ spid) {
  const int64_t sl = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (sl >= n_slices) return;
  const int64_t e = sl * kSlice;
  int lo = 0, hi = n_prob - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (eoff[mid] <= e) lo = mid;
    else hi = mid - 1;
  }
  spid[sl] = lo;
}

// y = L x over every problem: one wavefront per SELL slice (64 rows, one per lane), the global
// column and the whole complex coefficient of every stored entry streamed with nontemporal loads,
// eight entries of a lane in flight while a row has that many left; padding entries have
// coefficient 0 and padding rows only such entries, so they get 0.  A slice of a finished problem
// is skipped.  Blocks are numbered XCD by XCD, so each XCD walks a contiguous eighth of the slices
// (a problem or two at a time) and its L2 keeps those problems' x for the gathers.
typedef double adr_d2v __attribute__((ext_vector_type(2)));
__global__ __launch_bounds__(kAdrBlock) void k_adr_mv(int64_t n_slices, const int32_t* __restrict__ spid,
                                                      const uint32_t* __restrict__ sptr,
                                                      const uint32_t* __restrict__ col, const double2* __restrict__ E,
                                                      const uint8_t* __restrict__ done, const double2* __restrict__ x,
                                                      double2* __restrict__ y) {
  const int64_t nb = (n_slices * kSlice + kAdrBlock - 1) / kAdrBlock;
  const int64_t sl = __builtin_amdgcn_readfirstlane((int)((xcd_block(nb) * kAdrBlock + threadIdx.x) >> 6));
  if (sl >= n_slices) return;
  const int lane = threadIdx.x & 63;
  const int p = __builtin_amdgcn_readfirstlane(spid[sl]);
  if (done && done[p]) return;
  const uint32_t base = __builtin_amdgcn_readfirstlane(sptr[sl]);
  const uint32_t width = (__builtin_amdgcn_readfirstlane(sptr[sl + 1]) - base) / kSlice;
  const uint32_t* cl = col + base + lane;
  const adr_d2v* El = reinterpret_cast<const adr_d2v*>(E + base + lane);
  double ar = 0, ai = 0;
  constexpr int kU = 8;
  uint32_t q0 = 0;
  for (; q0 + kU <= width; q0 += kU) {
    uint32_t c[kU];
    adr_d2v v[kU];
    double2 xv[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) c[u] = __builtin_nontemporal_load(cl + (q0 + u) * kSlice);
#pragma unroll
    for (int u = 0; u < kU; ++u) v[u] = __builtin_nontemporal_load(El + (q0 + u) * kSlice);
#pragma unroll
    for (int u = 0; u < kU; ++u) xv[u] = x[c[u]];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      ar += v[u].x * xv[u].x - v[u].y * xv[u].y;
      ai += v[u].x * xv[u].y + v[u].y * xv[u].x;
    }
  }
  for (; q0 < width; ++q0) {
    const uint32_t c = __builtin_nontemporal_load(cl + q0 * kSlice);
    const adr_d2v v = __builtin_nontemporal_load(El + q0 * kSlice);
    const double2 xv = x[c];
    ar += v.x * xv.x - v.y * xv.y;
    ai += v.x * xv.y + v.y * xv.x;
  }
  __builtin_nontemporal_store(adr_d2v{ar, ai}, reinterpret_cast<adr_d2v*>(y + sl * kSlice + lane));
}

// per-problem BiCGSTAB scalars
struct AdrState {
  double2 rho, alpha, omega, beta;
  double rr, ff;
  int32_t iters, status;
};

__device__ inline double2 cmul(double2 a, double2 b) { return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
__device__ inline double2 cdiv(double2 a, double2 b) {
  const double den = b.x * b.x + b.y * b.y;
  return make_double2((a.x * b.x + a.y * b.y) / den, (a.y * b.x - a.x * b.y) / den);
}
// conj(a) b
__device__ inline double2 cdot(double2 a, double2 b) { return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x); }

// one block per problem: up to three complex inner products over its rows in a fixed order
__device__ void block_dots(int64_t e0, int64_t e1, const double2* a0, const double2* b0, const double2* a1,
                           const double2* b1, const double2* a2, const double2* b2, double2 out[3]) {
  __shared__ double2 s[3][kAdrBlock];
  double2 acc[3] = {make_double2(0, 0), make_double2(0, 0), make_double2(0, 0)};
  for (int64_t e = e0 + threadIdx.x; e < e1; e += kAdrBlock) {
    double2 t = cdot(a0[e], b0[e]);
    acc[0].x += t.x;
    acc[0].y += t.y;
    if (a1) {
      t = cdot(a1[e], b1[e]);
      acc[1].x += t.x;
      acc[1].y += t.y;
    }
    if (a2) {
      t = cdot(a2[e], b2[e]);
      acc[2].x += t.x;
      acc[2].y += t.y;
    }
  }
  for (int i = 0; i < 3; ++i) s[i][threadIdx.x] = acc[i];
  __syncthreads();
  for (int h = kAdrBlock / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h)
      for (int i = 0; i < 3; ++i) {
        s[i][threadIdx.x].x += s[i][threadIdx.x + h].x;
        s[i][threadIdx.x].y += s[i][threadIdx.x + h].y;
      }
    __syncthreads();
  }
  for (int i = 0; i < 3; ++i) out[i] = s[i][0];
}

enum { DOT_START = 0, DOT_ALPHA = 1, DOT_OMEGA = 2, DOT_RHO = 3 };

struct AdrVecs {
  double2 *f, *x, *r, *rh, *p, *ph, *v, *s, *sh, *t;
};

// the scalar steps of BiCGSTAB, one block per active problem
template <int MODE>
__global__ __launch_bounds__(kAdrBlock) void k_adr_dots(const int64_t* __restrict__ eoff, AdrVecs V,
                                                        AdrState* __restrict__ st, uint8_t* __restrict__ done,
                                                        double tol2) {
  const int p = blockIdx.x;
  if (done[p]) return;
  const int64_t e0 = eoff[p], e1 = eoff[p + 1];
  double2 o[3];
  AdrState S = st[p];
  if (MODE == DOT_START) {   // r = f - A x already formed: rh = r, |r|^2, |f|^2, rho = <rh, r>
    block_dots(e0, e1, V.r, V.r, V.f, V.f, nullptr, nullptr, o);
    S.rr = o[0].x;
    S.ff = o[1].x;
    S.rho = make_double2(o[0].x, 0.0);
    S.alpha = S.omega = make_double2(1.0, 0.0);
    S.beta = make_double2(0.0, 0.0);
    if (threadIdx.x == 0) {
      if (S.ff == 0.0 || S.rr <= tol2 * S.ff) {
        S.status = SS_OK;
        done[p] = 1;
      }
      st[p] = S;
    }
    return;
  }
  if (MODE == DOT_ALPHA) {   // alpha = rho / <rh, v>
    block_dots(e0, e1, V.rh, V.v, nullptr, nullptr, nullptr, nullptr, o);
    if (threadIdx.x == 0) {
      if (o[0].x == 0.0 && o[0].y == 0.0) {
        S.status = SS_EBREAKDOWN;
        done[p] = 1;
      } else {
        S.alpha = cdiv(S.rho, o[0]);
      }
      st[p] = S;
    }
    return;
  }
  if (MODE == DOT_OMEGA) {   // omega = <t, s> / <t, t>
    block_dots(e0, e1, V.t, V.s, V.t, V.t, nullptr, nullptr, o);
    if (threadIdx.x == 0) {
      S.omega = o[1].x > 0.0 ? make_double2(o[0].x / o[1].x, o[0].y / o[1].x) : make_double2(0.0, 0.0);
      st[p] = S;
    }
    return;
  }
  // DOT_RHO: rho' = <rh, r>, |r|^2; stop test; beta = (rho' / rho) (alpha / omega)
  block_dots(e0, e1, V.rh, V.r, V.r, V.r, nullptr, nullptr, o);
  if (threadIdx.x == 0) {
    S.iters += 1;
    S.rr = o[1].x;
    if (S.rr <= tol2 * S.ff) {
      S.status = SS_OK;
      done[p] = 1;
    } else if ((S.omega.x == 0.0 && S.omega.y == 0.0) || (o[0].x == 0.0 && o[0].y == 0.0) || !std::isfinite(S.rr)) {
      S.status = SS_EBREAKDOWN;
      done[p] = 1;
    } else {
      S.beta = cmul(cdiv(o[0], S.rho), cdiv(S.alpha, S.omega));
      S.rho = o[0];
    }
    st[p] = S;
  }
}

// p = r + beta (p - omega v); ph = p / D
__global__ void k_adr_p(int64_t n, const int32_t* __restrict__ pid, const uint8_t* __restrict__ done,
                        const AdrState* __restrict__ st, const double2* __restrict__ D, AdrVecs V) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const int p = pid[e];
  if (done[p]) return;
  const AdrState S = st[p];
  const double2 pv = V.p[e], vv = V.v[e], rv = V.r[e];
  const double2 t = cmul(S.omega, vv);
  const double2 q = cmul(S.beta, make_double2(pv.x - t.x, pv.y - t.y));
  const double2 np = make_double2(rv.x + q.x, rv.y + q.y);
  V.p[e] = np;
  V.ph[e] = cdiv(np, D[e]);
}

// s = r - alpha v; sh = s / D
__global__ void k_adr_s(int64_t n, const int32_t* __restrict__ pid, const uint8_t* __restrict__ done,
                        const AdrState* __restrict__ st, const double2* __restrict__ D, AdrVecs V) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const int p = pid[e];
  if (done[p]) return;
  const double2 t = cmul(st[p].alpha, V.v[e]);
  const double2 sv = make_double2(V.r[e].x - t.x, V.r[e].y - t.y);
  V.s[e] = sv;
  V.sh[e] = cdiv(sv, D[e]);
}

// x += alpha ph + omega sh; r = s - omega t
__global__ void k_adr_x(int64_t n, const int32_t* __restrict__ pid, const uint8_t* __restrict__ done,
                        const AdrState* __restrict__ st, AdrVecs V) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const int p = pid[e];
  if (done[p]) return;
  const AdrState S = st[p];
  const double2 a = cmul(S.alpha, V.ph[e]), b = cmul(S.omega, V.sh[e]), c = cmul(S.omega, V.t[e]);
  V.x[e] = make_double2(V.x[e].x + a.x + b.x, V.x[e].y + a.y + b.y);
  V.r[e] = make_double2(V.s[e].x - c.x, V.s[e].y - c.y);
}

// gather f to execution order, x = 0
__global__ void k_adr_start(int64_t n, const int64_t* __restrict__ exec2canon, const double2* __restrict__ fc,
                            AdrVecs V) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const int64_t g = exec2canon[e];
  const double2 z = make_double2(0.0, 0.0);
  V.f[e] = g >= 0 ? fc[g] : z;
  V.x[e] = z;
  V.p[e] = z;
  V.v[e] = z;
}

// r = f - t (t = A x), rh = r, for the problems not done; p = v = 0
__global__ void k_adr_resid(int64_t n, const int32_t* __restrict__ pid, const uint8_t* __restrict__ done,
                            AdrVecs V) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  if (done[pid[e]]) return;
  const double2 r = make_double2(V.f[e].x - V.t[e].x, V.f[e].y - V.t[e].y);
  V.r[e] = r;
  V.rh[e] = r;
  V.p[e] = make_double2(0.0, 0.0);
  V.v[e] = make_double2(0.0, 0.0);
}

// per problem: |f - A x|^2 with t = A x, and |f|^2
__global__ __launch_bounds__(kAdrBlock) void k_adr_true(const int64_t* __restrict__ eoff, AdrVecs V,
                                                        double2* __restrict__ out) {
  const int p = blockIdx.x;
  const int64_t e0 = eoff[p], e1 = eoff[p + 1];
  __shared__ double s0[kAdrBlock], s1[kAdrBlock];
  double a = 0, b = 0;
  for (int64_t e = e0 + threadIdx.x; e < e1; e += kAdrBlock) {
    const double rx = V.f[e].x - V.t[e].x, ry = V.f[e].y - V.t[e].y;
    a += rx * rx + ry * ry;
    b += V.f[e].x * V.f[e].x + V.f[e].y * V.f[e].y;
  }
  s0[threadIdx.x] = a;
  s1[threadIdx.x] = b;
  __syncthreads();
  for (int h = kAdrBlock / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) {
      s0[threadIdx.x] += s0[threadIdx.x + h];
      s1[threadIdx.x] += s1[threadIdx.x + h];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) out[p] = make_double2(s0[0], s1[0]);
}

__global__ void k_adr_scatter(int64_t n, const int64_t* __restrict__ exec2canon, const double2* __restrict__ x,
                              double2* __restrict__ u) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const int64_t g = exec2canon[e];
  if (g >= 0) u[g] = x[e];
}

}  // namespace

struct AdrImpl {
  const OpImpl* op = nullptr;
  int device = 0;
  double2* E = nullptr;        // [n_sell] whole coefficient of every stored entry
  uint32_t* col = nullptr;     // [n_sell] global execution column of every stored entry
  double2* D = nullptr;        // [n_exec] diagonal
  int32_t* pid = nullptr;      // [n_exec]
  int32_t* spid = nullptr;     // [n_slices]
};

ss_status adr_build_impl(const StampImpl* st, const OpImpl* op, const int32_t* n_b, const int16_t* b_freqs,
                         const double* b_hat, const int32_t* n_c, const int16_t* c_freqs, const double* c_hat,
                         hipStream_t s, AdrImpl** out) {
  if (!st || !op || !n_b || !n_c || !out) return fail(SS_EINVAL, "null argument");
  *out = nullptr;
  if (op->total != st->total || op->n_prob != st->n_prob) return fail(SS_EINVAL, "the operator was not built on this stamp");
  const int np = op->n_prob, d = op->d;
  // per problem: table index of every b and c frequency in the operator's (union) table
  std::vector<double2> Bt((size_t)np * kTab * d, make_double2(0, 0)), Ct((size_t)np * kTab, make_double2(0, 0));
  std::vector<int32_t> zj(np);
  int64_t bpos = 0, cpos = 0;
  for (int p = 0; p < np; ++p) {
    const int32_t a0 = st->a_off[p], a1 = st->a_off[p + 1];
    const int16_t* tab = st->a_keys.data() + (size_t)a0 * d;
    const int s_p = a1 - a0;
    zj[p] = st->a_zero[p];
    auto find = [&](const int16_t* w) -> int {
      for (int j = 0; j < s_p; ++j)
        if (std::memcmp(tab + (size_t)j * d, w, (size_t)d * sizeof(int16_t)) == 0) return j;
      return -1;
    };
    if (n_b[p] < 0 || n_c[p] < 0) return fail(SS_EINVAL, "negative support size");
    for (int i = 0; i < n_b[p]; ++i, ++bpos) {
      const int j = find(b_freqs + bpos * d);
      if (j < 0) return fail(SS_EINVAL, "a frequency of b is not in the operator's support (build on the union)");
      for (int t = 0; t < d; ++t) {
        const double re = b_hat[2 * (bpos * d + t)], im = b_hat[2 * (bpos * d + t) + 1];
        if (!std::isfinite(re) || !std::isfinite(im)) return fail(SS_EINVAL, "b_hat is not finite");
        double2& dst = Bt[((size_t)p * kTab + j) * d + t];
        dst.x += re;
        dst.y += im;
      }
    }
    bool c0 = false;
    for (int i = 0; i < n_c[p]; ++i, ++cpos) {
      const int j = find(c_freqs + cpos * d);
      if (j < 0) return fail(SS_EINVAL, "a frequency of c is not in the operator's support (build on the union)");
      const double re = c_hat[2 * cpos], im = c_hat[2 * cpos + 1];
      if (!std::isfinite(re) || !std::isfinite(im)) return fail(SS_EINVAL, "c_hat is not finite");
      Ct[(size_t)p * kTab + j].x += re;
      Ct[(size_t)p * kTab + j].y += im;
      if (j == zj[p]) c0 = true;
    }
    if (!c0 || !(Ct[(size_t)p * kTab + zj[p]].x > 0.0) || Ct[(size_t)p * kTab + zj[p]].y != 0.0)
      return fail(SS_EINVAL, "c_0 must be real and positive (the zero frequency is then an ordinary unknown)");
  }
  std::unique_ptr<AdrImpl, void (*)(AdrImpl*)> A(new AdrImpl(), adr_free_impl);   // frees on every error path
  A->op = op;
  A->device = op->device;
  double2 *dB = nullptr, *dC = nullptr;
  int32_t* dz = nullptr;
  struct Tmp {
    hipStream_t s;
    std::vector<void*> b;
    ~Tmp() {
      (void)hipStreamSynchronize(s);
      for (void* p : b) pool_free(p);
    }
  } tmp{s, {}};
  SS_TRY(dalloc(&dB, Bt.size()));
  tmp.b.push_back(dB);
  SS_TRY(dalloc(&dC, Ct.size()));
  tmp.b.push_back(dC);
  SS_TRY(dalloc(&dz, (size_t)np));
  tmp.b.push_back(dz);
  SS_HIP(h2d(dB, Bt.data(), Bt.size() * sizeof(double2), s));
  SS_HIP(h2d(dC, Ct.data(), Ct.size() * sizeof(double2), s));
  SS_HIP(h2d(dz, zj.data(), (size_t)np * sizeof(int32_t), s));
  if (op->n_exec >= (int64_t(1) << 32)) return fail(SS_ERANGE, "too many rows for 32-bit global columns");
  SS_TRY(dalloc(&A->E, (size_t)std::max<int64_t>(op->n_sell, 1)));
  SS_TRY(dalloc(&A->col, (size_t)std::max<int64_t>(op->n_sell, 1)));
  SS_TRY(dalloc(&A->D, (size_t)op->n_exec));
  SS_TRY(dalloc(&A->pid, (size_t)op->n_exec));
  SS_TRY(dalloc(&A->spid, (size_t)std::max<int64_t>(op->n_slices, 1)));
  const OpDev od = op->dev();
  const int64_t ne = op->n_exec;
  k_adr_pid<<<adr_grid(ne), kAdrBlock, 0, s>>>(ne, np, op->d_eoff, A->pid);
  k_adr_spid<<<adr_grid(op->n_slices), kAdrBlock, 0, s>>>(op->n_slices, np, op->d_eoff, A->spid);
  if (op->wide_norm)
    k_adr_coef<int64_t><<<adr_grid(ne), kAdrBlock, 0, s>>>(ne, d, A->pid, op->d_eoff, op->d_exec2canon, st->d_keys,
                                                           od.sent, od.sptr, (const int64_t*)od.norm, od.A64, od.nu,
                                                           dB, dC, dz, A->E, A->col, A->D);
  else
    k_adr_coef<int32_t><<<adr_grid(ne), kAdrBlock, 0, s>>>(ne, d, A->pid, op->d_eoff, op->d_exec2canon, st->d_keys,
                                                           od.sent, od.sptr, (const int32_t*)od.norm, od.A64, od.nu,
                                                           dB, dC, dz, A->E, A->col, A->D);
  SS_HIP(hipGetLastError());
  SS_HIP(hipStreamSynchronize(s));
  *out = A.release();
  return SS_OK;
}

void adr_free_impl(AdrImpl* A) {
  if (!A) return;
  dfree(A->E);
  dfree(A->col);
  dfree(A->D);
  dfree(A->pid);
  dfree(A->spid);
  delete A;
}

namespace {
ss_status adr_mv(const AdrImpl* A, const uint8_t* done, const double2* x, double2* y, hipStream_t s) {
  const OpImpl* op = A->op;
  const OpDev od = op->dev();
  const int64_t ns = op->n_slices;
  k_adr_mv<<<xcd_grid(ceil_div(ns * kSlice, kAdrBlock)), kAdrBlock, 0, s>>>(ns, A->spid, od.sptr, A->col, A->E, done, x, y);
  SS_HIP(hipGetLastError());
  return SS_OK;
}
}  // namespace

ss_status adr_apply_impl(const AdrImpl* A, const void* x, void* y, hipStream_t s) {
  if (!A || !x || !y) return fail(SS_EINVAL, "null argument");
  return adr_mv(A, nullptr, static_cast<const double2*>(x), static_cast<double2*>(y), s);
}

ss_status adr_solve_impl(const AdrImpl* A, const void* f, void* u, double tol, int32_t max_iter, hipStream_t s,
                         ss_solve_info* info) {
  if (!A || !f || !u) return fail(SS_EINVAL, "null argument");
  if (!(tol > 0.0) || max_iter < 1) return fail(SS_EINVAL, "tol must be positive and max_iter at least 1");
  const OpImpl* op = A->op;
  const int np = op->n_prob;
  const int64_t ne = op->n_exec;
  std::vector<void*> blocks;
  struct Release {
    hipStream_t s;
    std::vector<void*>* b;
    ~Release() {
      (void)hipStreamSynchronize(s);
      for (void* p : *b) pool_free(p);
    }
  } rel{s, &blocks};
  double2* vec = nullptr;
  SS_TRY(dalloc(&vec, (size_t)ne * 10));
  blocks.push_back(vec);
  AdrVecs V{vec, vec + ne, vec + 2 * ne, vec + 3 * ne, vec + 4 * ne, vec + 5 * ne, vec + 6 * ne, vec + 7 * ne,
            vec + 8 * ne, vec + 9 * ne};
  AdrState* st = nullptr;
  uint8_t* done = nullptr;
  double2* tr = nullptr;
  SS_TRY(dalloc((char**)&st, (size_t)np * sizeof(AdrState)));
  blocks.push_back(st);
  SS_TRY(dalloc(&done, (size_t)np));
  blocks.push_back(done);
  SS_TRY(dalloc(&tr, (size_t)np));
  blocks.push_back(tr);
  SS_HIP(hipMemsetAsync(st, 0, (size_t)np * sizeof(AdrState), s));
  SS_HIP(hipMemsetAsync(done, 0, (size_t)np, s));
  const unsigned g = adr_grid(ne);
  const double tol2 = tol * tol;
  k_adr_start<<<g, kAdrBlock, 0, s>>>(ne, op->d_exec2canon, static_cast<const double2*>(f), V);
  std::vector<uint8_t> hdone(np, 0);
  std::vector<double2> htr(np);
  int iters_done = 0;
  // a start (or restart from the true residual), then iterations until every problem stops by
  // its recursively updated residual; the true residual decides, with at most 3 restarts
  for (int restart = 0; restart < 4; ++restart) {
    SS_TRY(adr_mv(A, done, V.x, V.t, s));
    k_adr_resid<<<g, kAdrBlock, 0, s>>>(ne, A->pid, done, V);
    k_adr_dots<DOT_START><<<np, kAdrBlock, 0, s>>>(op->d_eoff, V, st, done, tol2);
    bool all = false;
    while (iters_done < max_iter && !all) {
      const int burst = std::min(8, max_iter - iters_done);
      for (int it = 0; it < burst; ++it) {
        k_adr_p<<<g, kAdrBlock, 0, s>>>(ne, A->pid, done, st, A->D, V);
        SS_TRY(adr_mv(A, done, V.ph, V.v, s));
        k_adr_dots<DOT_ALPHA><<<np, kAdrBlock, 0, s>>>(op->d_eoff, V, st, done, tol2);
        k_adr_s<<<g, kAdrBlock, 0, s>>>(ne, A->pid, done, st, A->D, V);
        SS_TRY(adr_mv(A, done, V.sh, V.t, s));
        k_adr_dots<DOT_OMEGA><<<np, kAdrBlock, 0, s>>>(op->d_eoff, V, st, done, tol2);
        k_adr_x<<<g, kAdrBlock, 0, s>>>(ne, A->pid, done, st, V);
        k_adr_dots<DOT_RHO><<<np, kAdrBlock, 0, s>>>(op->d_eoff, V, st, done, tol2);
      }
      SS_HIP(hipGetLastError());
      iters_done += burst;
      SS_HIP(hipMemcpyAsync(hdone.data(), done, (size_t)np, hipMemcpyDeviceToHost, s));
      SS_HIP(hipStreamSynchronize(s));
      all = std::all_of(hdone.begin(), hdone.end(), [](uint8_t v) { return v != 0; });
    }
    // true residuals; problems above tol start again from them
    SS_HIP(hipMemsetAsync(done, 0, (size_t)np, s));
    SS_TRY(adr_mv(A, nullptr, V.x, V.t, s));
    k_adr_true<<<np, kAdrBlock, 0, s>>>(op->d_eoff, V, tr);
    SS_HIP(hipMemcpyAsync(htr.data(), tr, (size_t)np * sizeof(double2), hipMemcpyDeviceToHost, s));
    SS_HIP(hipStreamSynchronize(s));
    bool again = false;
    for (int p = 0; p < np; ++p) {
      hdone[p] = !(htr[p].x > tol2 * htr[p].y);
      again |= !hdone[p];
    }
    if (!again || iters_done >= max_iter) break;
    SS_HIP(h2d(done, hdone.data(), (size_t)np, s));
  }
  k_adr_scatter<<<g, kAdrBlock, 0, s>>>(ne, op->d_exec2canon, V.x, static_cast<double2*>(u));
  SS_HIP(hipGetLastError());
  std::vector<AdrState> hs(np);
  SS_HIP(hipMemcpyAsync(hs.data(), st, (size_t)np * sizeof(AdrState), hipMemcpyDeviceToHost, s));
  SS_HIP(hipStreamSynchronize(s));
  ss_status worst = SS_OK;
  for (int p = 0; p < np; ++p) {
    const double rel = htr[p].y > 0 ? std::sqrt(htr[p].x / htr[p].y) : 0.0;
    ss_status stp = rel <= tol ? SS_OK : (hs[p].status == SS_EBREAKDOWN ? SS_EBREAKDOWN : SS_ENOCONV);
    if (info) {
      info[p] = ss_solve_info{};
      info[p].iters = hs[p].iters;
      info[p].rel_residual = rel;
      info[p].n = op->row_off[p + 1] - op->row_off[p];
      info[p].nnz = op->nnz_p[p];
      info[p].n_components = op->comps[p];
      info[p].status = stp;
    }
    if (stp != SS_OK && worst == SS_OK) worst = stp;
  }
  if (worst == SS_EBREAKDOWN) return fail(SS_EBREAKDOWN, "BiCGSTAB broke down for a problem");
  if (worst == SS_ENOCONV) return fail(SS_ENOCONV, "a problem missed the tolerance within max_iter");
  return SS_OK;
}

}  // namespace ss
