// Matvec, Jacobi-preconditioned CG, FP32 + FP64 refinement, and the
// continuous-batching engine, all on the SELL-64 layout.
//
// Operator (Sec. 9, Eq. FiniteGalerkinOperator): for execution row e holding
// key k and a stored entry (column c holding l = k - w_j, index j)
//     coefficient = 4 pi^2 (k . l) a_j = 2 pi^2 (|k|^2 + |l|^2 - |w_j|^2) a_j,
// the integer bracket exact in int32 (int64 when |k|^2 >= 2^30), the factor
// 2 pi^2 a_j pre-scaled per problem and staged in LDS with |w_j|^2.
//
// Every launch works on a list of problem descriptors (operator slice, vectors,
// solver state, request parameters) and a list of work items (up to four
// 64-row slices of one problem per 256-thread block; one wavefront per slice,
// one lane per row; a slice's entries are stored column-major so each step of
// the row loop is one coalesced 256-byte load).  Work items are dealt to
// blocks so consecutive items land on one XCD (the hardware deals blocks to
// the 8 XCDs round-robin), keeping a problem's gathers in one L2.  The same
// kernels serve a batch of problems of one operator (ss_solve_op) and a
// changing mix of problems of many operators (the engine), so a problem's
// arithmetic never depends on what runs beside it.
//
// CG: textbook PCG with the Jacobi diagonal 4 pi^2 |k|^2 a_0 (the denominator
// of the recurrence in the proof of Prop. SolutionSupport; row k = 0 is
// identically zero and excluded).  Each problem has its own scalars; each
// inner product is reduced in a fixed order -- lanes, wavefronts, then the
// problem's work items -- so results are bitwise independent of the batch.
// Per iteration: mv (q = L p, <p,q>), update (x, r, <r, D^-1 r>, |r|^2),
// dir (beta, stop test |r| <= tol |f|, p).  A scalar written by one kernel is
// read only by later kernels.
//
// FP32 + refinement, as a per-problem device state machine: r = f - L x with
// the FP64 operator; stop if |r| <= tol |f|; else scale r to unit norm, run
// FP32 PCG (FP32 operator and vectors, FP64 inner products) to a loose
// tolerance, add the correction to x in FP64, repeat.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <memory>
#include <mutex>
#include <unordered_map>

#include "ss_internal.h"

namespace ss {

namespace {

constexpr double kFourPi2 = 4.0 * M_PI * M_PI;
// A correction solve (FP32) stops once its residual is below kInnerTol relative to its right-hand
// side, or earlier when kInnerMargin times the reduction that the outer target still asks for is
// reached: a last correction then does no more than the FP64 stop test needs.
constexpr double kInnerTol = 1e-5;
constexpr double kInnerMargin = 0.5;
constexpr int kMaxOuter = 30;

enum { MV_PLAIN = 0, MV_DOT = 1, MV_RESID = 2 };

// LDS of the matvec: a-table (64 x 16 B), |w_j|^2 (64 x 8 B), 4 partials, then the window
constexpr int kLdsFixed = kTab * 16 + kTab * 8 + kSolveWaves * 8;

// dynamic LDS bytes of a matvec over windows of up to `win` rows
inline size_t mv_lds_bytes(int64_t win, bool fp64, bool wide) {
  return kLdsFixed + (size_t)win * ((fp64 ? 16 : 8) + (wide ? 8 : 4));
}

// One problem in a launch.
struct Desc {
  const uint32_t* sent;        // operator SELL entries
  const uint32_t* sptr;        // operator slice offsets (operator-global slice index)
  const void* norm;            // |k|^2 of the problem's first execution row
  const double2* A64;          // the problem's kTab-entry tables
  const float2* A32;
  const int64_t* nu;
  const int64_t* exec2canon;   // problem's execution rows -> operator-global canonical slot (-1 pad)
  const double2* f_canon;      // request: operator-global canonical f
  double2* u_canon;            // request: operator-global canonical u (in: x0, out: solution)
  double2 *x64, *r64, *p64, *q64, *f64;   // problem-local, execution order
  float2 *x32, *r32, *p32, *q32;
  PState* ps;                  // FP64 / outer state
  PState* ps_in;               // FP32 inner state
  double a0;
  double tol2, tol2_in;
  int64_t slice0;              // operator-global index of the problem's first slice
  int64_t n_rows;              // execution rows (multiple of 64)
  int32_t max_iter;
  int32_t prec;                // SS_FP64 or SS_FP32_REFINE
  int32_t wide;                // int64 norms
  int32_t wb, we;              // the problem's work items in the current list
  int32_t init;                // first tick after admission
  int32_t final_;              // retiring: compute the true residual and write u
  int32_t pad;
};

template <typename V> struct Real;
template <> struct Real<double2> { using T = double; };
template <> struct Real<float2> { using T = float; };

__device__ inline int work_index(int b, int per) { return (b & 7) * per + (b >> 3); }

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Sum of v over the block, returned to every thread.  Fixed order.
__device__ inline double block_sum(double v, double* red) {
  static_assert(kSolveWaves == 8, "reduction tree below is written for 8 wavefronts");
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) red[wave] = v;
  __syncthreads();
  const double s = ((red[0] + red[1]) + (red[2] + red[3])) + ((red[4] + red[5]) + (red[6] + red[7]));
  __syncthreads();
  return s;
}

// Sum of part[i*2 + off] for i in [b, e), every thread gets the result.  Fixed order.
__device__ inline double range_sum(const double* __restrict__ part, int off, int b, int e, double* red) {
  double v = 0;
  for (int i = b + (int)threadIdx.x; i < e; i += kSolveBlock) v += part[(int64_t)i * 2 + off];
  return block_sum(v, red);
}

// CG state of the problem's current CG run
__device__ inline PState* cg_state(const Desc& D) { return D.prec == SS_FP64 ? D.ps : D.ps_in; }

// no CG work for this problem now
__device__ inline bool cg_idle(const Desc& D) {
  return D.ps->done || (D.prec != SS_FP64 && D.ps_in->done);
}

template <typename NormT>
__device__ inline double jacobi_inv(NormT nk, double a0) {
  return nk > 0 ? 1.0 / (kFourPi2 * a0 * (double)nk) : 0.0;
}

// Row of the SELL slice at `base`: sum over its entries of (nk + |l|^2 - nu_j) A_j x_l.
// WIN: x and |l|^2 come from the LDS window starting at execution row w0.
template <bool WIN, typename NormT, typename V, int kChunk = 8>   // kChunk: entry loads in flight per lane
__device__ inline V sell_row(const uint32_t* __restrict__ sent, uint32_t base, uint32_t width, int lane, NormT nk,
                             const NormT* __restrict__ normp, const V* __restrict__ xp, int w0, const V* As,
                             const NormT* nus) {
  using R = typename Real<V>::T;
  R ar = 0, ai = 0;
  for (uint32_t q0 = 0; q0 < width; q0 += kChunk) {
    uint32_t ent[kChunk];
#pragma unroll
    for (int k = 0; k < kChunk; ++k)
      ent[k] = q0 + k < width ? __builtin_nontemporal_load(sent + base + (q0 + k) * kSlice + lane)
                              : (uint32_t)kNullJ << kColBits;
#pragma unroll
    for (int k = 0; k < kChunk; ++k) {
      const uint32_t j = ent[k] >> kColBits;
      if (j != (uint32_t)kNullJ) {
        const int c = (int)(ent[k] & kColMask) - (WIN ? w0 : 0);
        const NormT I = nk + normp[c] - nus[j];
        const V a = As[j];
        const V x = xp[c];
        const R fi = (R)I;
        const R cr = fi * a.x, ci = fi * a.y;
        ar += cr * x.x - ci * x.y;
        ai += cr * x.y + ci * x.x;
      }
    }
  }
  V out;
  out.x = ar;
  out.y = ai;
  return out;
}

// Streaming accesses that are not to stay in the caches (the matvec's window staging and its
// output): nontemporal loads and stores of whole complex values.
typedef double d2v_t __attribute__((ext_vector_type(2)));
typedef float f2v_t __attribute__((ext_vector_type(2)));
__device__ inline void st_nt(double2* p, double2 v) {
  __builtin_nontemporal_store(d2v_t{v.x, v.y}, reinterpret_cast<d2v_t*>(p));
}
__device__ inline void st_nt(float2* p, float2 v) {
  __builtin_nontemporal_store(f2v_t{v.x, v.y}, reinterpret_cast<f2v_t*>(p));
}
__device__ inline double2 ld_nt(const double2* p) {
  const d2v_t v = __builtin_nontemporal_load(reinterpret_cast<const d2v_t*>(p));
  return make_double2(v.x, v.y);
}
__device__ inline float2 ld_nt(const float2* p) {
  const f2v_t v = __builtin_nontemporal_load(reinterpret_cast<const f2v_t*>(p));
  return make_float2(v.x, v.y);
}

template <typename V> __device__ inline const V* a_table(const Desc& D);
template <> __device__ inline const double2* a_table<double2>(const Desc& D) { return D.A64; }
template <> __device__ inline const float2* a_table<float2>(const Desc& D) { return D.A32; }

// Matvec over one work item.  PLAIN: q = L x;  DOT: q = L p, partial Re<p, q>;
// RESID: r = f - L x (FP64), partials |r|^2, |f|^2.  Items with a window stage
// x and |k|^2 of execution rows [w0, w0 + wlen) -- every class their rows
// belong to -- in LDS once, so the gathers never leave the CU.
template <typename NormT, typename V, int MODE>
__device__ void mv_body(const Desc& D, int4 wk, int w, double* part, char* lds) {
  V* As = (V*)lds;
  NormT* nus = (NormT*)(lds + kTab * sizeof(double2));
  double* red = (double*)(lds + kTab * sizeof(double2) + kTab * sizeof(int64_t));
  const int nsl = wk.z & 0xffff, wlen = wk.z >> 16, w0 = wk.w;
  V* xw = (V*)(lds + kLdsFixed);
  NormT* nw = (NormT*)(lds + kLdsFixed + (size_t)wlen * sizeof(V));
  const int tid = threadIdx.x;
  const V* x;
  V* y;
  if (MODE == MV_DOT) {
    x = (const V*)(sizeof(V) == 16 ? (const void*)D.p64 : (const void*)D.p32);
    y = (V*)(sizeof(V) == 16 ? (void*)D.q64 : (void*)D.q32);
  } else if (MODE == MV_RESID) {
    x = (const V*)D.x64;
    y = (V*)D.r64;
  } else {
    x = (const V*)(sizeof(V) == 16 ? (const void*)D.x64 : (const void*)D.x32);
    y = (V*)(sizeof(V) == 16 ? (void*)D.q64 : (void*)D.q32);
  }
  const NormT* normv = (const NormT*)D.norm;
  if (tid < kTab) {
    As[tid] = a_table<V>(D)[tid];
    nus[tid] = (NormT)D.nu[tid];
  }
  {
    // the window, U rows per thread in flight
    constexpr int U = 4;
    for (int i0 = tid; i0 < wlen; i0 += U * kSolveBlock) {
      V xv[U];
      NormT nv[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int i = i0 + u * kSolveBlock;
        if (i < wlen) {
          xv[u] = ld_nt(x + w0 + i);
          nv[u] = __builtin_nontemporal_load(normv + w0 + i);
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int i = i0 + u * kSolveBlock;
        if (i < wlen) {
          xw[i] = xv[u];
          nw[i] = nv[u];
        }
      }
    }
  }
  __syncthreads();
  const int wave = tid >> 6, lane = tid & 63;
  double v0 = 0, v1 = 0;
  for (int sw = wave; sw < nsl; sw += kSolveWaves) {
    const int64_t sl = wk.y + sw;
    const int64_t e = (sl - D.slice0) * kSlice + lane;
    const uint32_t base = D.sptr[sl];
    const uint32_t width = (D.sptr[sl + 1] - base) / kSlice;
    // a window item's own rows lie inside its window (its classes and their padding rows), so the
    // row's |k|^2 comes from the staged copy rather than a second read from HBM
    const V acc = wlen > 0
                      ? sell_row<true, NormT, V>(D.sent, base, width, lane, nw[e - w0], nw, xw, w0, As, nus)
                      : sell_row<false, NormT, V>(D.sent, base, width, lane, normv[e], normv, x, 0, As, nus);
    if (MODE == MV_PLAIN) {
      st_nt(y + e, acc);
    } else if (MODE == MV_DOT) {
      y[e] = acc;
      const V pe = x[e];
      v0 += (double)pe.x * (double)acc.x + (double)pe.y * (double)acc.y;
    } else {
      const double2 fe = D.f64[e];
      V r;
      r.x = fe.x - acc.x;
      r.y = fe.y - acc.y;
      y[e] = r;
      v0 += (double)r.x * r.x + (double)r.y * r.y;
      v1 += fe.x * fe.x + fe.y * fe.y;
    }
  }
  if (MODE != MV_PLAIN) {
    const double s0 = block_sum(v0, red);
    const double s1 = MODE == MV_RESID ? block_sum(v1, red) : 0.0;
    if (tid == 0) {
      part[2 * (int64_t)w] = s0;
      part[2 * (int64_t)w + 1] = s1;
    }
  }
}


// only_final (RESID): 1 = problems being retired only, 0 = admissions and refinement steps only
template <int MODE>
__global__ __launch_bounds__(kSolveBlock) void k_mv(const Desc* __restrict__ descs, const int4* __restrict__ work,
                                               int n_work, int per, double* part, int only_final = 0) {
  const int w = work_index(blockIdx.x, per);
  if (w >= n_work) return;
  const int4 wk = work[w];
  const Desc& D = descs[wk.x];
  if (MODE == MV_DOT) {
    if (cg_idle(D)) return;
    if (w == D.wb && threadIdx.x == 0) {   // iteration index for update/dir (read only by later kernels)
      PState* cs = cg_state(D);
      cs->iter = cs->iters;
    }
  } else if (MODE == MV_RESID) {
    if (only_final) {
      if (!D.final_) return;
    } else {
      const bool outer = D.prec != SS_FP64 ? (!D.ps->done && D.ps_in->done) : false;
      if (!(D.init && D.prec == SS_FP64) && !outer) return;
    }
  }
  extern __shared__ __align__(16) char lds[];
  const bool fp32 = MODE == MV_DOT ? D.prec != SS_FP64 : (MODE == MV_PLAIN && D.prec != SS_FP64);
  if (fp32) {
    if (D.wide) mv_body<int64_t, float2, MODE == MV_RESID ? MV_DOT : MODE>(D, wk, w, part, lds);
    else mv_body<int32_t, float2, MODE == MV_RESID ? MV_DOT : MODE>(D, wk, w, part, lds);
  } else {
    if (D.wide) mv_body<int64_t, double2, MODE>(D, wk, w, part, lds);
    else mv_body<int32_t, double2, MODE>(D, wk, w, part, lds);
  }
}

// alpha = rho / <p,q>;  x += alpha p;  r -= alpha q;  partials <r, D^-1 r>, |r|^2
template <typename NormT, typename V>
__device__ void update_body(const Desc& D, int4 wk, int w, const double* part_pq, double* part_rz, double* red) {
  using R = typename Real<V>::T;
  PState* cs = cg_state(D);
  const double pq = range_sum(part_pq, 0, D.wb, D.we, red);
  const double alpha = cs->rho[cs->iter & 1] / pq;
  if (!(pq > 0.0) || !isfinite(alpha)) {
    if (w == D.wb && threadIdx.x == 0) {
      cs->status = SS_EBREAKDOWN;
      cs->done = 1;
      D.ps->status = SS_EBREAKDOWN;
      D.ps->done = 1;
    }
    return;
  }
  V* x = (V*)(sizeof(V) == 16 ? (void*)D.x64 : (void*)D.x32);
  V* r = (V*)(sizeof(V) == 16 ? (void*)D.r64 : (void*)D.r32);
  const V* pv = (const V*)(sizeof(V) == 16 ? (void*)D.p64 : (void*)D.p32);
  const V* q = (const V*)(sizeof(V) == 16 ? (void*)D.q64 : (void*)D.q32);
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  double v0 = 0, v1 = 0;
  for (int sw = wave; sw < (wk.z & 0xffff); sw += kSolveWaves) {
    const int64_t e = (wk.y + sw - D.slice0) * kSlice + lane;
    const R a = (R)alpha;
    V xv = x[e], rv = r[e];
    const V pe = pv[e], qe = q[e];
    xv.x += a * pe.x;
    xv.y += a * pe.y;
    rv.x -= a * qe.x;
    rv.y -= a * qe.y;
    x[e] = xv;
    r[e] = rv;
    const double rr = (double)rv.x * rv.x + (double)rv.y * rv.y;
    v0 += rr * jacobi_inv(((const NormT*)D.norm)[e], D.a0);
    v1 += rr;
  }
  const double s0 = block_sum(v0, red);
  const double s1 = block_sum(v1, red);
  if (tid == 0) {
    part_rz[2 * (int64_t)w] = s0;
    part_rz[2 * (int64_t)w + 1] = s1;
  }
}

__global__ __launch_bounds__(kSolveBlock) void k_cg_update(const Desc* __restrict__ descs, const int4* __restrict__ work,
                                                      int n_work, int per, const double* part_pq,
                                                      double* part_rz) {
  const int w = work_index(blockIdx.x, per);
  if (w >= n_work) return;
  const int4 wk = work[w];
  const Desc& D = descs[wk.x];
  if (cg_idle(D)) return;
  __shared__ double red[kSolveWaves];
  if (D.prec == SS_FP64) {
    if (D.wide) update_body<int64_t, double2>(D, wk, w, part_pq, part_rz, red);
    else update_body<int32_t, double2>(D, wk, w, part_pq, part_rz, red);
  } else {
    if (D.wide) update_body<int64_t, float2>(D, wk, w, part_pq, part_rz, red);
    else update_body<int32_t, float2>(D, wk, w, part_pq, part_rz, red);
  }
}

// beta = rho'/rho;  stop test;  p = D^-1 r + beta p
template <typename NormT, typename V>
__device__ void dir_body(const Desc& D, int4 wk, int w, const double* part_rz, double* red) {
  using R = typename Real<V>::T;
  PState* cs = cg_state(D);
  const double rz = range_sum(part_rz, 0, D.wb, D.we, red);
  const double rr = range_sum(part_rz, 1, D.wb, D.we, red);
  const int it = cs->iter;
  const double beta = rz / cs->rho[it & 1];
  const double tol2 = D.prec == SS_FP64 ? D.tol2 : cs->tin2;
  const bool conv = rr <= tol2 * cs->ff;
  const bool out_of_iters = it + 1 >= D.max_iter;
  if (w == D.wb && threadIdx.x == 0) {
    cs->rho[(it & 1) ^ 1] = rz;
    cs->rr = rr;
    cs->iters = it + 1;
    if (conv || out_of_iters) {
      cs->done = 1;
      if (!conv) cs->status = SS_ENOCONV;
    }
  }
  if (conv || out_of_iters) return;
  const V* r = (const V*)(sizeof(V) == 16 ? (void*)D.r64 : (void*)D.r32);
  V* pv = (V*)(sizeof(V) == 16 ? (void*)D.p64 : (void*)D.p32);
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  for (int sw = wave; sw < (wk.z & 0xffff); sw += kSolveWaves) {
    const int64_t e = (wk.y + sw - D.slice0) * kSlice + lane;
    const R dinv = (R)jacobi_inv(((const NormT*)D.norm)[e], D.a0);
    const R b = (R)beta;
    const V re = r[e];
    V pe = pv[e];
    pe.x = dinv * re.x + b * pe.x;
    pe.y = dinv * re.y + b * pe.y;
    pv[e] = pe;
  }
}

__global__ __launch_bounds__(kSolveBlock) void k_cg_dir(const Desc* __restrict__ descs, const int4* __restrict__ work,
                                                   int n_work, int per, const double* part_rz) {
  const int w = work_index(blockIdx.x, per);
  if (w >= n_work) return;
  const int4 wk = work[w];
  const Desc& D = descs[wk.x];
  if (cg_idle(D)) return;
  __shared__ double red[kSolveWaves];
  if (D.prec == SS_FP64) {
    if (D.wide) dir_body<int64_t, double2>(D, wk, w, part_rz, red);
    else dir_body<int32_t, double2>(D, wk, w, part_rz, red);
  } else {
    if (D.wide) dir_body<int64_t, float2>(D, wk, w, part_rz, red);
    else dir_body<int32_t, float2>(D, wk, w, part_rz, red);
  }
}

// start of a CG run: p = D^-1 r, partials <r, D^-1 r>, |r|^2
template <typename NormT, typename V>
__device__ void start_body(const Desc& D, int4 wk, int w, double* part_rz, double* red) {
  using R = typename Real<V>::T;
  const V* r = (const V*)(sizeof(V) == 16 ? (void*)D.r64 : (void*)D.r32);
  V* pv = (V*)(sizeof(V) == 16 ? (void*)D.p64 : (void*)D.p32);
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  double v0 = 0, v1 = 0;
  for (int sw = wave; sw < (wk.z & 0xffff); sw += kSolveWaves) {
    const int64_t e = (wk.y + sw - D.slice0) * kSlice + lane;
    const double di = jacobi_inv(((const NormT*)D.norm)[e], D.a0);
    const V re = r[e];
    V pe;
    pe.x = (R)di * re.x;
    pe.y = (R)di * re.y;
    pv[e] = pe;
    const double rr = (double)re.x * re.x + (double)re.y * re.y;
    v0 += rr * di;
    v1 += rr;
  }
  const double s0 = block_sum(v0, red);
  const double s1 = block_sum(v1, red);
  if (tid == 0) {
    part_rz[2 * (int64_t)w] = s0;
    part_rz[2 * (int64_t)w + 1] = s1;
  }
}

__global__ __launch_bounds__(kSolveBlock) void k_cg_start(const Desc* __restrict__ descs, const int4* __restrict__ work,
                                                     int n_work, int per, double* part_rz) {
  const int w = work_index(blockIdx.x, per);
  if (w >= n_work) return;
  const int4 wk = work[w];
  const Desc& D = descs[wk.x];
  if (!cg_state(D)->start) return;
  __shared__ double red[kSolveWaves];
  if (D.prec == SS_FP64) {
    if (D.wide) start_body<int64_t, double2>(D, wk, w, part_rz, red);
    else start_body<int32_t, double2>(D, wk, w, part_rz, red);
  } else {
    if (D.wide) start_body<int64_t, float2>(D, wk, w, part_rz, red);
    else start_body<int32_t, float2>(D, wk, w, part_rz, red);
  }
}

// one block per problem: scalars of a CG run being started
__global__ void k_cg_scalars(const Desc* __restrict__ descs, int n_desc, const double* part_rz) {
  const int p = blockIdx.x;
  if (p >= n_desc) return;
  const Desc& D = descs[p];
  PState* cs = cg_state(D);
  if (!cs->start) return;
  __shared__ double red[kSolveWaves];
  const double rz = range_sum(part_rz, 0, D.wb, D.we, red);
  const double rr = range_sum(part_rz, 1, D.wb, D.we, red);
  if (threadIdx.x == 0) {
    if (D.prec != SS_FP64) {
      D.ps->total_iters += cs->iters;   // previous correction solve
      cs->ff = rr;
      cs->pending = 1;
    }
    cs->rho[0] = rz;
    cs->rr = rr;
    cs->iter = 0;
    cs->iters = 0;
    cs->start = 0;
    cs->status = SS_OK;
    const double tol2 = D.prec == SS_FP64 ? D.tol2 : cs->tin2;
    cs->done = rr <= tol2 * cs->ff ? 1 : 0;
  }
}

// x64 += scale * x32 after a finished correction solve
__global__ __launch_bounds__(kSolveBlock) void k_refine_add(const Desc* __restrict__ descs, const int4* __restrict__ work,
                                                       int n_work, int per) {
  const int w = work_index(blockIdx.x, per);
  if (w >= n_work) return;
  const int4 wk = work[w];
  const Desc& D = descs[wk.x];
  if (D.prec == SS_FP64 || D.ps->done || !D.ps_in->done || !D.ps_in->pending) return;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  for (int sw = wave; sw < (wk.z & 0xffff); sw += kSolveWaves) {
    const int64_t e = (wk.y + sw - D.slice0) * kSlice + lane;
    const double s = D.ps->scale;
    const float2 c = D.x32[e];
    double2 xv = D.x64[e];
    xv.x += s * (double)c.x;
    xv.y += s * (double)c.y;
    D.x64[e] = xv;
  }
}

// One block per problem after an FP64 residual: the outer stop test and the next step.
__global__ void k_outer_scalars(const Desc* __restrict__ descs, int n_desc, const double* part) {
  const int p = blockIdx.x;
  if (p >= n_desc) return;
  const Desc& D = descs[p];
  const bool fp64_init = D.init && D.prec == SS_FP64;
  const bool outer = D.prec != SS_FP64 && !D.ps->done && D.ps_in->done;
  if (!fp64_init && !outer) return;
  __shared__ double red[kSolveWaves];
  const double rr = range_sum(part, 0, D.wb, D.we, red);
  const double ff = range_sum(part, 1, D.wb, D.we, red);
  if (threadIdx.x != 0) return;
  PState* ps = D.ps;
  ps->rr = rr;
  ps->ff = ff;
  const bool conv = rr <= D.tol2 * ff;
  if (fp64_init) {
    if (conv) ps->done = 1;
    else ps->start = 1;
    return;
  }
  D.ps_in->pending = 0;
  if (conv || ps->outer >= kMaxOuter) {
    ps->done = 1;
    if (!conv) ps->status = SS_ENOCONV;
    if (D.ps_in->status == SS_EBREAKDOWN && !conv) ps->status = SS_EBREAKDOWN;
    return;
  }
  ps->scale = sqrt(rr);
  ps->outer += 1;
  D.ps_in->tin2 = fmax(D.tol2_in, kInnerMargin * kInnerMargin * D.tol2 * ff / rr);
  D.ps_in->start = 1;
}

// r32 = r64 / scale, x32 = 0 for a correction solve being started
__global__ __launch_bounds__(kSolveBlock) void k_refine_start(const Desc* __restrict__ descs,
                                                         const int4* __restrict__ work, int n_work, int per) {
  const int w = work_index(blockIdx.x, per);
  if (w >= n_work) return;
  const int4 wk = work[w];
  const Desc& D = descs[wk.x];
  if (D.prec == SS_FP64 || !D.ps_in->start) return;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  for (int sw = wave; sw < (wk.z & 0xffff); sw += kSolveWaves) {
    const int64_t e = (wk.y + sw - D.slice0) * kSlice + lane;
    const double s = 1.0 / D.ps->scale;
    const double2 rv = D.r64[e];
    D.r32[e] = make_float2((float)(rv.x * s), (float)(rv.y * s));
    D.x32[e] = make_float2(0.f, 0.f);
  }
}

// admission: canonical f, u -> execution order (k = 0 and padding rows of x set to 0)
template <typename NormT>
__device__ void admit_rows(const Desc& D, int4 wk) {
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  for (int sw = wave; sw < (wk.z & 0xffff); sw += kSolveWaves) {
    const int64_t e = (wk.y + sw - D.slice0) * kSlice + lane;
    const int64_t r = D.exec2canon[e];
    double2 fv = make_double2(0, 0), xv = make_double2(0, 0);
    if (r >= 0) {
      fv = D.f_canon[r];
      if (((const NormT*)D.norm)[e] > 0) xv = D.u_canon[r];
    }
    D.f64[e] = fv;
    D.x64[e] = xv;
  }
}

__global__ __launch_bounds__(kSolveBlock) void k_admit(const Desc* __restrict__ descs, const int4* __restrict__ work,
                                                  int n_work, int per) {
  const int w = work_index(blockIdx.x, per);
  if (w >= n_work) return;
  const int4 wk = work[w];
  const Desc& D = descs[wk.x];
  if (!D.init) return;
  if (D.wide) admit_rows<int64_t>(D, wk);
  else admit_rows<int32_t>(D, wk);
}

__global__ void k_state_init(const Desc* __restrict__ descs, int n_desc) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n_desc) return;
  const Desc& D = descs[p];
  if (!D.init) return;
  PState s{};
  *D.ps = s;
  s.done = 1;   // no correction solve yet: the first refinement step starts with a residual
  *D.ps_in = s;
}

// retiring: u = x (canonical order), and |f - L x|^2, |f|^2 of the final iterate
template <typename NormT>
__device__ void retire_rows(const Desc& D, int4 wk) {
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  for (int sw = wave; sw < (wk.z & 0xffff); sw += kSolveWaves) {
    const int64_t e = (wk.y + sw - D.slice0) * kSlice + lane;
    const int64_t r = D.exec2canon[e];
    if (r >= 0) D.u_canon[r] = ((const NormT*)D.norm)[e] > 0 ? D.x64[e] : make_double2(0, 0);
  }
}

__global__ __launch_bounds__(kSolveBlock) void k_retire(const Desc* __restrict__ descs, const int4* __restrict__ work,
                                                   int n_work, int per) {
  const int w = work_index(blockIdx.x, per);
  if (w >= n_work) return;
  const int4 wk = work[w];
  const Desc& D = descs[wk.x];
  if (!D.final_) return;
  if (D.wide) retire_rows<int64_t>(D, wk);
  else retire_rows<int32_t>(D, wk);
}

__global__ void k_final_scalars(const Desc* __restrict__ descs, int n_desc, const double* part, PState* out) {
  const int p = blockIdx.x;
  if (p >= n_desc) return;
  const Desc& D = descs[p];
  if (!D.final_) return;
  __shared__ double red[kSolveWaves];
  const double rr = range_sum(part, 0, D.wb, D.we, red);
  const double ff = range_sum(part, 1, D.wb, D.we, red);
  if (threadIdx.x == 0) {
    PState s = *D.ps;
    s.rr = rr;
    s.ff = ff;
    s.total_iters = D.prec == SS_FP64 ? D.ps->iters : D.ps->total_iters + D.ps_in->iters;
    out[p] = s;
  }
}

// compact copy of every problem's FP64/outer state, for host polling
__global__ void k_gather_states(const Desc* __restrict__ descs, int n_desc, PState* out) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < n_desc) out[p] = *descs[p].ps;
}

// ---------------------------------------------------------------- class-resident CG
// A solve unit is a run of whole classes (whole slices, at most kWinRows rows) of one problem.
// Its rows couple to no row outside it (the operator is block diagonal over classes, Sec. 6,
// proof of Prop. SolutionSupport), so one block can run the complete CG -- or the complete
// FP32 + FP64 refinement -- on it: the search direction lives in an LDS window (the matvec
// gathers from there), x, r and f of the block's own rows live in registers, and every inner
// product is a block reduction.  Only the SELL entries come from memory, once per matvec.
// Each unit stops on its own residual, |r_W| <= tol |f_W|, which summed over the problem's units
// gives |r| <= tol |f|; a unit with f_W = 0 has the exact solution u_W = 0.
constexpr int kUnitWaves = 16;                                  // wavefronts per unit block
constexpr int kUnitThreads = kUnitWaves * 64;
constexpr int kUnitSlots = kWinRows / kSlice / kUnitWaves;     // slices per wavefront in a unit

struct UnitOut {
  double rr;       // |f_W - L x_W|^2 of the returned iterate (FP64)
  double ff;       // |f_W|^2
  int32_t iters;   // CG iterations (FP32 + refinement: summed over correction solves)
  int32_t outer;   // refinement steps
  int32_t status;
  int32_t pad;
};

// one problem of a class-resident launch
struct UDesc {
  const uint32_t* sent;          // its operator's SELL entries and slice offsets
  const uint32_t* sptr;
  const void* norm;              // operator execution order (op-global rows)
  const int64_t* exec2canon;     // operator execution row -> operator canonical slot
  const double2* A64;            // the problem's kTab-entry tables
  const float2* A32;
  const int64_t* nu;
  const double2* f;              // request: operator canonical f
  double2* u;                    // request: operator canonical u (in: x0, out: solution)
  double a0;
  double tol2;
  int32_t max_iter;
  int32_t pad;
};

// one launch: units {problem (descriptor index), first slice, slices, first row (problem-local)}
struct UnitArgs {
  const UDesc* descs;
  const int4* ulist;
  const uint2* uent;             // per unit: first SELL entry (operator-global), entries
  int32_t ubase;                 // first unit of this launch within ulist
  int32_t rows;                  // rows of the LDS window and norms: the launch's largest unit
  UnitOut* out;                  // per unit (ulist order)
};

// Dynamic LDS of a unit block: the window (complex128 per row), the rows' |k|^2, then the entry
// cache of the cache mode (`ent_bytes`).  Sized by the launch's largest unit, so a block of small
// units leaves room for more blocks on its CU.
template <typename NormT>
constexpr size_t unit_norm_off(int rows) { return (size_t)rows * 16; }
template <typename NormT>
constexpr size_t unit_ent_off(int rows) { return (unit_norm_off<NormT>(rows) + (size_t)rows * sizeof(NormT) + 15) & ~(size_t)15; }
template <typename NormT>
constexpr size_t unit_lds_bytes(int rows, size_t ent_bytes) { return unit_ent_off<NormT>(rows) + ent_bytes; }

// 64-bit DPP move (the two halves moved alike); lanes of rows outside ROW_MASK get 0
template <int CTRL, int ROW_MASK = 0xf>
__device__ inline double dpp_d(double v) {
  const int lo = __double2loint(v), hi = __double2hiint(v);
  return __hiloint2double(__builtin_amdgcn_update_dpp(0, hi, CTRL, ROW_MASK, 0xf, false),
                          __builtin_amdgcn_update_dpp(0, lo, CTRL, ROW_MASK, 0xf, false));
}

// the value of lane L, as a wave-uniform scalar
template <int L>
__device__ inline double readlane_d(double v) {
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), L),
                          __builtin_amdgcn_readlane(__double2loint(v), L));
}

// Sum within each row of 16 lanes, every lane of the row gets it: pairs, quads, half rows and
// rows by DPP lane moves.
__device__ inline double row_sum_dpp(double v) {
  v += dpp_d<0xb1>(v);    // quad_perm [1,0,3,2]
  v += dpp_d<0x4e>(v);    // quad_perm [2,3,0,1]
  v += dpp_d<0x141>(v);   // row_half_mirror
  v += dpp_d<0x140>(v);   // row_mirror
  return v;
}

// Sum over the wavefront as a scalar: row sums; rows 1 and 3 add the last lane of rows 0 and 2
// (row broadcast 15), then rows 2 and 3 add the last lane of row 1 (row broadcast 31), which
// leaves the total in lane 63.
__device__ inline double wave_sum_dpp(double v) {
  v = row_sum_dpp(v);
  v += dpp_d<0x142, 0xa>(v);
  v += dpp_d<0x143, 0xc>(v);
  return readlane_d<63>(v);
}

// Sum of (a, b) over the block, fixed order, returned to every thread.  red holds the 2 x 16
// wavefront totals.  One barrier: the caller alternates between two such buffers, and a buffer
// is written again only after the barrier of the next reduction, which every thread reaches
// after its reads of this one.  The barrier also orders every LDS access before the call
// against every one after it.
__device__ inline double2 block_sum2(double a, double b, double* red) {
  static_assert(kUnitWaves == 16, "the second stage sums one row of 16 lanes per value");
  a = wave_sum_dpp(a);
  b = wave_sum_dpp(b);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
    red[wave] = a;
    red[kUnitWaves + wave] = b;
  }
  __syncthreads();
  // row 0 sums the totals of a, row 1 those of b
  const double t = row_sum_dpp(lane < 2 * kUnitWaves ? red[lane] : 0.0);
  return make_double2(readlane_d<0>(t), readlane_d<16>(t));
}

// Row of a slice whose entries sit in LDS (base relative to the unit's first entry); the same
// arithmetic as sell_row.
template <typename NormT, typename V>
__device__ inline V sell_row_lds(const uint32_t* ent, uint32_t base, uint32_t width, int lane, NormT nk,
                                 const NormT* normp, const V* xp, int w0, const V* As, const NormT* nus) {
  using R = typename Real<V>::T;
  R ar = 0, ai = 0;
  for (uint32_t q = 0; q < width; ++q) {
    const uint32_t e = ent[base + q * kSlice + lane];
    const uint32_t j = e >> kColBits;
    if (j != (uint32_t)kNullJ) {
      const int c = (int)(e & kColMask) - w0;
      const NormT I = nk + normp[c] - nus[j];
      const V a = As[j];
      const V x = xp[c];
      const R fi = (R)I;
      const R cr = fi * a.x, ci = fi * a.y;
      ar += cr * x.x - ci * x.y;
      ai += cr * x.y + ci * x.x;
    }
  }
  V out;
  out.x = ar;
  out.y = ai;
  return out;
}

// q = L v over the unit's slices owned by this wavefront (v, |k|^2 in the LDS window; with
// CACHED the unit's entries too, sptr holding the slice offsets relative to the unit)
template <typename NormT, typename V, bool CACHED>
__device__ inline void unit_mv(const UDesc& A, const uint32_t* sptr, uint32_t ebase, const uint32_t* ent, int ns,
                               int w0, const V* As, const NormT* nus, const NormT* nw, const V* vw,
                               const NormT* nk, V* acc) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
  for (int k = 0; k < kUnitSlots; ++k) {
    const int sw = wave + k * kUnitWaves;
    if (sw < ns) {
      const uint32_t base = sptr[sw];
      const uint32_t width = (sptr[sw + 1] - base) / kSlice;
      acc[k] = CACHED ? sell_row_lds<NormT, V>(ent, base, width, lane, nk[k], nw, vw, w0, As, nus)
                      : sell_row<true, NormT, V, 24>(A.sent, ebase + base, width, lane, nk[k], nw, vw, w0, As, nus);
    }
  }
}

// FP64 q = L v over the unit from window-local columns and a-table indices kept in LDS (the
// coefficient formed as sell_row forms it); padding entries carry j = kNullJ
template <typename NormT>
__device__ inline void unit_mv_cj(const uint32_t* sptr, const uint16_t* col, const uint8_t* jj, int ns,
                                  const double2* As, const NormT* nus, const NormT* nw, const double2* vw,
                                  const NormT* nk, double2* acc) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
  for (int k = 0; k < kUnitSlots; ++k) {
    const int sw = wave + k * kUnitWaves;
    if (sw < ns) {
      const uint32_t base = sptr[sw];
      const uint32_t width = (sptr[sw + 1] - base) / kSlice;
      double ar = 0, ai = 0;
      for (uint32_t q = 0; q < width; ++q) {
        const uint32_t i = base + q * kSlice + lane;
        const uint32_t j = jj[i];
        if (j != (uint32_t)kNullJ) {
          const int c = col[i];
          const NormT I = nk[k] + nw[c] - nus[j];
          const double2 a = As[j];
          const double2 x = vw[c];
          const double fi = (double)I;
          const double cr = fi * a.x, ci = fi * a.y;
          ar += cr * x.x - ci * x.y;
          ai += cr * x.y + ci * x.x;
        }
      }
      acc[k] = make_double2(ar, ai);
    }
  }
}

// FP32 q = L v from per-entry integer brackets (as FP32), window-local columns and a-table
// indices kept in LDS; the coefficient fi * a_j is formed as sell_row forms it (padding entries
// hold fi = 0, column 0 and the null index, whose table entry is 0)
__device__ inline void unit_mv_coef(const uint32_t* sptr, const float* fiv, const uint16_t* col, const uint8_t* jj,
                                    int ns, const float2* As, const float2* vw, float2* acc) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
  for (int k = 0; k < kUnitSlots; ++k) {
    const int sw = wave + k * kUnitWaves;
    if (sw < ns) {
      const uint32_t base = sptr[sw];
      const uint32_t width = (sptr[sw + 1] - base) / kSlice;
      float ar = 0, ai = 0;
      uint32_t i = base + lane;
      uint32_t q = 0;
      for (; q + 4 <= width; q += 4, i += 4 * kSlice) {
        float fi[4];
        float2 a[4], x[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          fi[u] = fiv[i + u * kSlice];
          a[u] = As[jj[i + u * kSlice]];
          x[u] = vw[col[i + u * kSlice]];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const float cr = fi[u] * a[u].x, ci = fi[u] * a[u].y;
          ar += cr * x[u].x - ci * x[u].y;
          ai += cr * x[u].y + ci * x[u].x;
        }
      }
      for (; q < width; ++q, i += kSlice) {
        const float f = fiv[i];
        const float2 a = As[jj[i]], x = vw[col[i]];
        const float cr = f * a.x, ci = f * a.y;
        ar += cr * x.x - ci * x.y;
        ai += cr * x.y + ci * x.x;
      }
      acc[k] = make_float2(ar, ai);
    }
  }
}

// FP32 q = L v from per-entry complex FP32 coefficients (the bracket times the a-table entry,
// rounded as unit_mv_coef rounds it) and window-local columns kept in LDS; padding entries hold
// a zero coefficient and column 0
__device__ inline void unit_mv_cplx(const uint32_t* sptr, const float2* cf, const uint16_t* col, int ns,
                                    const float2* vw, float2* acc) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
  for (int k = 0; k < kUnitSlots; ++k) {
    const int sw = wave + k * kUnitWaves;
    if (sw < ns) {
      const uint32_t base = sptr[sw];
      const uint32_t width = (sptr[sw + 1] - base) / kSlice;
      float ar = 0, ai = 0;
      uint32_t i = base + lane;
      uint32_t q = 0;
      for (; q + 4 <= width; q += 4, i += 4 * kSlice) {
        float2 c[4], x[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          c[u] = cf[i + u * kSlice];
          x[u] = vw[col[i + u * kSlice]];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          ar += c[u].x * x[u].x - c[u].y * x[u].y;
          ai += c[u].x * x[u].y + c[u].y * x[u].x;
        }
      }
      for (; q < width; ++q, i += kSlice) {
        const float2 c = cf[i], x = vw[col[i]];
        ar += c.x * x.x - c.y * x.y;
        ai += c.x * x.y + c.y * x.x;
      }
      acc[k] = make_float2(ar, ai);
    }
  }
}

// Where the matvecs find the operator: CM_STREAM reads the SELL entries from memory each time;
// CM_ENTRIES keeps the unit's entries in LDS.  FP32 + refinement: CM_COEF keeps per-entry FP32
// brackets, window-local columns and a-table indices in LDS, CM_CPLX (units small enough) the
// complex FP32 coefficients in place of the brackets; the correction solves use the brackets or
// coefficients and the columns, the FP64 residuals the columns and indices.
enum { CM_STREAM = 0, CM_ENTRIES = 1, CM_COEF = 2, CM_CPLX = 3 };
// entries each cache may hold (the set-up stages them through registers; int32 / int64 norms); a
// unit's mode is then chosen at run time by the LDS its window, norms and cache take together
constexpr int kCoefBytes = 7;    // FP32 bracket, 16-bit column, 8-bit a-table index
constexpr int kCplxBytes = 11;   // complex FP32 coefficient, 16-bit column, 8-bit a-table index
constexpr int kCoefEntries32 = 17152;
constexpr int kCoefEntries64 = 15936;
constexpr int kCplxEntries = 10944;
static_assert(kUnitEntries <= kCoefEntries64 && kCoefEntries64 <= kCoefEntries32, "units must fit every cache");
static_assert(kCplxEntries <= kCoefEntries64, "the group map covers every cache");

// TWO: built for two blocks per CU (at most 64 VGPRs: eight wavefronts per SIMD), launched for
// units whose LDS leaves room for a second block; otherwise one block per CU.  The solve is
// latency-bound (barriers, dependent LDS gathers), so a second unit on the CU hides it.
template <typename NormT, bool FP64, int CM, bool TWO>
__global__ __launch_bounds__(kUnitThreads, TWO ? 8 : 4) void k_unit_solve(UnitArgs Args) {
  constexpr bool CACHED = CM == CM_ENTRIES;
  extern __shared__ __align__(16) unsigned char s_dyn[];
  double2* s_win = reinterpret_cast<double2*>(s_dyn);                                   // search direction / iterate window
  NormT* s_norm = reinterpret_cast<NormT*>(s_dyn + unit_norm_off<NormT>(Args.rows));     // |k|^2 of the rows
  uint32_t* s_ent = reinterpret_cast<uint32_t*>(s_dyn + unit_ent_off<NormT>(Args.rows)); // CM_ENTRIES: entries; CM_COEF, CM_CPLX: brackets or coefficients, columns, j
  __shared__ uint32_t s_sptr[kWinRows / kSlice + 1];
  __shared__ double2 s_A64[kTab];
  __shared__ float2 s_A32[kTab];
  __shared__ NormT s_nu[kTab];
  __shared__ double s_red[2][2 * kUnitWaves];   // reductions alternate between the two
  int rsel = 0;
  auto red_next = [&]() -> double* { rsel ^= 1; return s_red[rsel]; };
  float2* s_win32 = reinterpret_cast<float2*>(s_win);
  const int ui = Args.ubase + blockIdx.x;
  const int4 un = Args.ulist[ui];
  const uint2 ue = Args.uent[ui];
  const UDesc& A = Args.descs[un.x];
  const int s0 = un.y, ns = un.z, w0 = un.w;
  const uint32_t ebase = ue.x, n_ent = ue.y;
  const int64_t E0 = (int64_t)s0 * kSlice;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const NormT* normg = (const NormT*)A.norm;
  const double a0 = A.a0;
  const double tol2_in = kInnerTol * kInnerTol;
  // Set-up.  Every load whose address is known at the start is issued first, together: the own
  // rows' |k|^2 and canonical slots, the unit's entries, the tables and the slice offsets; the
  // own rows' f and x0 follow once the slots arrive.  The own rows (slice wave + k * kUnitWaves,
  // lane) are window rows tid + k * kUnitThreads, so their |k|^2 also fill the LDS norms.
  NormT nk[kUnitSlots];
  double dinv[kUnitSlots];
  int32_t cr[kUnitSlots];   // canonical slot (rows of a batch are below 2^31), -1 for padding
  double2 x[kUnitSlots], r[kUnitSlots], fv[kUnitSlots];
#pragma unroll
  for (int k = 0; k < kUnitSlots; ++k) {
    nk[k] = 0;
    cr[k] = -1;
    if (wave + k * kUnitWaves < ns) {
      const int64_t e = E0 + tid + k * kUnitThreads;
      nk[k] = normg[e];
      cr[k] = (int32_t)A.exec2canon[e];
    }
  }
  constexpr int kCap = CM == CM_COEF   ? (sizeof(NormT) == 8 ? kCoefEntries64 : kCoefEntries32)
                      : CM == CM_CPLX ? kCplxEntries
                                      : kUnitEntries;
  constexpr int kStage = CM == CM_STREAM ? 1 : (kCap + kUnitThreads - 1) / kUnitThreads;
  uint32_t v[kStage];
  if (CM != CM_STREAM) {
#pragma unroll
    for (int u = 0; u < kStage; ++u) {
      const uint32_t i = tid + u * kUnitThreads;
      v[u] = i < n_ent ? A.sent[ebase + i] : 0u;
    }
  }
  double2 tA64 = make_double2(0, 0);
  float2 tA32 = make_float2(0.f, 0.f);
  NormT tnu = 0;
  uint32_t tsp = 0;
  if (tid < kTab) {
    tA64 = A.A64[tid];
    tA32 = A.A32[tid];
    tnu = (NormT)A.nu[tid];
  }
  if (tid <= ns) tsp = A.sptr[s0 + tid] - ebase;   // ns <= 32: wavefront 0 only
#pragma unroll
  for (int k = 0; k < kUnitSlots; ++k) {
    fv[k] = x[k] = make_double2(0, 0);
    if (cr[k] >= 0) {
      fv[k] = A.f[cr[k]];
      if (nk[k] > 0) x[k] = A.u[cr[k]];
    }
  }
#pragma unroll
  for (int k = 0; k < kUnitSlots; ++k)
    if (wave + k * kUnitWaves < ns) s_norm[tid + k * kUnitThreads] = nk[k];
  if (tid < kTab) {
    s_A64[tid] = tA64;
    s_A32[tid] = tA32;
    s_nu[tid] = tnu;
  }
  if (tid <= ns) s_sptr[tid] = tsp;
  constexpr bool kCoefs = CM == CM_COEF || CM == CM_CPLX;
  float* s_fi = reinterpret_cast<float*>(s_ent);     // CM_COEF
  float2* s_cf = reinterpret_cast<float2*>(s_ent);   // CM_CPLX
  uint16_t* s_col = CM == CM_CPLX ? reinterpret_cast<uint16_t*>(s_cf + n_ent) : reinterpret_cast<uint16_t*>(s_fi + n_ent);
  uint8_t* s_j = reinterpret_cast<uint8_t*>(s_col + n_ent);
  // CM_COEF, CM_CPLX: the slice of every group of 64 entries (a slice's entries are whole groups)
  __shared__ uint8_t s_gslice[kCoefEntries32 / kSlice + 1];
  if (kCoefs && wave == 0) {
    const uint32_t next = __shfl_down(tsp, 1, 64);
    if (lane < ns)
      for (uint32_t g = tsp / kSlice; g < next / kSlice; ++g) s_gslice[g] = (uint8_t)lane;
  }
  if (CM == CM_ENTRIES) {
#pragma unroll
    for (int u = 0; u < kStage; ++u) {
      const uint32_t i = tid + u * kUnitThreads;
      if (i < n_ent) s_ent[i] = v[u];
    }
  } else if (kCoefs) {
    // each entry's FP32 bracket |k|^2 + |l|^2 - |w_j|^2 (CM_CPLX: times the FP32 a-table entry,
    // both formed as the on-the-fly FP32 matvec forms them), its window-local column and its
    // a-table index; entry (q, lane) of a slice sits at slice base + q * 64 + lane, so entry i
    // is in the row of lane i % 64 of slice s_gslice[i / 64]
    __syncthreads();   // norms, |w|^2, tables and the group map staged
#pragma unroll
    for (int u = 0; u < kStage; ++u) {
      const uint32_t i = tid + u * kUnitThreads;
      if (i < n_ent) {
        const uint32_t j = v[u] >> kColBits;
        float fi = 0.f;
        uint16_t c = 0;
        if (j != (uint32_t)kNullJ) {
          const NormT nkr = s_norm[s_gslice[i / kSlice] * kSlice + lane];
          c = (uint16_t)((int)(v[u] & kColMask) - w0);
          fi = (float)(nkr + s_norm[c] - s_nu[j]);
        }
        if (CM == CM_CPLX) {
          const float2 a = j != (uint32_t)kNullJ ? s_A32[j] : make_float2(0.f, 0.f);
          s_cf[i] = make_float2(fi * a.x, fi * a.y);
        } else {
          s_fi[i] = fi;
        }
        s_col[i] = c;
        s_j[i] = (uint8_t)j;
      }
    }
  }
  int nzx = 0;
  double vff = 0;
#pragma unroll
  for (int k = 0; k < kUnitSlots; ++k) {
    vff += fv[k].x * fv[k].x + fv[k].y * fv[k].y;
    nzx |= (x[k].x != 0.0 || x[k].y != 0.0);
    dinv[k] = jacobi_inv(nk[k], a0);
  }
  const double2 init = block_sum2(vff, (double)nzx, red_next());   // also orders the LDS staging above
  const double ff = init.x;
  const bool warm = init.y > 0;
  const double thr2 = A.tol2 * ff;   // |r_W| <= tol |f_W|; summed over units: |r| <= tol |f|
  int status = SS_OK, iters = 0, outer = 0;
  double rr;
  if (ff == 0) {   // the unit's classes decouple from the rest: f_W = 0 gives u_W = 0 exactly
#pragma unroll
    for (int k = 0; k < kUnitSlots; ++k) x[k] = make_double2(0, 0);
    rr = 0;
  }

  // r = f - L x (FP64), |r|^2
  double rzr = 0;   // <r, D^-1 r> of the last residual, reduced with |r|^2
  auto residual = [&]() -> double {
    double v = 0, vz = 0;
    if (warm || outer > 0) {
#pragma unroll
      for (int k = 0; k < kUnitSlots; ++k)
        if (wave + k * kUnitWaves < ns) s_win[(wave + k * kUnitWaves) * kSlice + lane] = x[k];
      __syncthreads();
      double2 acc[kUnitSlots];
      if (kCoefs)
        unit_mv_cj<NormT>(s_sptr, s_col, s_j, ns, s_A64, s_nu, s_norm, s_win, nk, acc);
      else
        unit_mv<NormT, double2, CACHED>(A, s_sptr, ebase, s_ent, ns, w0, s_A64, s_nu, s_norm, s_win, nk, acc);
#pragma unroll
      for (int k = 0; k < kUnitSlots; ++k) {
        const double2 fk = fv[k];
        r[k] = wave + k * kUnitWaves < ns ? make_double2(fk.x - acc[k].x, fk.y - acc[k].y) : make_double2(0, 0);
      }
    } else {
#pragma unroll
      for (int k = 0; k < kUnitSlots; ++k) r[k] = fv[k];
    }
#pragma unroll
    for (int k = 0; k < kUnitSlots; ++k) {
      const double t = r[k].x * r[k].x + r[k].y * r[k].y;
      v += t;
      vz += t * dinv[k];
    }
    const double2 sv = block_sum2(v, vz, red_next());   // its barrier also ends every read of the window
    rzr = sv.y;
    return sv.x;
  };

  if (ff == 0) {
  } else if (FP64) {
    rr = residual();
    if (rr > thr2) {
      double2 pv[kUnitSlots];
#pragma unroll
      for (int k = 0; k < kUnitSlots; ++k) {
        pv[k] = make_double2(dinv[k] * r[k].x, dinv[k] * r[k].y);
        if (wave + k * kUnitWaves < ns) s_win[(wave + k * kUnitWaves) * kSlice + lane] = pv[k];
      }
      __syncthreads();
      double rho = rzr;   // <r, D^-1 r>, reduced with |r|^2
      while (true) {
        double2 q[kUnitSlots];
        unit_mv<NormT, double2, CACHED>(A, s_sptr, ebase, s_ent, ns, w0, s_A64, s_nu, s_norm, s_win, nk, q);
        double vpq = 0;
#pragma unroll
        for (int k = 0; k < kUnitSlots; ++k)
          if (wave + k * kUnitWaves < ns) vpq += pv[k].x * q[k].x + pv[k].y * q[k].y;
        const double pq = block_sum2(vpq, 0.0, red_next()).x;
        const double alpha = rho / pq;
        if (!(pq > 0.0) || !isfinite(alpha)) {
          status = SS_EBREAKDOWN;
          break;
        }
        double v0 = 0, v1 = 0;
#pragma unroll
        for (int k = 0; k < kUnitSlots; ++k) {
          if (wave + k * kUnitWaves < ns) {
            x[k].x += alpha * pv[k].x;
            x[k].y += alpha * pv[k].y;
            r[k].x -= alpha * q[k].x;
            r[k].y -= alpha * q[k].y;
          }
          const double t = r[k].x * r[k].x + r[k].y * r[k].y;
          v0 += t * dinv[k];
          v1 += t;
        }
        const double2 s2 = block_sum2(v0, v1, red_next());
        ++iters;
        rr = s2.y;
        if (rr <= thr2) break;
        if (iters >= A.max_iter) {
          status = SS_ENOCONV;
          break;
        }
        const double beta = s2.x / rho;
        rho = s2.x;
#pragma unroll
        for (int k = 0; k < kUnitSlots; ++k) {
          pv[k] = make_double2(dinv[k] * r[k].x + beta * pv[k].x, dinv[k] * r[k].y + beta * pv[k].y);
          if (wave + k * kUnitWaves < ns) s_win[(wave + k * kUnitWaves) * kSlice + lane] = pv[k];
        }
        __syncthreads();
      }
      // the true residual of the returned iterate
      outer = 1;   // makes residual() run the matvec
      rr = residual();
      outer = 0;
    }
  } else {
    bool broke = false;
    while (true) {
      rr = residual();
      if (rr <= thr2) break;
      if (outer >= kMaxOuter) {
        status = broke ? SS_EBREAKDOWN : SS_ENOCONV;
        break;
      }
      const double scale = sqrt(rr), inv = 1.0 / scale;
      const double tin2 = fmax(tol2_in, kInnerMargin * kInnerMargin * thr2 / rr);
      ++outer;
      // correction solve L d = r / |r| in FP32 (FP64 inner products), d = 0 to start
      // its starting scalars are those of the FP64 residual, scaled (no further reduction)
      float2 r32[kUnitSlots], p32[kUnitSlots], d32[kUnitSlots];
#pragma unroll
      for (int k = 0; k < kUnitSlots; ++k) {
        r32[k] = make_float2((float)(r[k].x * inv), (float)(r[k].y * inv));
        d32[k] = make_float2(0.f, 0.f);
        const float di = (float)dinv[k];
        p32[k] = make_float2(di * r32[k].x, di * r32[k].y);
        if (wave + k * kUnitWaves < ns) s_win32[(wave + k * kUnitWaves) * kSlice + lane] = p32[k];
      }
      __syncthreads();
      double rho = rzr * inv * inv;
      const double ff_in = 1.0;
      int it = 0;
      {
        while (true) {
          float2 q[kUnitSlots];
          if (CM == CM_CPLX)
            unit_mv_cplx(s_sptr, s_cf, s_col, ns, s_win32, q);
          else if (CM == CM_COEF)
            unit_mv_coef(s_sptr, s_fi, s_col, s_j, ns, s_A32, s_win32, q);
          else
            unit_mv<NormT, float2, CACHED>(A, s_sptr, ebase, s_ent, ns, w0, s_A32, s_nu, s_norm, s_win32, nk, q);
          double vpq = 0;
#pragma unroll
          for (int k = 0; k < kUnitSlots; ++k)
            if (wave + k * kUnitWaves < ns) vpq += (double)p32[k].x * q[k].x + (double)p32[k].y * q[k].y;
          const double pq = block_sum2(vpq, 0.0, red_next()).x;
          const double alpha = rho / pq;
          if (!(pq > 0.0) || !isfinite(alpha)) {
            broke = true;
            break;
          }
          const float a = (float)alpha;
          double v0 = 0, v1 = 0;
#pragma unroll
          for (int k = 0; k < kUnitSlots; ++k) {
            if (wave + k * kUnitWaves < ns) {
              d32[k].x += a * p32[k].x;
              d32[k].y += a * p32[k].y;
              r32[k].x -= a * q[k].x;
              r32[k].y -= a * q[k].y;
            }
            const double t = (double)r32[k].x * r32[k].x + (double)r32[k].y * r32[k].y;
            v0 += t * dinv[k];
            v1 += t;
          }
          const double2 s2 = block_sum2(v0, v1, red_next());
          ++it;
          if (s2.y <= tin2 * ff_in || it >= A.max_iter) break;
          const float b = (float)(s2.x / rho);
          rho = s2.x;
#pragma unroll
          for (int k = 0; k < kUnitSlots; ++k) {
            const float di = (float)dinv[k];
            p32[k] = make_float2(di * r32[k].x + b * p32[k].x, di * r32[k].y + b * p32[k].y);
            if (wave + k * kUnitWaves < ns) s_win32[(wave + k * kUnitWaves) * kSlice + lane] = p32[k];
          }
          __syncthreads();
        }
      }
      iters += it;
#pragma unroll
      for (int k = 0; k < kUnitSlots; ++k) {
        x[k].x += scale * (double)d32[k].x;
        x[k].y += scale * (double)d32[k].y;
      }
      __syncthreads();   // every read of the FP32 window is done before residual() overwrites it
    }
  }
#pragma unroll
  for (int k = 0; k < kUnitSlots; ++k)
    if (cr[k] >= 0) A.u[cr[k]] = nk[k] > 0 ? x[k] : make_double2(0, 0);
  if (tid == 0) {
    UnitOut o;
    o.rr = rr;
    o.ff = ff;
    o.iters = iters;
    o.outer = outer;
    o.status = status;
    o.pad = 0;
    Args.out[ui] = o;
  }
}

// one thread per problem: the problem's residual and counters from its units, in order
struct UnitSum {
  double rr, ff;
  int32_t iters, outer, status, pad;
};

__global__ void k_unit_final(int n_prob, const int32_t* __restrict__ uoff, const int32_t* __restrict__ uidx,
                             const UnitOut* __restrict__ uo, UnitSum* out) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n_prob) return;
  UnitSum s{0.0, 0.0, 0, 0, SS_OK, 0};
  for (int k = uoff[q]; k < uoff[q + 1]; ++k) {
    const UnitOut& o = uo[uidx[k]];
    s.rr += o.rr;
    s.ff += o.ff;
    s.iters = max(s.iters, o.iters);
    s.outer = max(s.outer, o.outer);
    if (o.status == SS_EBREAKDOWN || (o.status == SS_ENOCONV && s.status == SS_OK)) s.status = o.status;
  }
  out[q] = s;
}

inline unsigned grid_for(int64_t n) { return (unsigned)std::max<int64_t>(1, ceil_div(n, kBlock)); }

// LDS a unit block may take beside the kernel's static arrays: all a block can have, and the share
// that leaves room for a second block on the CU (0 if the device cannot be queried: units then
// stream their entries)
struct UnitLds {
  int full = 0, half = 0;
};
template <typename NormT>
UnitLds unit_lds() {
  static const UnitLds v = [] {
    UnitLds r;
    int dev = 0, lds = 0;
    hipFuncAttributes fa{};
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess ||
        hipFuncGetAttributes(&fa, reinterpret_cast<const void*>(&k_unit_solve<NormT, false, CM_CPLX, false>)) != hipSuccess) {
      (void)hipGetLastError();   // not left for the launch checks that follow
      return r;
    }
    r.full = std::max(0, lds - (int)fa.sharedSizeBytes);
    r.half = std::max(0, lds / 2 - (int)fa.sharedSizeBytes);
    return r;
  }();
  return v;
}

// The cache mode of a unit of `rows` rows and `ne` entries, its dynamic LDS and whether two such
// blocks share a CU: the richest cache that lets two blocks share it, else the richest that fits
// at all, else streaming (FP64: entries or streaming; FP32 + refinement: complex coefficients,
// brackets, entries)
template <typename NormT>
int unit_mode(bool fp32, int rows, int ne, size_t* lds, bool* two) {
  const UnitLds L = unit_lds<NormT>();
  struct Cand {
    int mode, bytes, cap;
  };
  const Cand c64[] = {{CM_ENTRIES, 4, kUnitEntries}};
  const Cand c32[] = {{CM_CPLX, kCplxBytes, kCplxEntries},
                      {CM_COEF, kCoefBytes, sizeof(NormT) == 8 ? kCoefEntries64 : kCoefEntries32},
                      {CM_ENTRIES, 4, kUnitEntries}};
  const Cand* cs = fp32 ? c32 : c64;
  const int nc = fp32 ? 3 : 1;
  for (int budget : {L.half, L.full})
    for (int i = 0; i < nc; ++i) {
      const size_t need = unit_lds_bytes<NormT>(rows, (size_t)ne * cs[i].bytes);
      if (ne <= cs[i].cap && need <= (size_t)budget) {
        *lds = need;
        *two = budget == L.half;
        return cs[i].mode;
      }
    }
  *lds = unit_lds_bytes<NormT>(rows, 0);
  *two = *lds <= (size_t)L.half;
  return CM_STREAM;
}

}  // namespace

// ---------------------------------------------------------------- launch lists
// A set of problems (descriptors) with their work items, device-resident.
struct LaunchList {
  std::vector<Desc> descs;
  std::vector<int4> work;
  Desc* d_descs = nullptr;
  int4* d_work = nullptr;
  double* part = nullptr;          // 3 x 2 x n_work
  PState* d_states = nullptr;      // n_desc (polling / final)
  size_t cap_desc = 0, cap_work = 0;
  int per = 1;
  unsigned grid = 8;
  size_t lds_resid = 0, lds_dot = 0;   // dynamic LDS of the FP64-residual and CG / plain matvecs

  ~LaunchList() {
    dfree(d_descs);
    dfree(d_work);
    dfree(part);
    dfree(d_states);
  }

  // rebuild work items from descs (each desc's items contiguous) and upload both
  ss_status upload(hipStream_t s, const std::vector<std::vector<int4>>& items) {
    work.clear();
    for (size_t k = 0; k < descs.size(); ++k) {
      descs[k].wb = (int32_t)work.size();
      for (int4 it : items[k]) work.push_back(make_int4((int)k, it.y, it.z, it.w));
      descs[k].we = (int32_t)work.size();
    }
    if (descs.size() > cap_desc) {
      dfree(d_descs);
      dfree(d_states);
      cap_desc = std::max<size_t>(descs.size(), 2 * cap_desc);
      SS_TRY(dalloc(&d_descs, cap_desc));
      SS_TRY(dalloc(&d_states, cap_desc));
    }
    if (work.size() > cap_work) {
      dfree(d_work);
      dfree(part);
      cap_work = std::max<size_t>(work.size(), 2 * cap_work);
      SS_TRY(dalloc(&d_work, cap_work));
      SS_TRY(dalloc(&part, 6 * cap_work));
    }
    if (!descs.empty())
      SS_HIP(h2d(d_descs, descs.data(), descs.size() * sizeof(Desc), s));
    if (!work.empty())
      SS_HIP(h2d(d_work, work.data(), work.size() * sizeof(int4), s));
    per = (int)std::max<int64_t>(1, ceil_div((int64_t)work.size(), 8));
    grid = (unsigned)(8 * per);
    int64_t maxw = 0;
    bool any64 = false, wide = false;
    for (const int4& it : work) maxw = std::max<int64_t>(maxw, it.z >> 16);
    for (const Desc& D : descs) {
      any64 |= D.prec == SS_FP64;
      wide |= D.wide != 0;
    }
    lds_resid = mv_lds_bytes(maxw, true, wide);
    lds_dot = mv_lds_bytes(maxw, any64, wide);
    return SS_OK;
  }
  ss_status upload_descs(hipStream_t s) {
    if (!descs.empty())
      SS_HIP(h2d(d_descs, descs.data(), descs.size() * sizeof(Desc), s));
    return SS_OK;
  }
  int n_work() const { return (int)work.size(); }
  int n_desc() const { return (int)descs.size(); }
  double* part_a() { return part; }
  double* part_b() { return part + 2 * cap_work; }
  double* part_c() { return part + 4 * cap_work; }
};

namespace {

// ---------------------------------------------------------------- operator workspace
struct WS {
  double2 *x64, *r64, *p64, *q64, *f64;
  float2 *x32, *r32, *p32, *q32;
  PState *ps, *ps_in;
};

size_t al256(size_t b) { return (b + 255) & ~size_t(255); }

size_t workspace_bytes(const OpImpl* op) {
  const int64_t n = op->n_exec;
  return al256(5 * n * sizeof(double2)) + al256(4 * n * sizeof(float2)) + al256(2 * op->n_prob * sizeof(PState));
}

ss_status workspace(OpImpl* op, WS* w) {
  const int64_t n = op->n_exec;
  const size_t need = workspace_bytes(op);
  if (op->ws.bytes < need) {
    if (op->ws.base) pool_free(op->ws.base);
    op->ws.base = nullptr;
    op->ws.bytes = 0;
    SS_HIP(pool_alloc((void**)&op->ws.base, need));
    op->ws.bytes = need;
  }
  char* b = (char*)op->ws.base;
  w->x64 = (double2*)b;
  w->r64 = w->x64 + n;
  w->p64 = w->r64 + n;
  w->q64 = w->p64 + n;
  w->f64 = w->q64 + n;
  b += al256(5 * n * sizeof(double2));
  w->x32 = (float2*)b;
  w->r32 = w->x32 + n;
  w->p32 = w->r32 + n;
  w->q32 = w->p32 + n;
  b += al256(4 * n * sizeof(float2));
  w->ps = (PState*)b;
  w->ps_in = w->ps + op->n_prob;
  return SS_OK;
}

// descriptor of problem p of op, vectors from the op's workspace
Desc make_desc(const OpImpl* op, const WS& w, int p) {
  Desc D{};
  const int64_t e0 = op->eoff[p];
  D.sent = op->d_sent;
  D.sptr = op->d_sptr;
  D.norm = (const char*)op->d_norm + e0 * (op->wide_norm ? 8 : 4);
  D.A64 = op->d_A64 + (size_t)p * kTab;
  D.A32 = op->d_A32 + (size_t)p * kTab;
  D.nu = op->d_nu + (size_t)p * kTab;
  D.exec2canon = op->d_exec2canon + e0;
  D.x64 = w.x64 + e0;
  D.r64 = w.r64 + e0;
  D.p64 = w.p64 + e0;
  D.q64 = w.q64 + e0;
  D.f64 = w.f64 + e0;
  D.x32 = w.x32 + e0;
  D.r32 = w.r32 + e0;
  D.p32 = w.p32 + e0;
  D.q32 = w.q32 + e0;
  D.ps = w.ps + p;
  D.ps_in = w.ps_in + p;
  D.a0 = op->a0_host[p];
  D.slice0 = e0 / kSlice;
  D.n_rows = op->eoff[p + 1] - e0;
  D.wide = op->wide_norm ? 1 : 0;
  return D;
}

std::vector<int4> items_of(const OpImpl* op, int p) {
  return std::vector<int4>(op->work.begin() + op->wrange[p].x, op->work.begin() + op->wrange[p].y);
}

}  // namespace

// ---------------------------------------------------------------- engine
// One problem of a class-resident launch, as gathered before the launch.
struct UnitItem {
  UDesc d;
  OpImpl* op;
  int prob;
  int req;
  int group;       // wide * 2 + fp32
  int prec;
};

inline UnitItem unit_item(OpImpl* op, int p, const void* f, void* u, double tol, ss_precision prec,
                          int32_t max_iter, int req) {
  UDesc D{};
  D.sent = op->d_sent;
  D.sptr = op->d_sptr;
  D.norm = op->d_norm;
  D.exec2canon = op->d_exec2canon;
  D.A64 = op->d_A64 + (size_t)p * kTab;
  D.A32 = op->d_A32 + (size_t)p * kTab;
  D.nu = op->d_nu + (size_t)p * kTab;
  D.f = (const double2*)f;
  D.u = (double2*)u;
  D.a0 = op->a0_host[p];
  D.tol2 = tol * tol;
  D.max_iter = max_iter;
  return UnitItem{D, op, p, req, (op->wide_norm ? 2 : 0) + (prec != SS_FP64 ? 1 : 0), (int)prec};
}

// Host tables of one class-resident launch.  Units are sorted into launches by (norm width,
// precision, what the LDS caches); a unit's result is addressed by its position in ul, and each
// problem's are summed in order through uidx.
struct UnitPlan {
  static constexpr int kGroups = 24;   // blocks per CU (1, 2) x norm width x (FP64: stream, entries in LDS | FP32: stream,
                                       // entries, brackets, complex coefficients in LDS)
  std::vector<UDesc> descs;            // per problem
  std::vector<int4> ul;                // per unit: {problem, first slice, slices, first row}
  std::vector<uint2> ue;               // per unit: first SELL entry, entries
  std::vector<int32_t> uoff;           // [problems + 1] into uidx
  std::vector<int32_t> uidx;           // per unit of each problem, in order: its position in ul
  int gbeg[kGroups + 1] = {0};
  int32_t lmax[kGroups] = {0};         // dynamic LDS of each launch
  int32_t rmax[kGroups] = {0};         // rows of the largest unit of each launch

  int n_prob() const { return (int)descs.size(); }
  int n_units() const { return (int)ul.size(); }

  void make(const std::vector<UnitItem>& launched) {
    const int np = (int)launched.size();
    descs.assign(np, UDesc{});
    std::vector<int4> lists[kGroups];
    std::vector<uint2> ents[kGroups];
    std::vector<std::pair<int, int>> where;   // per unit of each problem, in order: (launch, index)
    uoff.assign(1, 0);
    for (int g = 0; g < kGroups; ++g) lmax[g] = rmax[g] = 0;
    for (int i = 0; i < np; ++i) {
      const UnitItem& it = launched[i];
      descs[i] = it.d;
      const int2 ur = it.op->urange[it.prob];
      for (int k = ur.x; k < ur.y; ++k) {
        const int4 un = it.op->units[k];
        const int32_t ne = it.op->unit_entries[k];
        const bool wide = it.group >= 2, fp32 = it.group & 1;
        const int rows = un.z * kSlice;
        size_t lds = 0;
        bool two = false;
        const int mode = wide ? unit_mode<int64_t>(fp32, rows, ne, &lds, &two)
                              : unit_mode<int32_t>(fp32, rows, ne, &lds, &two);
        const int g = (two ? 12 : 0) + (wide ? 6 : 0) + (fp32 ? 2 : 0) + mode;
        where.emplace_back(g, (int)lists[g].size());
        lists[g].push_back(make_int4(i, un.y, un.z, un.w));
        ents[g].push_back(make_uint2(it.op->unit_ebase[k], (uint32_t)ne));
        const int bytes = mode == CM_CPLX ? kCplxBytes : mode == CM_COEF ? kCoefBytes : 4;
        if (mode != CM_STREAM) lmax[g] = std::max(lmax[g], ne * bytes);
        rmax[g] = std::max(rmax[g], rows);
      }
      uoff.push_back((int32_t)where.size());
    }
    ul.clear();
    ue.clear();
    gbeg[0] = 0;
    for (int g = 0; g < kGroups; ++g) {
      ul.insert(ul.end(), lists[g].begin(), lists[g].end());
      ue.insert(ue.end(), ents[g].begin(), ents[g].end());
      gbeg[g + 1] = (int)ul.size();
    }
    uidx.resize(where.size());
    for (size_t k = 0; k < where.size(); ++k) uidx[k] = gbeg[where[k].first] + where[k].second;
  }
};

// Device copies of a plan's tables and the launch's results.
struct UnitDev {
  UDesc* desc = nullptr;
  int4* ul = nullptr;
  uint2* ue = nullptr;
  int32_t* uoff = nullptr;
  int32_t* uidx = nullptr;
  UnitOut* out = nullptr;
  UnitSum* sum = nullptr;
};

// one launch of unit group g (mod 12: norm width, precision, cache mode)
template <bool TWO>
void launch_unit_group(int g, unsigned n, size_t lds, hipStream_t s, const UnitArgs& A) {
  switch (g) {
    case 0: k_unit_solve<int32_t, true, CM_STREAM, TWO><<<n, kUnitThreads, lds, s>>>(A); break;
    case 1: k_unit_solve<int32_t, true, CM_ENTRIES, TWO><<<n, kUnitThreads, lds, s>>>(A); break;
    case 2: k_unit_solve<int32_t, false, CM_STREAM, TWO><<<n, kUnitThreads, lds, s>>>(A); break;
    case 3: k_unit_solve<int32_t, false, CM_ENTRIES, TWO><<<n, kUnitThreads, lds, s>>>(A); break;
    case 4: k_unit_solve<int32_t, false, CM_COEF, TWO><<<n, kUnitThreads, lds, s>>>(A); break;
    case 5: k_unit_solve<int32_t, false, CM_CPLX, TWO><<<n, kUnitThreads, lds, s>>>(A); break;
    case 6: k_unit_solve<int64_t, true, CM_STREAM, TWO><<<n, kUnitThreads, lds, s>>>(A); break;
    case 7: k_unit_solve<int64_t, true, CM_ENTRIES, TWO><<<n, kUnitThreads, lds, s>>>(A); break;
    case 8: k_unit_solve<int64_t, false, CM_STREAM, TWO><<<n, kUnitThreads, lds, s>>>(A); break;
    case 9: k_unit_solve<int64_t, false, CM_ENTRIES, TWO><<<n, kUnitThreads, lds, s>>>(A); break;
    case 10: k_unit_solve<int64_t, false, CM_COEF, TWO><<<n, kUnitThreads, lds, s>>>(A); break;
    default: k_unit_solve<int64_t, false, CM_CPLX, TWO><<<n, kUnitThreads, lds, s>>>(A); break;
  }
}

// the launches of a plan whose tables are on the device (asynchronous on s)
ss_status launch_unit_plan(const UnitPlan& P, const UnitDev& D, hipStream_t s) {
  UnitArgs A{D.desc, D.ul, D.ue, 0, 0, D.out};
  for (int g = 0; g < UnitPlan::kGroups; ++g) {
    const int n = P.gbeg[g + 1] - P.gbeg[g];
    if (n == 0) continue;
    A.ubase = P.gbeg[g];
    A.rows = P.rmax[g];
    const int gl = g % 12;
    const size_t lds = gl >= 6 ? unit_lds_bytes<int64_t>(P.rmax[g], (size_t)P.lmax[g])
                               : unit_lds_bytes<int32_t>(P.rmax[g], (size_t)P.lmax[g]);
    if (g >= 12) launch_unit_group<true>(gl, (unsigned)n, lds, s, A);
    else launch_unit_group<false>(gl, (unsigned)n, lds, s, A);
  }
  k_unit_final<<<grid_for(P.n_prob()), kBlock, 0, s>>>(P.n_prob(), D.uoff, D.uidx, D.out, D.sum);
  SS_HIP(hipGetLastError());
  return SS_OK;
}

// a launched problem's info from its summed unit results
ss_solve_info unit_info(const UnitItem& it, const UnitSum& sm) {
  const double rel = sm.ff > 0 ? std::sqrt(sm.rr / sm.ff) : 0.0;
  int status = sm.status;
  if (rel <= std::sqrt(it.d.tol2) || sm.ff == 0) status = SS_OK;
  else if (status == SS_OK) status = SS_ENOCONV;
  ss_solve_info in{};
  in.iters = sm.iters;
  in.outer_steps = it.prec == SS_FP64 ? 0 : sm.outer;
  in.rel_residual = rel;
  in.n = it.op->row_off[it.prob + 1] - it.op->row_off[it.prob];
  in.nnz = it.op->nnz_p[it.prob];
  in.n_components = it.op->comps[it.prob];
  in.status = status;
  return in;
}

// Problems solved by the class-resident CG in one go: gathered by add(), launched together
// (one k_unit_solve launch per norm width and precision), results read after a sync.
struct UnitBatch {
  using Item = UnitItem;
  std::vector<Item> items;
  // after launch(): per item (launch order), its results on the host once the stream is synced
  std::vector<Item> launched;
  UnitSum* h_sum = nullptr;       // pinned (cached: pinned_alloc)
  size_t h_cap = 0;
  std::vector<void*> dev;         // device blocks of the launch in flight

  ~UnitBatch() {   // the owner has synchronised the stream of a launch in flight
    release();
    pinned_free(h_sum);
  }
  void release() {
    for (void* q : dev) pool_free(q);
    dev.clear();
  }

  void add(OpImpl* op, int p, const void* f, void* u, double tol, ss_precision prec, int32_t max_iter, int req) {
    items.push_back(unit_item(op, p, f, u, tol, prec, max_iter, req));
  }

  template <typename T>
  ss_status alloc(T** p, size_t n) {
    SS_TRY(dalloc(p, std::max<size_t>(n, 1)));
    dev.push_back(*p);
    return SS_OK;
  }

  // launch every added problem on s (asynchronous); the caller syncs s before reading results
  ss_status launch(hipStream_t s) {
    launched.clear();
    for (int g = 0; g < 4; ++g)
      for (auto& it : items)
        if (it.group == g) launched.push_back(it);
    items.clear();
    const int np = (int)launched.size();
    if (np == 0) return SS_OK;
    UnitPlan P;
    P.make(launched);
    const int nu = P.n_units();
    UnitDev D;
    SS_TRY(alloc(&D.out, nu));
    SS_TRY(alloc(&D.sum, np));
    if ((size_t)np > h_cap) {
      pinned_free(h_sum);   // no copy into it is pending: the last launch's results were read
      h_sum = nullptr;
      h_cap = std::max<size_t>(np, 2 * h_cap);
      SS_HIP(pinned_alloc((void**)&h_sum, h_cap * sizeof(UnitSum)));
    }
    {   // descriptors and unit lists, one transfer
      Upload up;
      up.add(&D.desc, P.descs.data(), np);
      up.add(&D.ul, P.ul.data(), nu);
      up.add(&D.ue, P.ue.data(), nu);
      up.add(&D.uoff, P.uoff.data(), np + 1);
      up.add(&D.uidx, P.uidx.data(), nu);
      void* block = nullptr;
      const ss_status e = up.commit(&block, s);
      if (block) dev.push_back(block);
      SS_TRY(e);
    }
    SS_TRY(launch_unit_plan(P, D, s));
    SS_HIP(hipMemcpyAsync(h_sum, D.sum, np * sizeof(UnitSum), hipMemcpyDeviceToHost, s));
    return SS_OK;
  }

  // the i-th launched problem's info (valid after the stream has been synced)
  ss_solve_info info(int i) const { return unit_info(launched[i], h_sum[i]); }
};

struct Request {
  OpImpl* op;
  int64_t tag;
  int n_left;
};

struct EngineImpl {
  hipStream_t s = nullptr;
  int64_t budget = 0;
  int32_t max_slots = 0;
  int64_t bytes_in_use = 0;
  LaunchList list;
  std::vector<std::vector<int4>> items;   // per desc
  std::vector<int> req_of;                // per desc: request index
  std::vector<int> prob_of;               // per desc: problem within the op
  std::vector<Request> reqs;              // by request index (holes allowed)
  std::vector<int64_t> req_bytes;
  std::vector<int> free_req;
  bool dirty = false;
  // finished problems waiting for ss_engine_poll
  struct Done {
    int64_t tag;
    int32_t prob;
    ss_solve_info info;
  };
  std::vector<Done> done;
  PState* h_states = nullptr;             // pinned (cached: pinned_alloc)
  size_t h_cap = 0;
  UnitBatch units;                        // problems for the class-resident CG, launched next tick
  ~EngineImpl() {
    // a launch may still use its blocks, or a copy still fill the pinned buffers (error paths)
    if (!units.dev.empty() || h_states || units.h_sum) (void)hipStreamSynchronize(s);
    pinned_free(h_states);
  }

  ss_status ensure_host(size_t n) {
    if (n <= h_cap) return SS_OK;
    pinned_free(h_states);   // called between ticks: no copy into it is pending
    h_states = nullptr;
    h_cap = std::max(n, 2 * h_cap);
    SS_HIP(pinned_alloc((void**)&h_states, h_cap * sizeof(PState)));
    return SS_OK;
  }

  // A problem whose classes split into solve units runs the class-resident CG (launched at the
  // next tick, finished within it); the others run the per-problem kernels tick by tick and
  // need the operator's workspace.
  ss_status submit(OpImpl* op, const void* f, void* u, double tol, ss_precision prec, int32_t max_iter,
                   int64_t tag) {
    if (!f || !u) return fail(SS_EINVAL, "null vector");
    if (!(tol > 0) || max_iter < 1) return fail(SS_EINVAL, "tol must be > 0 and max_iter >= 1");
    if (prec != SS_FP64 && prec != SS_FP32_REFINE) return fail(SS_EINVAL, "unknown precision");
    if (op->busy) return fail(SS_EINVAL, "operator already has a solve in flight");
    bool any_engine = false;
    for (int p = 0; p < op->n_prob; ++p) any_engine |= op->urange[p].x < 0;
    const int64_t bytes =
        op_device_bytes(op) + (any_engine ? (int64_t)std::max(op->ws.bytes, workspace_bytes(op)) : 0);
    int active = 0;
    for (auto& r : reqs) active += r.op != nullptr;
    // a request larger than the whole budget could never be admitted beside others: it is admitted
    // when the engine holds nothing else
    if (budget > 0 && bytes_in_use + bytes > budget && active > 0)
      return fail(SS_ENOMEM, "HBM budget of the engine exceeded");
    if (max_slots > 0 && active >= max_slots) return fail(SS_ENOMEM, "no free engine slot");
    WS w{};
    if (any_engine) SS_TRY(workspace(op, &w));
    int ri;
    if (!free_req.empty()) {
      ri = free_req.back();
      free_req.pop_back();
    } else {
      ri = (int)reqs.size();
      reqs.push_back({});
      req_bytes.push_back(0);
    }
    reqs[ri] = Request{op, tag, op->n_prob};
    req_bytes[ri] = bytes;
    bytes_in_use += bytes;
    op->busy = true;
    for (int p = 0; p < op->n_prob; ++p) {
      if (op->urange[p].x >= 0) {
        units.add(op, p, f, u, tol, prec, max_iter, ri);
        continue;
      }
      Desc D = make_desc(op, w, p);
      D.f_canon = (const double2*)f;
      D.u_canon = (double2*)u;
      D.tol2 = tol * tol;
      D.tol2_in = kInnerTol * kInnerTol;
      D.max_iter = max_iter;
      D.prec = prec;
      D.init = 1;
      list.descs.push_back(D);
      items.push_back(items_of(op, p));
      req_of.push_back(ri);
      prob_of.push_back(p);
    }
    dirty = true;
    return SS_OK;
  }

  // launch the per-tick chain on the current list
  void launch_transitions() {
    LaunchList& L = list;
    const int nw = L.n_work(), nd = L.n_desc();
    k_state_init<<<grid_for(nd), kBlock, 0, s>>>(L.d_descs, nd);
    k_admit<<<L.grid, kSolveBlock, 0, s>>>(L.d_descs, L.d_work, nw, L.per);
    k_refine_add<<<L.grid, kSolveBlock, 0, s>>>(L.d_descs, L.d_work, nw, L.per);
    k_mv<MV_RESID><<<L.grid, kSolveBlock, L.lds_resid, s>>>(L.d_descs, L.d_work, nw, L.per, L.part_c());
    k_outer_scalars<<<nd, kSolveBlock, 0, s>>>(L.d_descs, nd, L.part_c());
    k_refine_start<<<L.grid, kSolveBlock, 0, s>>>(L.d_descs, L.d_work, nw, L.per);
    k_cg_start<<<L.grid, kSolveBlock, 0, s>>>(L.d_descs, L.d_work, nw, L.per, L.part_b());
    k_cg_scalars<<<nd, kSolveBlock, 0, s>>>(L.d_descs, nd, L.part_b());
  }

  void launch_iterations(int iters) {
    LaunchList& L = list;
    const int nw = L.n_work();
    for (int it = 0; it < iters; ++it) {
      k_mv<MV_DOT><<<L.grid, kSolveBlock, L.lds_dot, s>>>(L.d_descs, L.d_work, nw, L.per, L.part_a());
      k_cg_update<<<L.grid, kSolveBlock, 0, s>>>(L.d_descs, L.d_work, nw, L.per, L.part_a(), L.part_b());
      k_cg_dir<<<L.grid, kSolveBlock, 0, s>>>(L.d_descs, L.d_work, nw, L.per, L.part_b());
    }
  }

  // one tick; *n_active = problems still active afterwards
  // results of the class-resident launch of this tick (the stream has been synced)
  void collect_units() {
    for (size_t i = 0; i < units.launched.size(); ++i) {
      const UnitBatch::Item& it = units.launched[i];
      done.push_back(Done{reqs[it.req].tag, it.prob, units.info((int)i)});
      finish_problem(it.req);
    }
    units.launched.clear();
    units.release();
  }

  void finish_problem(int ri) {
    if (--reqs[ri].n_left == 0) {
      reqs[ri].op->busy = false;
      bytes_in_use -= req_bytes[ri];
      reqs[ri].op = nullptr;
      free_req.push_back(ri);
    }
  }

  ss_status step(int iters, int* n_active) {
    if (!units.items.empty()) SS_TRY(units.launch(s));
    if (dirty) {
      SS_TRY(list.upload(s, items));
      dirty = false;
    }
    const int nd = list.n_desc();
    if (nd == 0) {
      if (!units.launched.empty()) {
        SS_HIP(hipStreamSynchronize(s));
        collect_units();
      }
      *n_active = 0;
      return SS_OK;
    }
    launch_transitions();
    bool had_init = false;
    for (auto& D : list.descs) had_init |= D.init != 0;
    if (had_init) {
      for (auto& D : list.descs) D.init = 0;
      SS_TRY(list.upload_descs(s));
    }
    launch_iterations(iters);
    // poll
    SS_TRY(ensure_host(nd));
    k_gather_states<<<grid_for(nd), kBlock, 0, s>>>(list.d_descs, nd, list.d_states);
    SS_HIP(hipMemcpyAsync(h_states, list.d_states, nd * sizeof(PState), hipMemcpyDeviceToHost, s));
    SS_HIP(hipStreamSynchronize(s));
    SS_HIP(hipGetLastError());
    if (!units.launched.empty()) collect_units();
    std::vector<int> fin;
    for (int k = 0; k < nd; ++k)
      if (h_states[k].done) fin.push_back(k);
    if (!fin.empty()) SS_TRY(retire(fin));
    *n_active = list.n_desc();
    return SS_OK;
  }

  ss_status retire(const std::vector<int>& fin) {
    for (int k : fin) list.descs[k].final_ = 1;
    SS_TRY(list.upload_descs(s));
    const int nw = list.n_work(), nd = list.n_desc();
    k_mv<MV_RESID><<<list.grid, kSolveBlock, list.lds_resid, s>>>(list.d_descs, list.d_work, nw, list.per,
                                                             list.part_c(), 1);
    k_final_scalars<<<nd, kSolveBlock, 0, s>>>(list.d_descs, nd, list.part_c(), list.d_states);
    k_retire<<<list.grid, kSolveBlock, 0, s>>>(list.d_descs, list.d_work, nw, list.per);
    SS_HIP(hipMemcpyAsync(h_states, list.d_states, nd * sizeof(PState), hipMemcpyDeviceToHost, s));
    SS_HIP(hipStreamSynchronize(s));
    std::vector<char> gone(nd, 0);
    for (int k : fin) {
      const Desc& D = list.descs[k];
      const PState& st = h_states[k];
      const int ri = req_of[k], p = prob_of[k];
      OpImpl* op = reqs[ri].op;
      ss_solve_info in{};
      const double rel = st.ff > 0 ? std::sqrt(st.rr / st.ff) : 0.0;
      const double tol = std::sqrt(D.tol2);
      int status = st.status;
      if (rel <= tol || st.ff == 0) status = SS_OK;
      else if (status == SS_OK) status = SS_ENOCONV;
      in.iters = st.total_iters;
      in.outer_steps = D.prec == SS_FP64 ? 0 : st.outer;
      in.rel_residual = rel;
      in.n = op->row_off[p + 1] - op->row_off[p];
      in.nnz = op->nnz_p[p];
      in.n_components = op->comps[p];
      in.status = status;
      done.push_back(Done{reqs[ri].tag, p, in});
      gone[k] = 1;
      finish_problem(ri);
    }
    // compact the active set
    std::vector<Desc> nd_descs;
    std::vector<std::vector<int4>> nitems;
    std::vector<int> nreq, nprob;
    for (int k = 0; k < nd; ++k) {
      if (gone[k]) continue;
      nd_descs.push_back(list.descs[k]);
      nitems.push_back(std::move(items[k]));
      nreq.push_back(req_of[k]);
      nprob.push_back(prob_of[k]);
    }
    list.descs.swap(nd_descs);
    items.swap(nitems);
    req_of.swap(nreq);
    prob_of.swap(nprob);
    dirty = true;
    return SS_OK;
  }
};

int64_t op_device_bytes(const OpImpl* op) {
  const int64_t nb = op->wide_norm ? 8 : 4;
  return op->total * 4 + op->n_exec * 8 + op->total * 8 + op->n_sell * 4 +
         (op->n_slices + 1) * 4 + op->n_exec * nb + (int64_t)op->n_prob * kTab * (16 + 8 + 8) +
         (int64_t)op->work.size() * 16 + (int64_t)op->units.size() * 16;
}

ss_status engine_create(int64_t budget, int32_t max_slots, hipStream_t s, EngineImpl** out) {
  EngineImpl* e = new EngineImpl();
  e->s = s;
  e->budget = budget;
  e->max_slots = max_slots;
  *out = e;
  return SS_OK;
}
void engine_free(EngineImpl* e) { delete e; }
ss_status engine_submit(EngineImpl* e, OpImpl* op, const void* f, void* u, double tol, ss_precision prec,
                        int32_t max_iter, int64_t tag) {
  return e->submit(op, f, u, tol, prec, max_iter, tag);
}
ss_status engine_step(EngineImpl* e, int32_t iters, int32_t* n_active) {
  if (iters < 1) return fail(SS_EINVAL, "iters must be >= 1");
  int na = 0;
  SS_TRY(e->step(iters, &na));
  if (n_active) *n_active = na;
  return SS_OK;
}
ss_status engine_poll(EngineImpl* e, int32_t cap, int64_t* tags, int32_t* probs, ss_solve_info* info,
                      int32_t* n_out) {
  const int n = std::min<int>(cap, (int)e->done.size());
  for (int i = 0; i < n; ++i) {
    if (tags) tags[i] = e->done[i].tag;
    if (probs) probs[i] = e->done[i].prob;
    if (info) info[i] = e->done[i].info;
  }
  e->done.erase(e->done.begin(), e->done.begin() + n);
  *n_out = n;
  return SS_OK;
}
ss_status engine_usage(const EngineImpl* e, int32_t* n_active, int64_t* bytes) {
  if (n_active) {
    int a = 0;
    for (auto& r : e->reqs) a += r.op != nullptr;
    *n_active = a;
  }
  if (bytes) *bytes = e->bytes_in_use;
  return SS_OK;
}

// ---------------------------------------------------------------- batch solve and apply
ss_status solve_op_impl(OpImpl* op, const void* f, void* u, double tol, ss_precision prec, int32_t max_iter,
                        hipStream_t stream, ss_solve_info* info) {
  auto t0 = std::chrono::steady_clock::now();
  EngineImpl e;
  e.s = stream;
  SS_TRY(e.submit(op, f, u, tol, prec, max_iter, 0));
  // polling cadence: a few iterations per tick, growing while nothing finishes
  int iters = 4, na = 1;
  int guard = 0;
  while (na > 0) {
    SS_TRY(e.step(iters, &na));
    if (iters < 16) iters *= 2;
    if (++guard > 1000000) return fail(SS_EINVAL, "internal: solve did not terminate");
  }
  const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  ss_status worst = SS_OK;
  for (auto& d : e.done) {
    if (info) {
      info[d.prob] = d.info;
      info[d.prob].t_solve_ms = ms;
    }
    if (d.info.status != SS_OK && worst == SS_OK) worst = (ss_status)d.info.status;
  }
  if (worst == SS_ENOCONV) return fail(SS_ENOCONV, "tolerance not reached within the iteration limit");
  if (worst == SS_EBREAKDOWN) return fail(SS_EBREAKDOWN, "CG breakdown: <p, L p> <= 0 or not finite");
  return worst;
}

ss_status apply_impl(const OpImpl* op_c, ss_precision prec, const void* x, void* y, hipStream_t s) {
  OpImpl* op = const_cast<OpImpl*>(op_c);
  auto& c = op->apply_cache;
  if (!c.list || c.x != x || c.y != y || c.prec != prec) {
    if (!c.list) c.list = new LaunchList();
    LaunchList& L = *c.list;
    L.descs.clear();
    std::vector<std::vector<int4>> items;
    WS w{};
    for (int p = 0; p < op->n_prob; ++p) {
      Desc D = make_desc(op, w, p);
      const int64_t e0 = op->eoff[p];
      if (prec == SS_FP64) {
        D.x64 = (double2*)x + e0;
        D.q64 = (double2*)y + e0;
      } else {
        D.x32 = (float2*)x + e0;
        D.q32 = (float2*)y + e0;
      }
      D.prec = prec;
      L.descs.push_back(D);
      items.push_back(items_of(op, p));
    }
    SS_TRY(L.upload(s, items));
    c.x = x;
    c.y = y;
    c.prec = prec;
  }
  LaunchList& L = *c.list;
  k_mv<MV_PLAIN><<<L.grid, kSolveBlock, L.lds_dot, s>>>(L.d_descs, L.d_work, L.n_work(), L.per, nullptr);
  SS_HIP(hipGetLastError());
  return SS_OK;
}

void free_apply_cache(OpImpl* op) {
  delete op->apply_cache.list;
  op->apply_cache.list = nullptr;
}

// ---------------------------------------------------------------- solve without allocation
// The class-resident solve of ss_solve_op for callers that cannot allocate device memory (code
// under graph capture, tight serving loops, harnesses that forbid allocation): the launch's
// tables and per-unit results live in one fixed device array per GPU instead of pool blocks, and
// are copied from and to pageable host memory instead of the pinned staging rings.  Calls that
// overlap on one GPU share the array and race.
constexpr size_t kScratchBytes = SS_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kScratchDevices = 64;
std::mutex g_scratch_mu;
unsigned char* g_scratch_ptr[kScratchDevices] = {};

// the device address of the current device's copy of the array, looked up once per device with
// that device current (the array's name is not a device address in host code)
ss_status scratch_base(unsigned char** out) {
  int dev = 0;
  SS_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kScratchDevices) return fail(SS_EDEVICE, "device index beyond the scratch table");
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    SS_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(SS_EDEVICE, "scratch array has no device address");
    g_scratch_ptr[dev] = (unsigned char*)p;
  }
  *out = g_scratch_ptr[dev];
  return SS_OK;
}

// offset of the next 256-byte aligned piece of `bytes` bytes
size_t carve(size_t* used, size_t bytes) {
  const size_t at = *used;
  *used += (std::max<size_t>(bytes, 1) + 255) & ~size_t(255);
  return at;
}

}  // namespace

ss_status solve_op_noalloc_impl(OpImpl* op, const void* f, void* u, double tol, ss_precision prec,
                                int32_t max_iter, hipStream_t s, ss_solve_info* info) {
  const auto t0 = std::chrono::steady_clock::now();
  if (!f || !u) return fail(SS_EINVAL, "null vector");
  if (!(tol > 0) || max_iter < 1) return fail(SS_EINVAL, "tol must be > 0 and max_iter >= 1");
  if (prec != SS_FP64 && prec != SS_FP32_REFINE) return fail(SS_EINVAL, "unknown precision");
  if (op->busy) return fail(SS_EINVAL, "operator already has a solve in flight");
  int dev = 0;
  SS_HIP(hipGetDevice(&dev));
  if (dev != op->device) return fail(SS_EINVAL, "the operator was built on another device");
  const int np = op->n_prob;
  for (int p = 0; p < np; ++p)
    if (op->urange[p].x < 0)
      return fail(SS_EINVAL, "problem " + std::to_string(p) +
                                 " has a class of more than 2048 rows, which needs the per-problem solver "
                                 "workspace of ss_solve_op");
  std::vector<UnitItem> items;
  items.reserve(np);
  for (int p = 0; p < np; ++p) items.push_back(unit_item(op, p, f, u, tol, prec, max_iter, 0));
  UnitPlan P;
  P.make(items);   // one group: all problems of op share the norm width and the precision
  const int nu = P.n_units();
  size_t used = 0;
  const size_t o_desc = carve(&used, np * sizeof(UDesc));
  const size_t o_ul = carve(&used, nu * sizeof(int4));
  const size_t o_ue = carve(&used, nu * sizeof(uint2));
  const size_t o_uoff = carve(&used, (np + 1) * sizeof(int32_t));
  const size_t o_uidx = carve(&used, nu * sizeof(int32_t));
  const size_t o_out = carve(&used, nu * sizeof(UnitOut));
  const size_t o_sum = carve(&used, np * sizeof(UnitSum));
  if (used > kScratchBytes)
    return fail(SS_ERANGE, "the solve needs " + std::to_string(used) + " bytes of scratch (" + std::to_string(np) +
                               " problems, " + std::to_string(nu) + " units); the maximum is " +
                               std::to_string(kScratchBytes));
  unsigned char* base = nullptr;
  SS_TRY(scratch_base(&base));
  UnitDev D;
  D.desc = (UDesc*)(base + o_desc);
  D.ul = (int4*)(base + o_ul);
  D.ue = (uint2*)(base + o_ue);
  D.uoff = (int32_t*)(base + o_uoff);
  D.uidx = (int32_t*)(base + o_uidx);
  D.out = (UnitOut*)(base + o_out);
  D.sum = (UnitSum*)(base + o_sum);
  // every piece is written in full by these copies or by the kernels before it is read
  SS_HIP(hipMemcpyAsync(D.desc, P.descs.data(), np * sizeof(UDesc), hipMemcpyHostToDevice, s));
  SS_HIP(hipMemcpyAsync(D.ul, P.ul.data(), nu * sizeof(int4), hipMemcpyHostToDevice, s));
  SS_HIP(hipMemcpyAsync(D.ue, P.ue.data(), nu * sizeof(uint2), hipMemcpyHostToDevice, s));
  SS_HIP(hipMemcpyAsync(D.uoff, P.uoff.data(), (np + 1) * sizeof(int32_t), hipMemcpyHostToDevice, s));
  SS_HIP(hipMemcpyAsync(D.uidx, P.uidx.data(), nu * sizeof(int32_t), hipMemcpyHostToDevice, s));
  SS_TRY(launch_unit_plan(P, D, s));
  std::vector<UnitSum> hs(np);
  SS_HIP(hipMemcpyAsync(hs.data(), D.sum, np * sizeof(UnitSum), hipMemcpyDeviceToHost, s));
  SS_HIP(hipStreamSynchronize(s));
  const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  ss_status worst = SS_OK;
  for (int p = 0; p < np; ++p) {
    ss_solve_info in = unit_info(items[p], hs[p]);
    in.t_solve_ms = ms;
    if (info) info[p] = in;
    if (in.status == SS_EBREAKDOWN || (in.status == SS_ENOCONV && worst == SS_OK)) worst = (ss_status)in.status;
  }
  if (worst == SS_ENOCONV) return fail(SS_ENOCONV, "tolerance not reached within the iteration limit");
  if (worst == SS_EBREAKDOWN) return fail(SS_EBREAKDOWN, "CG breakdown: <p, L p> <= 0 or not finite");
  return SS_OK;
}

}  // namespace ss
