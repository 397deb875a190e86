// Matvec and Jacobi-preconditioned CG on the SELL-64 layout.
//
// Operator (Sec. 9, Eq. FiniteGalerkinOperator): for execution row e holding
// key k and a stored entry (column c holding l = k - w_j, index j)
//     coefficient = 4 pi^2 (k . l) a_j = 2 pi^2 (|k|^2 + |l|^2 - |w_j|^2) a_j,
// the integer bracket exact in int32 (int64 when |k|^2 >= 2^30), the factor
// 2 pi^2 a_j pre-scaled per problem and staged in LDS with |w_j|^2.
//
// Mapping: one 256-thread block per work item = up to four 64-row slices of
// one problem; one wavefront per slice, one lane per row; entries of a slice
// are stored column-major, so each step of the row loop is one coalesced
// 256-byte load per wavefront.  Gathers of x and |l|^2 stay inside the row's
// problem and class.  Work items are assigned to blocks so that consecutive
// items land on the same XCD (blocks are dealt to the 8 XCDs round-robin), so
// one problem's gathers hit one L2.
//
// CG (textbook PCG, the Jacobi diagonal 4 pi^2 |k|^2 a_0 being the
// denominator of the recurrence in the proof of Prop. SolutionSupport; row
// k = 0 is identically zero and is excluded).  Each problem of a batch runs
// its own CG with its own scalars.  Every inner product is reduced in a fixed
// order -- lanes, then wavefronts, then the problem's work items -- that
// depends only on the problem itself, so a problem's iterates are bitwise the
// same alone and inside any batch.  Three kernels per iteration:
//   mv_dot  q = L p,  partial <p, q>
//   update  alpha = rho / <p, q>;  x += alpha p;  r -= alpha q;  partial <r, D^-1 r>, |r|^2
//   dir     beta = rho' / rho;  stop test |r| <= tol |f|;  p = D^-1 r + beta p
// Scalars that one kernel writes are read only by later kernels (rho is
// double-buffered by iteration parity).
//
// FP32 + refinement: the outer loop forms r = f - L x with the FP64 operator,
// scales it to unit norm, runs FP32 PCG (FP32 operator, FP32 vectors, FP64
// inner products) to a loose tolerance, and adds the correction to x in FP64,
// until the FP64 residual meets tol.
#include <algorithm>
#include <chrono>
#include <cmath>

#include "ss_internal.h"

namespace ss {

namespace {

constexpr double kTwoPi2 = 2.0 * M_PI * M_PI;
constexpr double kFourPi2 = 4.0 * M_PI * M_PI;

enum { MV_PLAIN = 0, MV_DOT = 1, MV_RESID = 2 };

template <typename V> struct Real;
template <> struct Real<double2> { using T = double; };
template <> struct Real<float2> { using T = float; };

template <typename V> __device__ inline const V* atab(const OpDev& op);
template <> __device__ inline const double2* atab<double2>(const OpDev& op) { return op.A64; }
template <> __device__ inline const float2* atab<float2>(const OpDev& op) { return op.A32; }

__device__ inline int work_index(int b, int per) { return (b & 7) * per + (b >> 3); }

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Sum of v over the block; valid in thread 0 only.  Fixed order.
__device__ inline double block_sum(double v, double* red) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) red[wave] = v;
  __syncthreads();
  const double s = (red[0] + red[1]) + (red[2] + red[3]);
  __syncthreads();
  return s;
}

// Sum of part[i*stride + off] for i in [b, e), every thread gets the result.  Fixed order.
__device__ inline double range_sum(const double* __restrict__ part, int stride, int off, int b, int e,
                                   double* red) {
  double v = 0;
  for (int i = b + (int)threadIdx.x; i < e; i += kBlock) v += part[(int64_t)i * stride + off];
  return block_sum(v, red);
}

template <typename NormT, typename V>
__device__ inline V sell_row(const uint32_t* __restrict__ sent, uint32_t base, uint32_t width, int lane,
                             NormT nk, const NormT* __restrict__ normp, const V* __restrict__ xp,
                             const V* As, const NormT* nus) {
  using R = typename Real<V>::T;
  R ar = 0, ai = 0;
  for (uint32_t q = 0; q < width; ++q) {
    const uint32_t ent = sent[base + q * kSlice + lane];
    const uint32_t j = ent >> kColBits;
    if (j != (uint32_t)kNullJ) {
      const uint32_t c = ent & kColMask;
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

// y = L x (PLAIN);  q = L p with partial Re<p, q> (DOT);  r = f - L x with partials |r|^2, |f|^2 (RESID)
template <typename NormT, typename V, int MODE>
__global__ __launch_bounds__(kBlock) void k_mv(OpDev op, const V* __restrict__ x, V* __restrict__ y,
                                               const V* __restrict__ f, double* __restrict__ part,
                                               const PState* __restrict__ ps, int per) {
  const int w = work_index(blockIdx.x, per);
  if (w >= op.n_work) return;
  const int4 wk = op.work[w];
  const int p = wk.x;
  if (MODE != MV_PLAIN && ps[p].done) return;
  __shared__ V As[64];
  __shared__ NormT nus[64];
  __shared__ double red[4];
  const int tid = threadIdx.x;
  if (tid < 64) {
    As[tid] = atab<V>(op)[p * 64 + tid];
    nus[tid] = (NormT)op.nu[p * 64 + tid];
  }
  __syncthreads();
  const int wave = tid >> 6, lane = tid & 63;
  double v0 = 0, v1 = 0;
  if (wave < wk.z) {
    const int64_t sl = wk.y + wave;
    const int64_t e = sl * kSlice + lane;
    const int64_t eb = op.eoff[p];
    const NormT* normv = (const NormT*)op.norm;
    const uint32_t base = op.sptr[sl];
    const uint32_t width = (op.sptr[sl + 1] - base) / kSlice;
    const V acc = sell_row<NormT, V>(op.sent, base, width, lane, normv[e], normv + eb, x + eb, As, nus);
    if (MODE == MV_PLAIN) {
      y[e] = acc;
    } else if (MODE == MV_DOT) {
      y[e] = acc;
      const V pe = x[e];
      v0 = (double)pe.x * (double)acc.x + (double)pe.y * (double)acc.y;
    } else {
      const V fe = f[e];
      V r;
      r.x = fe.x - acc.x;
      r.y = fe.y - acc.y;
      y[e] = r;
      v0 = (double)r.x * r.x + (double)r.y * r.y;
      v1 = (double)fe.x * fe.x + (double)fe.y * fe.y;
    }
  }
  if (MODE == MV_DOT) {
    const double s = block_sum(v0, red);
    if (tid == 0) part[2 * (int64_t)w] = s;
  } else if (MODE == MV_RESID) {
    const double s0 = block_sum(v0, red);
    const double s1 = block_sum(v1, red);
    if (tid == 0) {
      part[2 * (int64_t)w] = s0;
      part[2 * (int64_t)w + 1] = s1;
    }
  }
}

template <typename NormT>
__device__ inline double jacobi_inv(NormT nk, double a0) {
  return nk > 0 ? 1.0 / (kFourPi2 * a0 * (double)nk) : 0.0;
}

// alpha = rho / <p,q>;  x += alpha p;  r -= alpha q;  partials <r, D^-1 r>, |r|^2
template <typename NormT, typename V>
__global__ __launch_bounds__(kBlock) void k_cg_update(OpDev op, V* __restrict__ x, V* __restrict__ r,
                                                      const V* __restrict__ pv, const V* __restrict__ q,
                                                      const double* __restrict__ part_pq,
                                                      double* __restrict__ part_rz, PState* ps, int par,
                                                      int per) {
  using R = typename Real<V>::T;
  const int w = work_index(blockIdx.x, per);
  if (w >= op.n_work) return;
  const int4 wk = op.work[w];
  const int p = wk.x;
  if (ps[p].done) return;
  __shared__ double red[4];
  const int2 wr = op.wrange[p];
  const double pq = range_sum(part_pq, 2, 0, wr.x, wr.y, red);
  const double alpha = ps[p].rho[par] / pq;
  if (!(pq > 0.0) || !isfinite(alpha)) {
    if (w == wr.x && threadIdx.x == 0) {
      ps[p].status = SS_EBREAKDOWN;
      ps[p].done = 1;
    }
    return;
  }
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  double v0 = 0, v1 = 0;
  if (wave < wk.z) {
    const int64_t e = (int64_t)(wk.y + wave) * kSlice + lane;
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
    v0 = rr * jacobi_inv(((const NormT*)op.norm)[e], op.a0[p]);
    v1 = rr;
  }
  const double s0 = block_sum(v0, red);
  const double s1 = block_sum(v1, red);
  if (tid == 0) {
    part_rz[2 * (int64_t)w] = s0;
    part_rz[2 * (int64_t)w + 1] = s1;
  }
}

// beta = rho'/rho;  convergence;  p = D^-1 r + beta p
template <typename NormT, typename V>
__global__ __launch_bounds__(kBlock) void k_cg_dir(OpDev op, const V* __restrict__ r, V* __restrict__ pv,
                                                   const double* __restrict__ part_rz, PState* ps, int par,
                                                   double tol2, int per) {
  using R = typename Real<V>::T;
  const int w = work_index(blockIdx.x, per);
  if (w >= op.n_work) return;
  const int4 wk = op.work[w];
  const int p = wk.x;
  if (ps[p].done) return;
  __shared__ double red[4];
  const int2 wr = op.wrange[p];
  const double rz = range_sum(part_rz, 2, 0, wr.x, wr.y, red);
  const double rr = range_sum(part_rz, 2, 1, wr.x, wr.y, red);
  const double beta = rz / ps[p].rho[par];
  const bool conv = rr <= tol2 * ps[p].ff;
  if (w == wr.x && threadIdx.x == 0) {
    ps[p].rho[par ^ 1] = rz;
    ps[p].rr = rr;
    ps[p].iters += 1;
    if (conv) ps[p].done = 1;
  }
  if (conv) return;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  if (wave < wk.z) {
    const int64_t e = (int64_t)(wk.y + wave) * kSlice + lane;
    const R dinv = (R)jacobi_inv(((const NormT*)op.norm)[e], op.a0[p]);
    const R b = (R)beta;
    const V re = r[e];
    V pe = pv[e];
    pe.x = dinv * re.x + b * pe.x;
    pe.y = dinv * re.y + b * pe.y;
    pv[e] = pe;
  }
}

// Start of a CG run from residual r (x already consistent): p = D^-1 r, partial <r, D^-1 r>, |r|^2.
template <typename NormT, typename V>
__global__ __launch_bounds__(kBlock) void k_cg_start(OpDev op, const V* __restrict__ r, V* __restrict__ pv,
                                                     double* __restrict__ part_rz, const PState* ps, int per) {
  using R = typename Real<V>::T;
  const int w = work_index(blockIdx.x, per);
  if (w >= op.n_work) return;
  const int4 wk = op.work[w];
  const int p = wk.x;
  if (ps[p].done) return;
  __shared__ double red[4];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  double v0 = 0, v1 = 0;
  if (wave < wk.z) {
    const int64_t e = (int64_t)(wk.y + wave) * kSlice + lane;
    const double di = jacobi_inv(((const NormT*)op.norm)[e], op.a0[p]);
    const V re = r[e];
    V pe;
    pe.x = (R)di * re.x;
    pe.y = (R)di * re.y;
    pv[e] = pe;
    const double rr = (double)re.x * re.x + (double)re.y * re.y;
    v0 = rr * di;
    v1 = rr;
  }
  const double s0 = block_sum(v0, red);
  const double s1 = block_sum(v1, red);
  if (tid == 0) {
    part_rz[2 * (int64_t)w] = s0;
    part_rz[2 * (int64_t)w + 1] = s1;
  }
}

// One block per problem: scalars of a fresh CG run.  ff is |rhs|^2 (taken
// from `part_f` column 1 when given, else equal to the start residual).
__global__ void k_cg_scalars(OpDev op, const double* __restrict__ part_rz, const double* __restrict__ part_f,
                             PState* ps, double tol2) {
  const int p = blockIdx.x;
  if (p >= op.n_prob) return;
  __shared__ double red[4];
  const int2 wr = op.wrange[p];
  const double rz = range_sum(part_rz, 2, 0, wr.x, wr.y, red);
  const double rr = range_sum(part_rz, 2, 1, wr.x, wr.y, red);
  const double ff = part_f ? range_sum(part_f, 2, 1, wr.x, wr.y, red) : rr;
  if (threadIdx.x == 0 && !ps[p].done) {
    ps[p].rho[0] = rz;
    ps[p].rr = rr;
    ps[p].rr0 = rr;
    ps[p].ff = ff;
    ps[p].iters = 0;
    if (rr <= tol2 * ff) ps[p].done = 1;
  }
}

// One block per problem: |r|^2 and |f|^2 of an FP64 residual; outer stop test.
__global__ void k_resid_scalars(OpDev op, const double* __restrict__ part, PState* ps, double tol2,
                                int mark_done) {
  const int p = blockIdx.x;
  if (p >= op.n_prob) return;
  __shared__ double red[4];
  const int2 wr = op.wrange[p];
  const double rr = range_sum(part, 2, 0, wr.x, wr.y, red);
  const double ff = range_sum(part, 2, 1, wr.x, wr.y, red);
  if (threadIdx.x == 0) {
    ps[p].rr = rr;
    ps[p].ff = ff;
    ps[p].scale = sqrt(rr);
    if (mark_done && !ps[p].done && rr <= tol2 * ff) ps[p].done = 1;
  }
}

__global__ void k_count_active(int n_prob, const PState* ps, int* out) {
  __shared__ int cnt;
  if (threadIdx.x == 0) cnt = 0;
  __syncthreads();
  int c = 0;
  for (int p = threadIdx.x; p < n_prob; p += blockDim.x) c += ps[p].done ? 0 : 1;
  atomicAdd(&cnt, c);
  __syncthreads();
  if (threadIdx.x == 0) *out = cnt;
}

// canonical -> execution order (padding rows get 0); k = 0 rows of x forced to 0
__global__ void k_gather_in(int64_t n_exec, const int64_t* __restrict__ exec2canon, const double2* __restrict__ fc,
                            const double2* __restrict__ uc, double2* __restrict__ f, double2* __restrict__ x) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n_exec) return;
  const int64_t r = exec2canon[e];
  double2 fv = make_double2(0, 0), xv = make_double2(0, 0);
  if (r >= 0) {
    fv = fc[r];
    xv = uc[r];
  }
  f[e] = fv;
  x[e] = xv;
}

template <typename NormT>
__global__ void k_scatter_out(int64_t n_exec, const int64_t* __restrict__ exec2canon, const NormT* __restrict__ norm,
                              const double2* __restrict__ x, double2* __restrict__ uc) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n_exec) return;
  const int64_t r = exec2canon[e];
  if (r >= 0) uc[r] = norm[e] > 0 ? x[e] : make_double2(0, 0);
}

template <typename NormT>
__global__ void k_zero_k0(int64_t n_exec, const NormT* __restrict__ norm, double2* __restrict__ x) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n_exec && norm[e] == 0) x[e] = make_double2(0, 0);
}

// FP32 inner start: r32 = r64 / scale, x32 = 0 (problems still open)
__global__ void k_refine_start(OpDev op, const double2* __restrict__ r64, float2* __restrict__ r32,
                               float2* __restrict__ x32, const PState* ps_outer, int per) {
  const int w = work_index(blockIdx.x, per);
  if (w >= op.n_work) return;
  const int4 wk = op.work[w];
  const int p = wk.x;
  if (ps_outer[p].done) return;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  if (wave < wk.z) {
    const int64_t e = (int64_t)(wk.y + wave) * kSlice + lane;
    const double s = ps_outer[p].scale > 0 ? 1.0 / ps_outer[p].scale : 0.0;
    const double2 rv = r64[e];
    r32[e] = make_float2((float)(rv.x * s), (float)(rv.y * s));
    x32[e] = make_float2(0.f, 0.f);
  }
}

// x64 += scale * x32
__global__ void k_refine_add(OpDev op, double2* __restrict__ x64, const float2* __restrict__ x32,
                             const PState* ps_outer, int per) {
  const int w = work_index(blockIdx.x, per);
  if (w >= op.n_work) return;
  const int4 wk = op.work[w];
  const int p = wk.x;
  if (ps_outer[p].done) return;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  if (wave < wk.z) {
    const int64_t e = (int64_t)(wk.y + wave) * kSlice + lane;
    const double s = ps_outer[p].scale;
    const float2 c = x32[e];
    double2 xv = x64[e];
    xv.x += s * (double)c.x;
    xv.y += s * (double)c.y;
    x64[e] = xv;
  }
}

__global__ void k_accum_iters(int n_prob, PState* ps, const PState* ps_in) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < n_prob) ps[p].total_iters += ps_in[p].iters;
}

__global__ void k_init_state(int n_prob, PState* ps, const PState* copy_done_from) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n_prob) return;
  PState s{};
  s.done = copy_done_from ? copy_done_from[p].done : 0;
  s.status = SS_OK;
  ps[p] = s;
}

inline unsigned grid_for(int64_t n) { return (unsigned)std::max<int64_t>(1, ceil_div(n, kBlock)); }

// ---------------------------------------------------------------- workspace
struct WS {
  double2 *x64, *r64, *p64, *q64, *f64;
  float2 *x32, *r32, *p32, *q32;
  double *part_a, *part_b, *part_c;
  PState *ps, *ps_in;
  int* active;   // pinned host
};

ss_status workspace(OpImpl* op, WS* w) {
  const int64_t n = op->n_exec;
  const int64_t nw = (int64_t)op->work.size();
  auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
  const size_t need = al(5 * n * sizeof(double2)) + al(4 * n * sizeof(float2)) + al(3 * 2 * nw * sizeof(double)) +
                      al(2 * op->n_prob * sizeof(PState)) + 4096;
  if (op->ws.bytes < need) {
    if (op->ws.base) (void)hipFree(op->ws.base);
    op->ws.base = nullptr;
    op->ws.bytes = 0;
    SS_HIP(hipMalloc(&op->ws.base, need));
    op->ws.bytes = need;
  }
  char* b = (char*)op->ws.base;
  auto take = [&](size_t bytes) {
    char* r = b;
    b += al(bytes);
    return (void*)r;
  };
  w->x64 = (double2*)take(n * sizeof(double2));
  w->r64 = w->x64 + n;
  w->p64 = w->r64 + n;
  w->q64 = w->p64 + n;
  w->f64 = w->q64 + n;
  b = (char*)op->ws.base + al(5 * n * sizeof(double2));
  w->x32 = (float2*)take(4 * n * sizeof(float2));
  w->r32 = w->x32 + n;
  w->p32 = w->r32 + n;
  w->q32 = w->p32 + n;
  w->part_a = (double*)take(3 * 2 * nw * sizeof(double));
  w->part_b = w->part_a + 2 * nw;
  w->part_c = w->part_b + 2 * nw;
  w->ps = (PState*)take(2 * op->n_prob * sizeof(PState));
  w->ps_in = w->ps + op->n_prob;
  return SS_OK;
}

template <typename NormT>
struct Solver {
  OpImpl* op;
  OpDev od;
  hipStream_t s;
  int per;
  unsigned grid;
  int* h_active = nullptr;
  int* d_active = nullptr;

  ss_status count_active(const PState* ps, int* out) {
    k_count_active<<<1, kBlock, 0, s>>>(op->n_prob, ps, d_active);
    SS_HIP(hipMemcpyAsync(h_active, d_active, 4, hipMemcpyDeviceToHost, s));
    SS_HIP(hipStreamSynchronize(s));
    *out = *h_active;
    return SS_OK;
  }

  // CG on L x = rhs from the residual already in r (x consistent with it).
  template <typename V>
  ss_status cg(V* x, V* r, V* p, V* q, PState* ps, double* part_pq, double* part_rz, const double* part_f,
               double tol, int max_iter, int* iters_run) {
    const double tol2 = tol * tol;
    k_cg_start<NormT, V><<<grid, kBlock, 0, s>>>(od, r, p, part_rz, ps, per);
    k_cg_scalars<<<op->n_prob, kBlock, 0, s>>>(od, part_rz, part_f, ps, tol2);
    int it = 0;
    int check = 4;
    while (it < max_iter) {
      const int par = it & 1;
      k_mv<NormT, V, MV_DOT><<<grid, kBlock, 0, s>>>(od, p, q, nullptr, part_pq, ps, per);
      k_cg_update<NormT, V><<<grid, kBlock, 0, s>>>(od, x, r, p, q, part_pq, part_rz, ps, par, per);
      k_cg_dir<NormT, V><<<grid, kBlock, 0, s>>>(od, r, p, part_rz, ps, par, tol2, per);
      ++it;
      if (it % check == 0 || it == max_iter) {
        int act = 0;
        SS_TRY(count_active(ps, &act));
        if (act == 0) break;
        if (check < 16) check *= 2;
      }
    }
    *iters_run = it;
    return SS_OK;
  }
};

template <typename NormT>
ss_status solve_t(OpImpl* op, const void* f, void* u, double tol, ss_precision prec, int32_t max_iter,
                  hipStream_t s, ss_solve_info* info) {
  WS w;
  SS_TRY(workspace(op, &w));
  Solver<NormT> sv;
  sv.op = op;
  sv.od = op->dev();
  sv.s = s;
  sv.per = (int)ceil_div((int64_t)op->work.size(), 8);
  sv.grid = (unsigned)(8 * sv.per);
  if (!op->h_pinned) SS_HIP(hipHostMalloc((void**)&op->h_pinned, 64, hipHostMallocDefault));
  sv.h_active = op->h_pinned;
  sv.d_active = (int*)(w.ps_in + op->n_prob);   // spare bytes of the workspace
  const int64_t n = op->n_exec;
  const OpDev od = sv.od;
  const double tol2 = tol * tol;
  auto t0 = std::chrono::steady_clock::now();

  k_gather_in<<<grid_for(n), kBlock, 0, s>>>(n, op->d_exec2canon, (const double2*)f, (const double2*)u, w.f64, w.x64);
  k_zero_k0<NormT><<<grid_for(n), kBlock, 0, s>>>(n, (const NormT*)op->d_norm, w.x64);
  k_init_state<<<grid_for(op->n_prob), kBlock, 0, s>>>(op->n_prob, w.ps, nullptr);
  int total_iters = 0, outer = 0;
  if (prec == SS_FP64) {
    k_mv<NormT, double2, MV_RESID><<<sv.grid, kBlock, 0, s>>>(od, w.x64, w.r64, w.f64, w.part_c, w.ps, sv.per);
    int it = 0;
    SS_TRY(sv.cg(w.x64, w.r64, w.p64, w.q64, w.ps, w.part_a, w.part_b, w.part_c, tol, max_iter, &it));
    total_iters = it;
  } else {
    // outer refinement loop; inner tolerance loose enough for FP32
    const double inner_tol = 1e-5;
    const int max_outer = 30;
    for (outer = 0; outer < max_outer; ++outer) {
      k_mv<NormT, double2, MV_RESID><<<sv.grid, kBlock, 0, s>>>(od, w.x64, w.r64, w.f64, w.part_c, w.ps, sv.per);
      k_resid_scalars<<<op->n_prob, kBlock, 0, s>>>(od, w.part_c, w.ps, tol2, 1);
      int act = 0;
      SS_TRY(sv.count_active(w.ps, &act));
      if (act == 0) break;
      k_init_state<<<grid_for(op->n_prob), kBlock, 0, s>>>(op->n_prob, w.ps_in, w.ps);
      k_refine_start<<<sv.grid, kBlock, 0, s>>>(od, w.r64, w.r32, w.x32, w.ps, sv.per);
      int it = 0;
      SS_TRY(sv.cg(w.x32, w.r32, w.p32, w.q32, w.ps_in, w.part_a, w.part_b, nullptr, inner_tol, max_iter, &it));
      total_iters += it;
      k_accum_iters<<<grid_for(op->n_prob), kBlock, 0, s>>>(op->n_prob, w.ps, w.ps_in);
      k_refine_add<<<sv.grid, kBlock, 0, s>>>(od, w.x64, w.x32, w.ps, sv.per);
    }
  }
  // final FP64 true residual of every problem (for the report and status)
  k_init_state<<<grid_for(op->n_prob), kBlock, 0, s>>>(op->n_prob, w.ps_in, nullptr);
  k_mv<NormT, double2, MV_RESID><<<sv.grid, kBlock, 0, s>>>(od, w.x64, w.r64, w.f64, w.part_c, w.ps_in, sv.per);
  k_resid_scalars<<<op->n_prob, kBlock, 0, s>>>(od, w.part_c, w.ps_in, tol2, 0);
  k_scatter_out<NormT><<<grid_for(n), kBlock, 0, s>>>(n, op->d_exec2canon, (const NormT*)op->d_norm, w.x64,
                                                      (double2*)u);
  std::vector<PState> hs(op->n_prob), hf(op->n_prob);
  SS_HIP(hipMemcpyAsync(hs.data(), w.ps, op->n_prob * sizeof(PState), hipMemcpyDeviceToHost, s));
  SS_HIP(hipMemcpyAsync(hf.data(), w.ps_in, op->n_prob * sizeof(PState), hipMemcpyDeviceToHost, s));
  SS_HIP(hipStreamSynchronize(s));
  const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  ss_status worst = SS_OK;
  for (int p = 0; p < op->n_prob; ++p) {
    const double rel = hf[p].ff > 0 ? std::sqrt(hf[p].rr / hf[p].ff) : 0.0;
    ss_status stp = SS_OK;
    if (hs[p].status == SS_EBREAKDOWN && !(rel <= tol)) stp = SS_EBREAKDOWN;
    else if (!(rel <= tol) && hf[p].ff > 0) stp = SS_ENOCONV;
    if (stp != SS_OK && worst == SS_OK) worst = stp;
    if (info) {
      ss_solve_info& in = info[p];
      in.iters = prec == SS_FP64 ? hs[p].iters : hs[p].total_iters;
      in.outer_steps = prec == SS_FP64 ? 0 : outer;
      in.rel_residual = rel;
      in.n = op->row_off[p + 1] - op->row_off[p];
      in.nnz = op->nnz_p[p];
      in.n_components = op->comps[p];
      in.status = stp;
      in.t_build_ms = 0;
      in.t_solve_ms = ms;
    }
  }
  if (worst == SS_ENOCONV) return fail(SS_ENOCONV, "tolerance not reached within max_iter");
  if (worst == SS_EBREAKDOWN) return fail(SS_EBREAKDOWN, "CG breakdown: <p, L p> <= 0 or not finite");
  return SS_OK;
}

}  // namespace

ss_status apply_impl(const OpImpl* op, ss_precision prec, const void* x, void* y, hipStream_t s) {
  const OpDev od = op->dev();
  const int per = (int)ceil_div((int64_t)op->work.size(), 8);
  const unsigned grid = (unsigned)(8 * per);
  if (prec == SS_FP64) {
    if (op->wide_norm)
      k_mv<int64_t, double2, MV_PLAIN><<<grid, kBlock, 0, s>>>(od, (const double2*)x, (double2*)y, nullptr, nullptr, nullptr, per);
    else
      k_mv<int32_t, double2, MV_PLAIN><<<grid, kBlock, 0, s>>>(od, (const double2*)x, (double2*)y, nullptr, nullptr, nullptr, per);
  } else {
    if (op->wide_norm)
      k_mv<int64_t, float2, MV_PLAIN><<<grid, kBlock, 0, s>>>(od, (const float2*)x, (float2*)y, nullptr, nullptr, nullptr, per);
    else
      k_mv<int32_t, float2, MV_PLAIN><<<grid, kBlock, 0, s>>>(od, (const float2*)x, (float2*)y, nullptr, nullptr, nullptr, per);
  }
  SS_HIP(hipGetLastError());
  return SS_OK;
}

ss_status solve_op_impl(OpImpl* op, const void* f, void* u, double tol, ss_precision prec, int32_t max_iter,
                        hipStream_t stream, ss_solve_info* info) {
  if (!f || !u) return fail(SS_EINVAL, "null vector");
  if (!(tol > 0) || max_iter < 1) return fail(SS_EINVAL, "tol must be > 0 and max_iter >= 1");
  if (prec != SS_FP64 && prec != SS_FP32_REFINE) return fail(SS_EINVAL, "unknown precision");
  return op->wide_norm ? solve_t<int64_t>(op, f, u, tol, prec, max_iter, stream, info)
                       : solve_t<int32_t>(op, f, u, tol, prec, max_iter, stream, info);
}

}  // namespace ss
