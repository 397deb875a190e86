// Exact proxy error of level-N solutions (Sec. 10.1, Lemma ProxyError): |f - L u^N|_2 / |f|_2
// with L untruncated.  L u^N lives on S^N + supp(a) = S^{N+1} (Prop. LExpansion), so with u^N
// extended by zero to S^{N+1} the norm is that of f - L_{N+1} u^N over S^{N+1}: one matvec of the
// level-(N+1) operator.  S^N sits inside S^{N+1} as the keys of first-appearance level <= N, in
// the same (lexicographic) order, so the extension is a stream compaction by level.
#include <hipcub/hipcub.hpp>

#include "ss_internal.h"

namespace ss {

namespace {

constexpr int kProxyBlock = 256;

// 1 where canonical row r of S^{N+1} is a key of S^N (first-appearance level below N + 1)
__global__ void k_proxy_flags(int64_t n, const uint8_t* __restrict__ lev, const int32_t* __restrict__ pid,
                              const int32_t* __restrict__ plevel, uint32_t* __restrict__ flag) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r < n) flag[r] = (int32_t)lev[r] < plevel[pid[r]] ? 1u : 0u;
}

// x in execution order of the level-(N+1) operator: u^N at the rows holding keys of S^N, else 0
__global__ void k_proxy_embed(int64_t n_exec, const int64_t* __restrict__ exec2canon,
                              const uint32_t* __restrict__ flag, const uint32_t* __restrict__ rank,
                              const double2* __restrict__ u, double2* __restrict__ x) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n_exec) return;
  const int64_t c = exec2canon[e];
  x[e] = c >= 0 && flag[c] ? u[rank[c]] : make_double2(0.0, 0.0);
}

// one block per problem: |f - y|^2 and |f|^2 over its execution rows, in a fixed order
__global__ __launch_bounds__(kProxyBlock) void k_proxy_sums(const int64_t* __restrict__ eoff,
                                                             const int64_t* __restrict__ exec2canon,
                                                             const double2* __restrict__ f,
                                                             const double2* __restrict__ y, double2* out) {
  const int p = blockIdx.x;
  const int64_t e0 = eoff[p], e1 = eoff[p + 1];
  double rr = 0, ff = 0;
  for (int64_t e = e0 + threadIdx.x; e < e1; e += kProxyBlock) {
    const int64_t c = exec2canon[e];
    const double2 fv = c >= 0 ? f[c] : make_double2(0.0, 0.0);
    const double2 yv = y[e];
    const double rx = fv.x - yv.x, ry = fv.y - yv.y;
    rr += rx * rx + ry * ry;
    ff += fv.x * fv.x + fv.y * fv.y;
  }
  __shared__ double s_rr[kProxyBlock], s_ff[kProxyBlock];
  s_rr[threadIdx.x] = rr;
  s_ff[threadIdx.x] = ff;
  __syncthreads();
  for (int h = kProxyBlock / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) {
      s_rr[threadIdx.x] += s_rr[threadIdx.x + h];
      s_ff[threadIdx.x] += s_ff[threadIdx.x + h];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) out[p] = make_double2(s_rr[0], s_ff[0]);
}

// device blocks of one call, returned to the pool after a stream sync
struct ProxyScratch {
  hipStream_t s;
  std::vector<void*> blocks;
  explicit ProxyScratch(hipStream_t st) : s(st) {}
  template <typename T>
  ss_status get(T** p, size_t n) {
    SS_TRY(dalloc(p, std::max<size_t>(n, 1)));
    blocks.push_back((void*)*p);
    return SS_OK;
  }
  ~ProxyScratch() {
    (void)hipStreamSynchronize(s);
    for (void* b : blocks) pool_free(b);
  }
};

inline unsigned grid_of(int64_t n) { return (unsigned)std::max<int64_t>(1, ceil_div(n, kProxyBlock)); }

}  // namespace

ss_status proxy_error_impl(const StampImpl* st, const OpImpl* op, const void* u, int64_t n_u, const double* f_hat,
                           double* err, hipStream_t s) {
  if (!st || !op || !u || !f_hat || !err) return fail(SS_EINVAL, "null argument");
  if (op->total != st->total || op->n_prob != st->n_prob)
    return fail(SS_EINVAL, "the operator was not built on this stamp");
  for (int p = 0; p < st->n_prob; ++p)
    if (st->level[p] < 1) return fail(SS_EINVAL, "the level-(N+1) stamp needs level >= 1 for every problem");
  const int64_t n = st->total, ne = op->n_exec;
  const int np = st->n_prob;
  ProxyScratch sc(s);
  uint32_t *flag = nullptr, *rank = nullptr;
  int32_t* plev = nullptr;
  double2 *f = nullptr, *x = nullptr, *y = nullptr, *sums = nullptr;
  SS_TRY(sc.get(&flag, n));
  SS_TRY(sc.get(&rank, n));
  SS_TRY(sc.get(&plev, np));
  SS_TRY(sc.get(&f, n));
  SS_TRY(sc.get(&x, ne));
  SS_TRY(sc.get(&y, ne));
  SS_TRY(sc.get(&sums, np));
  SS_HIP(h2d(plev, st->level.data(), np * sizeof(int32_t), s));
  k_proxy_flags<<<grid_of(n), kProxyBlock, 0, s>>>(n, st->d_lev, st->d_pid, plev, flag);
  size_t tb = 0;
  SS_HIP(hipcub::DeviceScan::ExclusiveSum(nullptr, tb, flag, rank, n, s));
  void* tmp = nullptr;
  SS_TRY(sc.get((char**)&tmp, tb));
  SS_HIP(hipcub::DeviceScan::ExclusiveSum(tmp, tb, flag, rank, n, s));
  // the keys of S^N number exactly the entries of u (else u belongs to other problems)
  uint32_t last[2] = {0, 0};
  SS_HIP(hipMemcpyAsync(&last[0], rank + (n - 1), 4, hipMemcpyDeviceToHost, s));
  SS_HIP(hipMemcpyAsync(&last[1], flag + (n - 1), 4, hipMemcpyDeviceToHost, s));
  SS_HIP(hipStreamSynchronize(s));
  if ((int64_t)last[0] + last[1] != n_u)
    return fail(SS_EINVAL, "u does not hold one entry per key of S^N of these problems");
  SS_TRY(stamp_forcing_impl(st, f_hat, f, s));
  k_proxy_embed<<<grid_of(ne), kProxyBlock, 0, s>>>(ne, op->d_exec2canon, flag, rank,
                                                     static_cast<const double2*>(u), x);
  SS_TRY(apply_impl(op, SS_FP64, x, y, s));
  k_proxy_sums<<<np, kProxyBlock, 0, s>>>(op->d_eoff, op->d_exec2canon, f, y, sums);
  SS_HIP(hipGetLastError());
  std::vector<double2> h(np);
  SS_HIP(hipMemcpyAsync(h.data(), sums, np * sizeof(double2), hipMemcpyDeviceToHost, s));
  SS_HIP(hipStreamSynchronize(s));
  for (int p = 0; p < np; ++p) err[p] = h[p].y > 0 ? std::sqrt(h[p].x / h[p].y) : 0.0;
  return SS_OK;
}

}  // namespace ss
