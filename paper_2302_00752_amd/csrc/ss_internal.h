// Internal declarations shared by the sparsespec translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <functional>
#include <string>
#include <vector>

#include "../../include/sparsespec.h"

namespace ss {

// ------------------------------------------------------------------ errors
void set_error(const std::string& msg);
const char* last_error_cstr();
ss_status fail(ss_status st, const std::string& msg);

#define SS_HIP(call)                                                               \
  do {                                                                             \
    hipError_t e_ = (call);                                                        \
    if (e_ != hipSuccess)                                                          \
      return ::ss::fail(e_ == hipErrorOutOfMemory ? SS_ENOMEM : SS_EDEVICE,        \
                        std::string(#call) + ": " + hipGetErrorString(e_));        \
  } while (0)

#define SS_TRY(expr)                 \
  do {                               \
    ss_status s_ = (expr);           \
    if (s_ != SS_OK) return s_;      \
  } while (0)

// ------------------------------------------------------------------ limits
constexpr int kJBits = 7;             // bits of an a-table index
constexpr int kTab = 1 << kJBits;     // per-problem stride of the a-tables (coefficients, |w|^2)
constexpr int kMaxA = kTab - 1;       // a-table entries per problem (index kTab - 1 = null entry)
constexpr int kNullJ = kTab - 1;
constexpr uint32_t kJMask = kTab - 1;
constexpr int kColBits = 32 - kJBits; // execution-layout column bits in a packed entry
constexpr uint32_t kColMask = (1u << kColBits) - 1;
constexpr int kSlice = 64;            // SELL slice height = wavefront size
constexpr int kBlock = 256;           // threads per block (4 wavefronts)
constexpr int kSlicesPerBlock = kBlock / kSlice;
constexpr int kSolveBlock = 512;      // threads per block of the matvec / CG kernels (8 wavefronts)
constexpr int kSolveWaves = kSolveBlock / kSlice;
constexpr int kWinRows = 2048;        // rows of x / |k|^2 a block stages in LDS
constexpr int kMaxItemSlices = 64;    // slices per work item (window items)
constexpr int kUnitEntries = 15936;   // SELL entries of a class-resident solve unit kept in LDS
constexpr int64_t kMaxRowsPerProblem = (1 << 22) - 1;
constexpr int kMaxProblems = (1 << 14) - 1;

// hash-slot encoding
// Build hash table: one word per slot.  MAIN: a key of an earlier level, its index (bits 0-30)
// and fingerprint = hash >> 33 (bits 31-61); CAND: a candidate of the level being built,
// (frontier key << kJBits) | a-table index in bits 0-61.  0 = empty.
constexpr uint64_t kTagMain = 1ull << 62;
constexpr uint64_t kTagCand = 2ull << 62;
constexpr uint64_t kTagMask = 3ull << 62;
constexpr uint64_t kIdxMask = ~kTagMask;
constexpr uint64_t kMainIdxMask = 0x7fffffffull;
__host__ __device__ inline uint64_t main_word(uint64_t h, uint64_t idx) { return kTagMain | (h >> 33 << 31) | idx; }
__host__ __device__ inline bool main_fp_eq(uint64_t v, uint64_t h) { return ((v >> 31) & 0x7fffffffull) == (h >> 33); }
constexpr uint32_t kNoSlot = 0xffffffffu;

// a == b + sign * w over d int16 coordinates, in int arithmetic (no wrap-around).  No early
// exit: every load is independent, so a wavefront keeps all of them in flight at once.
__device__ inline bool key_eq_shift(const int16_t* __restrict__ a, const int16_t* __restrict__ b,
                                    const int16_t* __restrict__ w, int sign, int d) {
  int acc = 0;
#pragma unroll 8
  for (int t = 0; t < d; ++t) acc |= (int)a[t] ^ ((int)b[t] + sign * (int)w[t]);
  return acc == 0;
}
// b1 + w1 == b2 + w2
__device__ inline bool key_eq_shift2(const int16_t* __restrict__ b1, const int16_t* __restrict__ w1,
                                     const int16_t* __restrict__ b2, const int16_t* __restrict__ w2, int d) {
  int acc = 0;
#pragma unroll 8
  for (int t = 0; t < d; ++t) acc |= ((int)b1[t] + (int)w1[t]) ^ ((int)b2[t] + (int)w2[t]);
  return acc == 0;
}

// Linear probing inside one problem's power-of-two table region [base, base + mask + 1) (at least
// 64 slots).  The first probe slot is the top log2(region) bits of the key's hash, a sum of
// coordinate x random odd coefficient products mod 2^64 (multiply-shift hashing: its high bits
// are evenly spread, and h(k - w) = h(k) - h(w) gives a neighbour's slot with one subtraction).
__host__ __device__ inline int slot_shift(uint64_t mask) { return __builtin_clzll(mask); }
__host__ __device__ inline uint64_t slot_first(uint64_t h, uint64_t base, uint64_t mask) {
  return base + (h >> slot_shift(mask));
}
// a lookup-table word: the key's fingerprint (hash >> 33, as in the build table) in the high half and
// its canonical index + 1 in the low half
__host__ __device__ inline uint64_t lslot_from_fp(uint64_t fp, uint64_t idx) { return (fp << 32) | (idx + 1); }
__host__ __device__ inline bool lslot_fp_eq(uint64_t v, uint64_t h) { return (v >> 32) == (h >> 33); }
__host__ __device__ inline int64_t lslot_idx(uint64_t v) { return (int64_t)(v & 0xffffffffull) - 1; }

__host__ __device__ inline uint64_t slot_next(uint64_t pos, uint64_t base, uint64_t mask) {
  return base + ((pos - base + 1) & mask);
}

// Rank-1 lattice values (Sec. 8, Definition of a reconstructing rank-1 lattice): k . z mod M with
// the prime M = 2^61 - 1 and z drawn uniformly from [1, M - 1]^d.  The map is linear,
// lat(k - w) = lat(k) - lat(w) mod M, so the value of a neighbour k - w_j follows from two stored
// values without reading a key; two distinct keys share a value with probability 1 / M over z
// (Lemma RandomRank1Lattice's argument).
constexpr uint64_t kLatM = (uint64_t(1) << 61) - 1;
__host__ __device__ inline uint64_t lat_fold(uint64_t r) {   // r < 2^63 -> r mod M
  r = (r & kLatM) + (r >> 61);
  return r >= kLatM ? r - kLatM : r;
}
__host__ __device__ inline uint64_t lat_mulmod(uint64_t a, uint64_t b) {   // a, b < M
  const unsigned __int128 p = (unsigned __int128)a * b;                    // < 2^122
  const uint64_t hi = (uint64_t)(p >> 64), lo = (uint64_t)p;               // 2^64 = 8 mod M
  return lat_fold((hi << 3) + (lo & kLatM) + (lo >> 61));
}
__host__ __device__ inline uint64_t lat_add(uint64_t a, uint64_t b) { return lat_fold(a + b); }
__host__ __device__ inline uint64_t lat_sub(uint64_t a, uint64_t b) { return lat_fold(a + (kLatM - b)); }
__host__ __device__ inline uint64_t lat_of_coord(int v) { return v >= 0 ? (uint64_t)v : kLatM - (uint64_t)(-v); }
// k . z mod M of a key with int16 coordinates, accumulated without a 128-bit product per
// coordinate: with z_t = zh_t 2^31 + zl_t (zl_t < 2^31, zh_t < 2^30) the sums lo = sum k_t zl_t
// and hi = sum k_t zh_t are exact in int64 for d <= 1024, and since 2^61 = 1 mod M,
// hi 2^31 = (hi >> 30) 2^61 + (hi mod 2^30) 2^31 = (hi >> 30) + (hi mod 2^30) 2^31 (mod M).
// Partial sums over different coordinates add (lanes of a wavefront combine theirs).
struct LatAcc {
  int64_t lo = 0, hi = 0;
  __host__ __device__ void add(int v, uint64_t z) {
    lo += (int64_t)v * (int64_t)(int32_t)(z & 0x7fffffffu);
    hi += (int64_t)v * (int64_t)(int32_t)(z >> 31);
  }
  __host__ __device__ uint64_t value() const {
    int64_t t = (hi >> 30) + ((hi & ((int64_t(1) << 30) - 1)) << 31) + lo;   // |t| < 2^62
    if (t < 0) t += (int64_t)kLatM;
    if (t >= (int64_t)kLatM) t -= (int64_t)kLatM;
    return (uint64_t)t;
  }
};

inline uint64_t splitmix64(uint64_t x) {
  x += 0x9e3779b97f4a7c15ULL;
  x = (x ^ (x >> 30)) * 0xbf58476d1ce4e5b9ULL;
  x = (x ^ (x >> 27)) * 0x94d049bb133111ebULL;
  return x ^ (x >> 31);
}

// ------------------------------------------------------------------ objects
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};

// A batch of stamping sets, keys in canonical order.
struct StampImpl {
  int device = 0;
  int32_t d = 0;
  int32_t n_prob = 0;
  std::vector<int32_t> level;
  // canonical a-tables (host): per problem s entries, lexicographic
  std::vector<int32_t> a_off;          // [n_prob+1] offsets into a_keys (entries)
  std::vector<int16_t> a_keys;         // [sum s x d]
  std::vector<int32_t> a_zero;         // index of w = 0 in each problem's table
  int32_t* d_azero = nullptr;          // [n_prob]
  // device: a-tables
  int16_t* d_akeys = nullptr;          // [sum s x d]
  uint64_t* d_ahash = nullptr;         // [sum s] linear hash (no problem term)
  int64_t* d_anorm = nullptr;          // [sum s] |w|^2
  int32_t* d_aoff = nullptr;           // [n_prob+1]
  // keys, canonical order, grouped by problem
  int64_t total = 0;
  std::vector<int64_t> row_off;        // [n_prob+1]
  int16_t* d_keys = nullptr;           // [total x d]
  uint8_t* d_lev = nullptr;            // [total]
  int64_t* d_norm = nullptr;           // [total] |k|^2
  uint64_t* d_hash = nullptr;          // [total] linear hash of the key
  int32_t* d_pid = nullptr;            // [total]
  int64_t* d_root = nullptr;           // [total] canonical slot of the forcing key the first path started at
  int64_t* d_rowoff = nullptr;         // [n_prob+1]
  int64_t n_f = 0;                     // forcing frequencies given to the build (all problems)
  uint32_t* d_fslot = nullptr;         // [n_f] canonical slot of each, in the order given
  uint64_t* d_coef = nullptr;          // [d] hash multipliers
  uint64_t* d_latz = nullptr;          // [d] rank-1 lattice generating vector (entries in [1, M - 1])
  uint64_t* d_lat = nullptr;           // [total] lattice value k . z mod M of every key
  uint64_t* d_alat = nullptr;          // [sum s] lattice value of every a-table entry
  void* d_upload = nullptr;            // one block holding d_akeys .. d_alat and d_coef, d_latz (views)
  uint64_t* d_table = nullptr;         // build only: one word per slot (MAIN / CAND words)
  uint64_t* d_ltable = nullptr;        // lookups: one word per slot, the same positions:
                                       // (hash >> 32) << 32 | (canonical index + 1), 0 = empty
  int64_t* d_toff = nullptr;           // [n_prob] first slot of each problem's region
  uint64_t* d_tmask = nullptr;         // [n_prob] region size - 1 (a view: d_toff + n_prob)
  uint64_t n_slots = 0;
  std::vector<uint64_t> tcap;
  int64_t max_norm = 0;
};

// Per-problem solver state (device).  A field written by one kernel of an
// iteration is read only by later kernels.
struct PState {
  double rho[2];        // <r, D^-1 r>, indexed by iteration parity
  double ff;            // |rhs|^2 of the current CG run (|f|^2 for FP64 / outer)
  double rr;            // |r|^2 of the current residual
  double scale;         // refinement: |r64| that normalises the FP32 right-hand side
  double tin2;          // refinement, inner state: squared relative stop of the running correction solve
  int32_t iter;         // index of the running iteration (read by update / dir)
  int32_t iters;        // completed iterations of the current CG run
  int32_t done;
  int32_t status;
  int32_t total_iters;  // refinement: iterations of finished correction solves
  int32_t outer;        // refinement steps taken
  int32_t start;        // a CG run is to be started this tick
  int32_t pending;      // refinement: a finished correction awaits the FP64 update
};

// Plain-old-data view of an operator passed to kernels by value.
struct OpDev {
  const uint32_t* sent;      // SELL entries: local exec column | j << kColBits
  const uint32_t* sptr;      // [n_slices+1] entry offset of each slice
  const void* norm;          // [n_exec] |k|^2 per exec row (int32 or int64)
  const int64_t* eoff;       // [n_prob+1] first exec row of each problem
  const int4* work;          // [n_work] {problem, first slice, slices, 0}
  const int2* wrange;        // [n_prob] {first work item, end work item}
  const double2* A64;        // [n_prob x 64] 2 pi^2 a_j (index 63 = 0)
  const float2* A32;         // [n_prob x 64]
  const int64_t* nu;         // [n_prob x 64] |w_j|^2
  const double* a0;          // [n_prob] a_0 (real)
  int32_t n_work;
  int32_t n_prob;
};

struct LaunchList;

struct OpImpl {
  int device = 0;
  int32_t n_prob = 0;
  int32_t d = 0;
  int64_t total = 0;                   // canonical rows
  int64_t n_exec = 0;                  // padded execution rows
  int64_t nnz = 0;
  int64_t n_components = 0;
  int64_t n_slices = 0;
  int64_t n_sell = 0;                  // stored SELL entries (incl. padding)
  bool wide_norm = false;              // |k|^2 needs int64
  std::vector<int64_t> row_off;        // canonical offsets [n_prob+1]
  std::vector<int64_t> eoff;           // exec offsets [n_prob+1]
  std::vector<int32_t> comps;          // classes per problem
  std::vector<int64_t> cls_e0;         // first global exec row of every class, in exec order
  std::vector<int64_t> cls_n;          // rows of every class
  std::vector<int64_t> nnz_p;          // per problem
  std::vector<int4> work;               // {problem, first slice, slices | window rows << 16, window start row}
  std::vector<int2> wrange;
  int64_t max_window = 0;
  // class-resident solve units: runs of whole slices that start and end on class boundaries,
  // at most kWinRows rows: {problem, first slice, slices, first exec row (problem-local)}.
  // urange[p] = [first, end) unit of problem p, or {-1, -1} when its classes do not split so.
  std::vector<int4> units;
  std::vector<int2> urange;
  std::vector<int32_t> unit_entries;   // SELL entries of each unit
  std::vector<uint32_t> unit_ebase;    // first SELL entry of each unit
  int4* d_units = nullptr;
  int32_t* d_comp = nullptr;           // [total] local class label
  // execution layout
  int64_t* d_exec2canon = nullptr;     // [n_exec] global canonical or -1
  int64_t* d_canon2exec = nullptr;     // [total]
  uint32_t* d_sent = nullptr;
  uint32_t* d_sptr = nullptr;
  void* d_norm = nullptr;
  int64_t* d_eoff = nullptr;
  int4* d_work = nullptr;
  int2* d_wrange = nullptr;
  double2* d_A64 = nullptr;
  float2* d_A32 = nullptr;
  int64_t* d_nu = nullptr;
  double* d_a0 = nullptr;
  void* d_upload[2] = {nullptr, nullptr};   // blocks holding d_eoff, then d_units .. d_a0 (views)
  // solver workspace (lazily allocated, reused)
  struct Work {
    size_t bytes = 0;
    void* base = nullptr;
  } ws;
  int* h_pinned = nullptr;             // pinned host word for convergence polling
  std::vector<double> a0_host;         // a_0 per problem
  bool busy = false;                   // a solve of this operator is in flight
  struct ApplyCache {
    LaunchList* list = nullptr;
    const void* x = nullptr;
    void* y = nullptr;
    ss_precision prec = SS_FP64;
  } apply_cache;
  OpDev dev() const;
};

struct EngineImpl;
ss_status engine_create(int64_t budget, int32_t max_slots, hipStream_t s, EngineImpl** out);
void engine_free(EngineImpl* e);
ss_status engine_submit(EngineImpl* e, OpImpl* op, const void* f, void* u, double tol, ss_precision prec,
                        int32_t max_iter, int64_t tag);
ss_status engine_step(EngineImpl* e, int32_t iters, int32_t* n_active);
ss_status engine_poll(EngineImpl* e, int32_t cap, int64_t* tags, int32_t* probs, ss_solve_info* info,
                      int32_t* n_out);
ss_status engine_usage(const EngineImpl* e, int32_t* n_active, int64_t* bytes);
int64_t op_device_bytes(const OpImpl* op);
void free_apply_cache(OpImpl* op);

// ------------------------------------------------------------------ entry points (internal)
ss_status build_stamp_impl(int32_t n_prob, int32_t d, const int32_t* n_a, const int16_t* a_freqs,
                           const int32_t* n_f, const int16_t* f_freqs, const int32_t* level,
                           hipStream_t stream, StampImpl** out);
void free_stamp_impl(StampImpl* st);
// prob >= 0: all queries of that problem, local slots out; prob < 0: per-query
// problem ids in probs (host), global slots out.
ss_status stamp_lookup_impl(const StampImpl* st, int32_t prob, int64_t nq, const int16_t* q,
                            int64_t* slot_out, hipStream_t stream, const int32_t* probs = nullptr);

ss_status stamp_forcing_impl(const StampImpl* st, const double* f_hat, void* f, hipStream_t stream);
ss_status lattice_modulus_impl(int64_t K, int64_t n, double sigma, int64_t* M);
ss_status stamp_lattice_impl(const StampImpl* st, const int64_t* z, int64_t M, int64_t* values,
                             int32_t* reconstructing, hipStream_t s);
// proxy error of level-N solutions u (canonical order of the level-N stamp) from the stamp and
// operator built at level N + 1 (proxy.hip); err: host [n_prob]
struct AdrImpl;
ss_status adr_build_impl(const StampImpl* st, const OpImpl* op, const int32_t* n_b, const int16_t* b_freqs,
                         const double* b_hat, const int32_t* n_c, const int16_t* c_freqs, const double* c_hat,
                         hipStream_t s, AdrImpl** out);
ss_status adr_apply_impl(const AdrImpl* A, const void* x, void* y, hipStream_t s);
ss_status adr_solve_impl(const AdrImpl* A, const void* f, void* u, double tol, int32_t max_iter, hipStream_t s,
                         ss_solve_info* info);
void adr_free_impl(AdrImpl* A);
struct DirectStats {
  double factor_ms = 0;    // factorisation kernels (all tile columns), summed over chunks
  int64_t tiles = 0;       // lower 32 x 32 tiles factored
  int32_t chunks = 0;      // chunks of classes the workspace budget split the batch into
  int32_t refine_steps = 0;    // substitution steps of the chunk that needed most
  double rel_residual = 0;     // max over classes of |f_c - L u_c| / |f_c|
};
ss_status direct_solve_impl(const OpImpl* op, const void* f_dev, void* u_dev, ss_precision prec, double tol,
                            hipStream_t s, DirectStats* stats);
ss_status proxy_error_impl(const StampImpl* st, const OpImpl* op, const void* u, int64_t n_u, const double* f_hat,
                           double* err, hipStream_t stream);

// whole-path batch solve, split into concurrently running parts
struct BatchImpl {
  struct Part {
    int p0 = 0, p1 = 0;              // problems [p0, p1)
    int64_t n = 0;                   // rows of the part
    std::vector<int64_t> off;        // part-local problem offsets [p1 - p0 + 1]
    double2* u = nullptr;            // device, canonical order
  };
  int32_t n_prob = 0, d = 0;
  int device = 0;
  std::vector<Part> parts;
  std::vector<int64_t> offsets;      // [n_prob + 1] batch-global canonical offsets
};
ss_status batch_solve_impl(int32_t n_prob, int32_t d, const int32_t* n_a, const int16_t* a_freqs,
                           const double* a_hat, const int32_t* n_f, const int16_t* f_freqs, const double* f_hat,
                           const int32_t* level, double tol, ss_precision prec, int32_t max_iter, uint32_t flags,
                           int32_t n_parts, ss_solve_info* info, BatchImpl** out);
ss_status batch_solution_impl(const BatchImpl* b, void* u, hipStream_t stream);
void free_batch_impl(BatchImpl* b);

ss_status build_op_impl(const StampImpl* st, const int32_t* n_a, const int16_t* a_freqs,
                        const double* a_hat, uint32_t flags, hipStream_t stream, OpImpl** out);
void free_op_impl(OpImpl* op);

ss_status apply_impl(const OpImpl* op, ss_precision prec, const void* x, void* y,
                     hipStream_t stream);
ss_status solve_op_impl(OpImpl* op, const void* f, void* u, double tol, ss_precision prec,
                        int32_t max_iter, hipStream_t stream, ss_solve_info* info);
// the class-resident solve with its tables in a fixed device array (no allocation)
ss_status solve_op_noalloc_impl(OpImpl* op, const void* f, void* u, double tol, ss_precision prec,
                                int32_t max_iter, hipStream_t stream, ss_solve_info* info);

// host-side canonicalisation of a-support (shared by stamp and op builders)
// |x + iy|: the plain formula where the squares cannot overflow or underflow to zero
// (std::hypot's rescaling costs more than the rest of the host-side table work)
inline double cabs2d(double x, double y) {
  const double m = std::max(std::fabs(x), std::fabs(y));
  if (m == 0) return 0;
  if (m < 1e150 && m > 1e-150) return std::sqrt(x * x + y * y);
  return std::hypot(x, y);
}

struct ATable {
  int d = 0;
  std::vector<int16_t> keys;   // [size x d], lexicographic
  std::vector<double2> coef;   // one per key (1 when only the support was given)
  int zero = -1;               // index of w = 0
  int size() const { return d ? (int)(keys.size() / d) : 0; }
  const int16_t* key(int j) const { return keys.data() + (size_t)j * d; }
};
ss_status canonical_a(int32_t d, int32_t n_a, const int16_t* freqs, const double* coef,
                      bool drop_zero_coef, ATable* out);

// device memory: a caching allocator (see alloc.hip)
hipError_t pool_alloc(void** out, size_t bytes);
void pool_free(void* p);
// bytes in blocks handed out, bytes cached, and allocations taken from the driver so far (all devices)
void pool_stats(int64_t* live_bytes, int64_t* cached_bytes, int64_t* driver_allocs);
// pinned host memory for small result buffers, cached (see alloc.hip); released only after the
// stream that filled it has been synchronised
hipError_t pinned_alloc(void** out, size_t bytes);
void pinned_free(void* p);
// Host-to-device copy of `bytes` from pageable host memory, queued on `stream` without holding the
// calling thread: the bytes are first copied into a pinned buffer of the thread.
hipError_t h2d(void* dst, const void* src, size_t bytes, hipStream_t stream);

template <typename T>
ss_status dalloc(T** p, size_t count) {
  *p = nullptr;
  if (count == 0) count = 1;
  hipError_t e = pool_alloc((void**)p, count * sizeof(T));
  if (e != hipSuccess) {
    *p = nullptr;
    return fail(e == hipErrorOutOfMemory ? SS_ENOMEM : SS_EDEVICE,
                std::string("device allocation: ") + hipGetErrorString(e));
  }
  return SS_OK;
}
template <typename T>
void dfree(T*& p) {
  pool_free((void*)p);
  p = nullptr;
}

// Device-to-host reads that end in a stream synchronisation, staged through the calling thread's
// pinned buffer: a read into pageable memory is staged by the runtime, and in the batch pipeline
// one part's read could wait for milliseconds behind another part's stream.  add() queues a copy
// on `stream`; sync() synchronises the stream and moves every staged copy to its destination.
// One Readback is in use per thread at a time.
struct Readback {
  hipStream_t stream;
  explicit Readback(hipStream_t s) : stream(s) {}
  ss_status add(void* dst, const void* src, size_t bytes);
  ss_status sync();

 private:
  struct Part {
    void* dst;
    size_t off, bytes;
  };
  std::vector<Part> parts;
  size_t used = 0;
};

// Small host arrays sent to the device in one transfer: every array gets a 256-byte aligned slice
// of one pooled device block, and the arrays are staged side by side in the thread's pinned
// buffer, so a build phase pays one copy (and one host call) instead of one per array.  The block
// belongs to the caller (released with pool_free); the slices are views into it and are never
// freed on their own.
struct Upload {
  struct Piece {
    std::function<void(char*)> point;   // sets the caller's device pointer to its slice
    const void* host;
    size_t bytes;
  };
  std::vector<Piece> pieces;
  template <typename T>
  void add(T** dev, const T* host, size_t count) {
    pieces.push_back(Piece{[dev](char* q) { *dev = reinterpret_cast<T*>(q); }, host, count * sizeof(T)});
  }
  // allocates the block into *block, points every slice into it and queues the copy on `stream`
  ss_status commit(void** block, hipStream_t stream);
};

__host__ __device__ inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// XCD-aware block numbering: the hardware deals blocks to the 8 XCDs round-robin;
// renumbering so each XCD gets a contiguous eighth of the logical blocks keeps the
// data of neighbouring blocks (one problem's table region, keys, CSR) in one L2.
// Launch with xcd_grid(n) blocks; a block whose logical index is >= n exits.
inline unsigned xcd_grid(int64_t nblocks) { return (unsigned)(8 * ceil_div(nblocks, 8)); }
__device__ inline int64_t xcd_block(int64_t nblocks) {
  const int64_t per = (nblocks + 7) / 8;
  return (int64_t)(blockIdx.x & 7) * per + (blockIdx.x >> 3);
}
// The global thread index under that numbering, for a grid of xcd_grid(n) blocks (a multiple of 8,
// so the numbering is a bijection on the launched blocks); kernels check the index against their
// size as with plain numbering.  Work items of one problem lie together in most arrays, so
// consecutive blocks on one XCD keep a problem's gathers and scatters in that XCD's L2.
__device__ inline int64_t xcd_tid() { return xcd_block(gridDim.x) * blockDim.x + threadIdx.x; }

}  // namespace ss
