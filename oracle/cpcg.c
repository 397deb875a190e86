/*
 * Sparse FP64 Jacobi-preconditioned CG for the truncated Galerkin system, in plain C with
 * OpenMP: the timed CPU baseline.  Test infrastructure only (the benchmark's CPU leg and the
 * tests call it); it shares no code with the GPU library.
 *
 * For each problem of a batch, three phases, each timed:
 *   stamp  S^N[a](F) (Sec. 6, Eq. StampSet): S^0 = F and level n adds k + w for every key k of
 *          level n - 1 and every w in supp(a) not yet in the set (0 is in supp(a), so this is the
 *          Minkowski recursion); a hash set dedups.  Keys are then put in ascending lexicographic
 *          order of their signed coordinates (coordinate 0 most significant): the slot order.
 *   index  for every key k and every w in supp(a): the slot of l = k - w if l is in S^N (the
 *          finite operator sums over l in S^N only, Sec. 9, Eq. FiniteGalerkinOperator); the
 *          entry 4 pi^2 (k . l) a_{k-l} is formed from the definition (k . l in 64-bit integers)
 *          and stored in a CSR matrix.
 *   solve  Jacobi-preconditioned CG on L_N u = f with D_k = 4 pi^2 |k|^2 a_0 (the denominator of
 *          the recurrence in the proof of Prop. SolutionSupport), u_0 = 0 and the zero
 *          frequency's row left out (Prop. ExistenceUniquenessStability: f_0 = 0), stopped when
 *          |f - L u|_2 <= tol |f|_2 (recursively updated residual).
 * Problems are spread over the OpenMP threads (one problem per thread at a time).
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define CPCG_OK 0
#define CPCG_ENOMEM 2
#define CPCG_ERANGE 3
#define CPCG_ENOCONV 5

typedef struct {
  int64_t n;          /* |S^N| */
  int64_t nnz;        /* stored (k, l) pairs */
  int32_t iters;
  int32_t status;
  double rel_residual;
  double stamp_ms, index_ms, solve_ms, matvec_ms;   /* matvec_ms: one y = L x, mean of repetitions */
} cpcg_info;

/* ------------------------------------------------------------ key set (open addressing) */
typedef struct {
  int d;
  int64_t n, cap_keys;
  int16_t* keys;       /* [cap_keys x d] in insertion order */
  uint8_t* level;      /* [cap_keys] */
  int64_t* table;      /* [tsize] key index + 1, 0 = empty */
  int64_t tsize;
} keyset;

static uint64_t key_hash(const int16_t* k, int d) {
  uint64_t h = 0x9e3779b97f4a7c15ull;
  for (int t = 0; t < d; ++t) {
    h ^= (uint64_t)(uint16_t)k[t];
    h *= 0x100000001b3ull;
    h ^= h >> 29;
  }
  return h ^ (h >> 32);
}

static int keyset_init(keyset* s, int d, int64_t cap) {
  s->d = d;
  s->n = 0;
  s->cap_keys = cap < 16 ? 16 : cap;
  s->keys = (int16_t*)malloc((size_t)s->cap_keys * d * sizeof(int16_t));
  s->level = (uint8_t*)malloc((size_t)s->cap_keys);
  s->tsize = 64;
  while (s->tsize < 2 * s->cap_keys) s->tsize <<= 1;
  s->table = (int64_t*)calloc((size_t)s->tsize, sizeof(int64_t));
  return s->keys && s->level && s->table ? CPCG_OK : CPCG_ENOMEM;
}

static void keyset_free(keyset* s) {
  free(s->keys);
  free(s->level);
  free(s->table);
}

/* slot of key k in the table: the index of an equal key, or -1 (pos gets the empty slot) */
static int64_t keyset_find(const keyset* s, const int16_t* k, int64_t* pos) {
  const uint64_t mask = (uint64_t)s->tsize - 1;
  uint64_t p = key_hash(k, s->d) & mask;
  while (1) {
    const int64_t v = s->table[p];
    if (v == 0) {
      if (pos) *pos = (int64_t)p;
      return -1;
    }
    if (memcmp(s->keys + (v - 1) * s->d, k, (size_t)s->d * sizeof(int16_t)) == 0) return v - 1;
    p = (p + 1) & mask;
  }
}

static int keyset_grow(keyset* s) {
  const int64_t ncap = 2 * s->cap_keys;
  int16_t* nk = (int16_t*)realloc(s->keys, (size_t)ncap * s->d * sizeof(int16_t));
  if (!nk) return CPCG_ENOMEM;
  s->keys = nk;
  uint8_t* nl = (uint8_t*)realloc(s->level, (size_t)ncap);
  if (!nl) return CPCG_ENOMEM;
  s->level = nl;
  s->cap_keys = ncap;
  int64_t nts = s->tsize;
  while (nts < 2 * ncap) nts <<= 1;
  if (nts != s->tsize) {
    free(s->table);
    s->tsize = nts;
    s->table = (int64_t*)calloc((size_t)nts, sizeof(int64_t));
    if (!s->table) return CPCG_ENOMEM;
    for (int64_t i = 0; i < s->n; ++i) {
      int64_t pos = 0;
      keyset_find(s, s->keys + i * s->d, &pos);
      s->table[pos] = i + 1;
    }
  }
  return CPCG_OK;
}

/* insert k (if new) with level lev; returns 1 if inserted, 0 if present, < 0 on error */
static int keyset_add(keyset* s, const int16_t* k, int lev) {
  int64_t pos = 0;
  if (keyset_find(s, k, &pos) >= 0) return 0;
  if (s->n == s->cap_keys) {
    if (keyset_grow(s) != CPCG_OK) return -1;
    keyset_find(s, k, &pos);
  }
  memcpy(s->keys + s->n * s->d, k, (size_t)s->d * sizeof(int16_t));
  s->level[s->n] = (uint8_t)lev;
  s->table[pos] = s->n + 1;
  s->n++;
  return 1;
}

/* ------------------------------------------------------------ lexicographic order */
static _Thread_local const int16_t* g_sort_keys;
static _Thread_local int g_sort_d;

static int lex_cmp(const void* a, const void* b) {
  const int16_t* x = g_sort_keys + *(const int64_t*)a * g_sort_d;
  const int16_t* y = g_sort_keys + *(const int64_t*)b * g_sort_d;
  for (int t = 0; t < g_sort_d; ++t)
    if (x[t] != y[t]) return x[t] < y[t] ? -1 : 1;
  return 0;
}

/* ------------------------------------------------------------ one problem */
typedef struct {
  int64_t n, nnz;
  int64_t* row_ptr;   /* [n + 1] */
  int32_t* col;       /* [nnz] */
  double* val;        /* [2 nnz] interleaved complex */
  double* diag;       /* [n] Jacobi diagonal, 0 at k = 0 */
} csr;

static double now_ms(void) { return 1e3 * omp_get_wtime(); }

static void matvec(const csr* A, const double* x, double* y) {
  for (int64_t r = 0; r < A->n; ++r) {
    double sr = 0, si = 0;
    for (int64_t e = A->row_ptr[r]; e < A->row_ptr[r + 1]; ++e) {
      const double ar = A->val[2 * e], ai = A->val[2 * e + 1];
      const double xr = x[2 * A->col[e]], xi = x[2 * A->col[e] + 1];
      sr += ar * xr - ai * xi;
      si += ar * xi + ai * xr;
    }
    y[2 * r] = sr;
    y[2 * r + 1] = si;
  }
}

static int solve_one(int d, int n_a, const int16_t* af, const double* ah, int n_f, const int16_t* ff,
                     const double* fh, int level, double tol, int max_iter, int matvec_reps, double** u_keep,
                     cpcg_info* info) {
  const double pi = 3.14159265358979323846;
  const double four_pi2 = 4.0 * pi * pi;
  memset(info, 0, sizeof(*info));
  /* ---- stamp */
  double t0 = now_ms();
  keyset S;
  int64_t guess = n_f;
  for (int n = 0; n < level && guess < (1 << 20); ++n) guess *= n_a;
  if (keyset_init(&S, d, guess) != CPCG_OK) return CPCG_ENOMEM;
  int16_t* cand = (int16_t*)malloc((size_t)d * sizeof(int16_t));
  for (int i = 0; i < n_f; ++i)
    if (keyset_add(&S, ff + (int64_t)i * d, 0) < 0) return CPCG_ENOMEM;
  int64_t lo = 0, hi = S.n;
  for (int n = 1; n <= level; ++n) {
    for (int64_t i = lo; i < hi; ++i) {
      for (int j = 0; j < n_a; ++j) {
        const int16_t* w = af + (int64_t)j * d;
        int zero = 1;
        for (int t = 0; t < d; ++t) {
          const int v = (int)S.keys[i * d + t] + (int)w[t];
          if (v < -32768 || v > 32767) {
            free(cand);
            keyset_free(&S);
            return CPCG_ERANGE;
          }
          cand[t] = (int16_t)v;
          zero &= w[t] == 0;
        }
        if (zero) continue;
        if (keyset_add(&S, cand, n) < 0) return CPCG_ENOMEM;
      }
    }
    lo = hi;
    hi = S.n;
  }
  const int64_t n = S.n;
  int64_t* order = (int64_t*)malloc((size_t)n * sizeof(int64_t));
  for (int64_t i = 0; i < n; ++i) order[i] = i;
  g_sort_keys = S.keys;
  g_sort_d = d;
  qsort(order, (size_t)n, sizeof(int64_t), lex_cmp);
  int16_t* keys = (int16_t*)malloc((size_t)n * d * sizeof(int16_t));
  for (int64_t r = 0; r < n; ++r) memcpy(keys + r * d, S.keys + order[r] * d, (size_t)d * sizeof(int16_t));
  /* re-index the hash set to canonical slots */
  memset(S.table, 0, (size_t)S.tsize * sizeof(int64_t));
  memcpy(S.keys, keys, (size_t)n * d * sizeof(int16_t));
  for (int64_t r = 0; r < n; ++r) {
    int64_t pos = 0;
    keyset_find(&S, S.keys + r * d, &pos);
    S.table[pos] = r + 1;
  }
  double t1 = now_ms();
  info->stamp_ms = t1 - t0;
  /* ---- index: neighbours and entries */
  int64_t a0_idx = -1;
  for (int j = 0; j < n_a; ++j) {
    int zero = 1;
    for (int t = 0; t < d; ++t) zero &= af[(int64_t)j * d + t] == 0;
    if (zero) a0_idx = j;
  }
  csr A;
  A.n = n;
  A.row_ptr = (int64_t*)malloc((size_t)(n + 1) * sizeof(int64_t));
  A.col = (int32_t*)malloc((size_t)n * n_a * sizeof(int32_t));
  A.val = (double*)malloc((size_t)n * n_a * 2 * sizeof(double));
  A.diag = (double*)malloc((size_t)n * sizeof(double));
  if (!A.row_ptr || !A.col || !A.val || !A.diag || a0_idx < 0) return CPCG_ENOMEM;
  const double a0 = ah[2 * a0_idx];
  int64_t e = 0;
  for (int64_t r = 0; r < n; ++r) {
    A.row_ptr[r] = e;
    const int16_t* k = keys + r * d;
    int64_t kk = 0;
    for (int t = 0; t < d; ++t) kk += (int64_t)k[t] * k[t];
    A.diag[r] = four_pi2 * (double)kk * a0;
    for (int j = 0; j < n_a; ++j) {
      const int16_t* w = af + (int64_t)j * d;
      int ok = 1;
      for (int t = 0; t < d; ++t) {
        const int v = (int)k[t] - (int)w[t];
        if (v < -32768 || v > 32767) ok = 0;
        cand[t] = (int16_t)v;
      }
      if (!ok) continue;
      const int64_t c = keyset_find(&S, cand, NULL);
      if (c < 0) continue;
      int64_t kl = 0;
      for (int t = 0; t < d; ++t) kl += (int64_t)k[t] * cand[t];
      A.col[e] = (int32_t)c;
      A.val[2 * e] = four_pi2 * (double)kl * ah[2 * j];
      A.val[2 * e + 1] = four_pi2 * (double)kl * ah[2 * j + 1];
      ++e;
    }
  }
  A.row_ptr[n] = e;
  A.nnz = e;
  double t2 = now_ms();
  info->index_ms = t2 - t1;
  /* ---- right-hand side at the forcing slots */
  double* f = (double*)calloc((size_t)2 * n, sizeof(double));
  double* x = (double*)calloc((size_t)2 * n, sizeof(double));
  double* r = (double*)malloc((size_t)2 * n * sizeof(double));
  double* z = (double*)malloc((size_t)2 * n * sizeof(double));
  double* p = (double*)malloc((size_t)2 * n * sizeof(double));
  double* q = (double*)malloc((size_t)2 * n * sizeof(double));
  for (int i = 0; i < n_f; ++i) {
    const int64_t s = keyset_find(&S, ff + (int64_t)i * d, NULL);
    f[2 * s] = fh[2 * i];
    f[2 * s + 1] = fh[2 * i + 1];
  }
  /* ---- Jacobi-preconditioned CG, x = 0 to start */
  double ff2 = 0;
  for (int64_t i = 0; i < 2 * n; ++i) ff2 += f[i] * f[i];
  memcpy(r, f, (size_t)2 * n * sizeof(double));
  double rho = 0, rr = ff2;
  for (int64_t i = 0; i < n; ++i) {
    const double inv = A.diag[i] > 0 ? 1.0 / A.diag[i] : 0.0;
    z[2 * i] = inv * r[2 * i];
    z[2 * i + 1] = inv * r[2 * i + 1];
    rho += r[2 * i] * z[2 * i] + r[2 * i + 1] * z[2 * i + 1];
  }
  memcpy(p, z, (size_t)2 * n * sizeof(double));
  int it = 0, status = CPCG_OK;
  const double thr2 = tol * tol * ff2;
  while (rr > thr2) {
    if (it >= max_iter) {
      status = CPCG_ENOCONV;
      break;
    }
    matvec(&A, p, q);
    double pq = 0;
    for (int64_t i = 0; i < 2 * n; ++i) pq += p[i] * q[i];   /* <p, L p> is real */
    const double alpha = rho / pq;
    double rho1 = 0;
    rr = 0;
    for (int64_t i = 0; i < n; ++i) {
      x[2 * i] += alpha * p[2 * i];
      x[2 * i + 1] += alpha * p[2 * i + 1];
      r[2 * i] -= alpha * q[2 * i];
      r[2 * i + 1] -= alpha * q[2 * i + 1];
      const double inv = A.diag[i] > 0 ? 1.0 / A.diag[i] : 0.0;
      z[2 * i] = inv * r[2 * i];
      z[2 * i + 1] = inv * r[2 * i + 1];
      rho1 += r[2 * i] * z[2 * i] + r[2 * i + 1] * z[2 * i + 1];
      rr += r[2 * i] * r[2 * i] + r[2 * i + 1] * r[2 * i + 1];
    }
    const double beta = rho1 / rho;
    rho = rho1;
    for (int64_t i = 0; i < 2 * n; ++i) p[i] = z[i] + beta * p[i];
    ++it;
  }
  double t3 = now_ms();
  info->solve_ms = t3 - t2;
  /* the true residual of the result */
  matvec(&A, x, q);
  double res2 = 0;
  for (int64_t i = 0; i < 2 * n; ++i) res2 += (f[i] - q[i]) * (f[i] - q[i]);
  info->rel_residual = ff2 > 0 ? sqrt(res2 / ff2) : 0.0;
  if (matvec_reps > 0) {
    const double tm = now_ms();
    for (int k = 0; k < matvec_reps; ++k) matvec(&A, x, q);
    info->matvec_ms = (now_ms() - tm) / matvec_reps;
  }
  info->n = n;
  info->nnz = A.nnz;
  info->iters = it;
  info->status = status;
  free(f);
  if (u_keep) *u_keep = x;   /* the caller takes the solution */
  else free(x);
  free(r);
  free(z);
  free(p);
  free(q);
  free(A.row_ptr);
  free(A.col);
  free(A.val);
  free(A.diag);
  free(order);
  free(keys);
  free(cand);
  keyset_free(&S);
  return status;
}

/*
 * cpcg_solve_batch -- solve n_prob problems of dimension d on n_threads OpenMP threads.
 *   n_a[p], a_freqs [sum n_a x d], a_hat [2 sum n_a]: supp(a_p) closed under negation with 0,
 *     and its coefficients (interleaved complex), problems concatenated.
 *   n_f[p], f_freqs, f_hat: F_p and f_hat on it.  level[p]: the stamping level.
 *   u_out (nullable): concatenated solutions in canonical order; u_off [n_prob + 1] (nullable with
 *     it) receives each problem's first entry; u_cap: complex entries available.
 *   info [n_prob]: per-problem sizes, iterations, residual, phase times.
 *   *threads_used: threads of the parallel team.
 * Returns 0, or the first non-zero per-problem status.
 */
int cpcg_solve_batch(int n_prob, int d, const int32_t* n_a, const int16_t* a_freqs, const double* a_hat,
                     const int32_t* n_f, const int16_t* f_freqs, const double* f_hat, const int32_t* level,
                     double tol, int max_iter, int n_threads, int matvec_reps, double* u_out, int64_t* u_off,
                     int64_t u_cap, cpcg_info* info, int* threads_used) {
  int64_t* a_off = (int64_t*)malloc((size_t)(n_prob + 1) * sizeof(int64_t));
  int64_t* f_off = (int64_t*)malloc((size_t)(n_prob + 1) * sizeof(int64_t));
  a_off[0] = f_off[0] = 0;
  for (int p = 0; p < n_prob; ++p) {
    a_off[p + 1] = a_off[p] + n_a[p];
    f_off[p + 1] = f_off[p] + n_f[p];
  }
  int worst = 0, team = 1;
  double** tmp = (double**)calloc((size_t)n_prob, sizeof(double*));
#pragma omp parallel num_threads(n_threads)
  {
#pragma omp single
    team = omp_get_num_threads();
#pragma omp for schedule(dynamic, 1)
    for (int p = 0; p < n_prob; ++p) {
      const int st = solve_one(d, n_a[p], a_freqs + a_off[p] * d, a_hat + 2 * a_off[p], n_f[p],
                               f_freqs + f_off[p] * d, f_hat + 2 * f_off[p], level[p], tol, max_iter,
                               matvec_reps, u_out ? &tmp[p] : NULL, &info[p]);
      if (st != 0) {
#pragma omp critical
        if (worst == 0) worst = st;
      }
    }
  }
  if (u_out) {
    int64_t off = 0;
    for (int p = 0; p < n_prob; ++p) {
      if (u_off) u_off[p] = off;
      if (tmp[p] && off + info[p].n <= u_cap) memcpy(u_out + 2 * off, tmp[p], (size_t)2 * info[p].n * sizeof(double));
      off += info[p].n;
    }
    if (u_off) u_off[n_prob] = off;
  }
  for (int p = 0; p < n_prob; ++p) free(tmp[p]);
  free(tmp);
  free(a_off);
  free(f_off);
  if (threads_used) *threads_used = team;
  return worst;
}
