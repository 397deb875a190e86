// C ABI of sparsespec: argument checks, handle lifetime, error text, and the
// one-shot solve (Alg. 1, steps 3-5, from host data).
#include <chrono>
#include <cmath>
#include <cstring>
#include <memory>
#include <new>
#include <stdexcept>

#include "ss_internal.h"

struct ss_stamp {
  ss::StampImpl* impl;
};
struct ss_op {
  ss::OpImpl* impl;
};
struct ss_engine {
  ss::EngineImpl* impl;
};
struct ss_batch {
  ss::BatchImpl* impl;
};
struct ss_adr {
  ss::AdrImpl* impl;
};

namespace ss {

namespace {
thread_local std::string g_last_error;
}

void set_error(const std::string& msg) { g_last_error = msg; }

ss_status fail(ss_status st, const std::string& msg) {
  g_last_error = msg;
  return st;
}

const char* last_error_cstr() { return g_last_error.c_str(); }

}  // namespace ss

using namespace ss;

namespace {

hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

// Nothing may propagate through the C ABI: C++ exceptions become status codes.
template <typename F>
ss_status guarded(F&& f) {
  try {
    return f();
  } catch (const std::bad_alloc&) {
    return fail(SS_ENOMEM, "host allocation failed");
  } catch (const std::exception& e) {
    return fail(SS_EINVAL, std::string("internal error: ") + e.what());
  } catch (...) {
    return fail(SS_EINVAL, "internal error");
  }
}

struct DevMem {
  void* p = nullptr;
  ~DevMem() {
    if (p) pool_free(p);
  }
};

}  // namespace

extern "C" {

const char* ss_last_error(void) { return last_error_cstr(); }

const char* ss_version(void) { return "sparsespec 0.1 (gfx950)"; }

ss_status ss_memory_stats(int64_t* live_bytes, int64_t* cached_bytes, int64_t* driver_allocs) {
  return guarded([&]() -> ss_status {
    if (!live_bytes || !cached_bytes || !driver_allocs) return fail(SS_EINVAL, "null argument");
    pool_stats(live_bytes, cached_bytes, driver_allocs);
    return SS_OK;
  });
}

ss_status ss_build_stamp_batch(int32_t n_prob, int32_t d, const int32_t* n_a, const int16_t* a_freqs,
                               const int32_t* n_f, const int16_t* f_freqs, const int32_t* level, void* stream,
                               ss_stamp** out) {
  return guarded([&]() -> ss_status {
    if (!out) return fail(SS_EINVAL, "out is null");
    *out = nullptr;
    StampImpl* impl = nullptr;
    SS_TRY(build_stamp_impl(n_prob, d, n_a, a_freqs, n_f, f_freqs, level, as_stream(stream), &impl));
    *out = new ss_stamp{impl};
    return SS_OK;
  });
}

ss_status ss_build_stamp(int32_t d, int32_t n_a, const int16_t* a_freqs, int32_t n_f, const int16_t* f_freqs,
                         int32_t level, void* stream, ss_stamp** out) {
  return ss_build_stamp_batch(1, d, &n_a, a_freqs, &n_f, f_freqs, &level, stream, out);
}

ss_status ss_stamp_size(const ss_stamp* st, int64_t* n_total, int32_t* n_prob, int64_t* offsets) {
  return guarded([&]() -> ss_status {
    if (!st || !st->impl) return fail(SS_EINVAL, "null stamp");
    if (n_total) *n_total = st->impl->total;
    if (n_prob) *n_prob = st->impl->n_prob;
    if (offsets) std::memcpy(offsets, st->impl->row_off.data(), (st->impl->n_prob + 1) * sizeof(int64_t));
    return SS_OK;
  });
}

ss_status ss_stamp_keys(const ss_stamp* st, int16_t* keys_out, uint8_t* level_out) {
  return guarded([&]() -> ss_status {
    if (!st || !st->impl) return fail(SS_EINVAL, "null stamp");
    const StampImpl* s = st->impl;
    if (keys_out) SS_HIP(hipMemcpy(keys_out, s->d_keys, (size_t)s->total * s->d * 2, hipMemcpyDeviceToHost));
    if (level_out) SS_HIP(hipMemcpy(level_out, s->d_lev, (size_t)s->total, hipMemcpyDeviceToHost));
    return SS_OK;
  });
}

ss_status ss_stamp_lookup(const ss_stamp* st, int32_t prob, int64_t nq, const int16_t* q, int64_t* slot_out) {
  return guarded([&]() -> ss_status {
    if (!st || !st->impl) return fail(SS_EINVAL, "null stamp");
    return stamp_lookup_impl(st->impl, prob, nq, q, slot_out, nullptr);
  });
}

ss_status ss_stamp_lookup_batch(const ss_stamp* st, int64_t nq, const int32_t* prob, const int16_t* q,
                                int64_t* slot_out) {
  return guarded([&]() -> ss_status {
    if (!st || !st->impl) return fail(SS_EINVAL, "null stamp");
    if (nq > 0 && !prob) return fail(SS_EINVAL, "null problem ids");
    return stamp_lookup_impl(st->impl, -1, nq, q, slot_out, nullptr, prob);
  });
}

ss_status ss_stamp_forcing(const ss_stamp* st, const double* f_hat, void* f, void* stream) {
  return guarded([&]() -> ss_status {
    if (!st || !st->impl) return fail(SS_EINVAL, "null stamp");
    return stamp_forcing_impl(st->impl, f_hat, f, as_stream(stream));
  });
}

ss_status ss_lattice_modulus(int64_t expansion, int64_t n, double sigma, int64_t* M) {
  return guarded([&]() -> ss_status { return lattice_modulus_impl(expansion, n, sigma, M); });
}

ss_status ss_stamp_lattice(const ss_stamp* st, const int64_t* z, int64_t M, void* values, int32_t* reconstructing,
                           void* stream) {
  return guarded([&]() -> ss_status {
    if (!st || !st->impl) return fail(SS_EINVAL, "null stamp");
    return stamp_lattice_impl(st->impl, z, M, static_cast<int64_t*>(values), reconstructing, as_stream(stream));
  });
}

void ss_free_stamp(ss_stamp* st) {
  if (!st) return;
  free_stamp_impl(st->impl);
  delete st;
}

ss_status ss_build_op(const ss_stamp* st, const int32_t* n_a, const int16_t* a_freqs, const double* a_hat,
                      uint32_t flags, void* stream, ss_op** out) {
  return guarded([&]() -> ss_status {
    if (!out) return fail(SS_EINVAL, "out is null");
    *out = nullptr;
    if (!st || !st->impl) return fail(SS_EINVAL, "null stamp");
    OpImpl* impl = nullptr;
    SS_TRY(build_op_impl(st->impl, n_a, a_freqs, a_hat, flags, as_stream(stream), &impl));
    *out = new ss_op{impl};
    return SS_OK;
  });
}

ss_status ss_op_info(const ss_op* op, int64_t* n_total, int64_t* n_exec, int64_t* nnz, int64_t* n_components) {
  return guarded([&]() -> ss_status {
    if (!op || !op->impl) return fail(SS_EINVAL, "null operator");
    if (n_total) *n_total = op->impl->total;
    if (n_exec) *n_exec = op->impl->n_exec;
    if (nnz) *nnz = op->impl->nnz;
    if (n_components) *n_components = op->impl->n_components;
    return SS_OK;
  });
}

ss_status ss_op_csr(const ss_op* op, int64_t* row_ptr, int32_t* cols, int32_t* js, int32_t* component) {
  return guarded([&]() -> ss_status {
    if (!op || !op->impl) return fail(SS_EINVAL, "null operator");
    const OpImpl* o = op->impl;
    if (row_ptr || cols || js) {
      // the canonical CSR is read back from the SELL-64 layout: canonical row r is execution row
      // e = canon2exec[r] (lane e % 64 of slice e / 64); its entries, in j order, are followed by
      // null entries up to the slice width, and columns are mapped back to canonical rows
      std::vector<uint32_t> sptr(o->n_slices + 1), sent(std::max<int64_t>(o->n_sell, 1));
      std::vector<int64_t> c2e(o->total), e2c(o->n_exec);
      SS_HIP(hipMemcpy(sptr.data(), o->d_sptr, sptr.size() * 4, hipMemcpyDeviceToHost));
      if (o->n_sell) SS_HIP(hipMemcpy(sent.data(), o->d_sent, o->n_sell * 4, hipMemcpyDeviceToHost));
      SS_HIP(hipMemcpy(c2e.data(), o->d_canon2exec, o->total * 8, hipMemcpyDeviceToHost));
      SS_HIP(hipMemcpy(e2c.data(), o->d_exec2canon, o->n_exec * 8, hipMemcpyDeviceToHost));
      int64_t pos = 0;
      for (int p = 0; p < o->n_prob; ++p) {
        const int64_t ro = o->row_off[p], eo = o->eoff[p];
        for (int64_t r = ro; r < o->row_off[p + 1]; ++r) {
          if (row_ptr) row_ptr[r] = pos;
          const int64_t e = c2e[r], sl = e / kSlice, lane = e % kSlice;
          const uint32_t base = sptr[sl], w = (sptr[sl + 1] - base) / kSlice;
          for (uint32_t q = 0; q < w; ++q) {
            const uint32_t v = sent[base + q * kSlice + lane];
            if ((v >> kColBits) == (uint32_t)kNullJ) break;
            if (pos >= o->nnz) return fail(SS_EDEVICE, "operator layout holds more entries than its count");
            if (cols) cols[pos] = (int32_t)(e2c[eo + (v & kColMask)] - ro);
            if (js) js[pos] = (int32_t)(v >> kColBits);
            ++pos;
          }
        }
      }
      if (pos != o->nnz) return fail(SS_EDEVICE, "operator layout holds fewer entries than its count");
      if (row_ptr) row_ptr[o->total] = pos;
    }
    if (component) SS_HIP(hipMemcpy(component, o->d_comp, o->total * 4, hipMemcpyDeviceToHost));
    return SS_OK;
  });
}

ss_status ss_op_exec_map(const ss_op* op, int64_t* exec_to_canon) {
  return guarded([&]() -> ss_status {
    if (!op || !op->impl || !exec_to_canon) return fail(SS_EINVAL, "null argument");
    SS_HIP(hipMemcpy(exec_to_canon, op->impl->d_exec2canon, op->impl->n_exec * 8, hipMemcpyDeviceToHost));
    return SS_OK;
  });
}

ss_status ss_apply(const ss_op* op, ss_precision prec, const void* x_dev, void* y_dev, void* stream) {
  return guarded([&]() -> ss_status {
    if (!op || !op->impl) return fail(SS_EINVAL, "null operator");
    if (!x_dev || !y_dev) return fail(SS_EINVAL, "null vector");
    if (prec != SS_FP64 && prec != SS_FP32_REFINE) return fail(SS_EINVAL, "unknown precision");
    return apply_impl(op->impl, prec, x_dev, y_dev, as_stream(stream));
  });
}

ss_status ss_proxy_error(const ss_stamp* st_next, const ss_op* op_next, const void* u_dev, int64_t n_u,
                         const double* f_hat, double* err_out, void* stream) {
  return guarded([&]() -> ss_status {
    if (!st_next || !st_next->impl || !op_next || !op_next->impl) return fail(SS_EINVAL, "null stamp or operator");
    return proxy_error_impl(st_next->impl, op_next->impl, u_dev, n_u, f_hat, err_out, as_stream(stream));
  });
}

ss_status ss_solve_direct(const ss_op* op, const void* f_dev, void* u_dev, ss_precision prec, double tol,
                          void* stream, ss_direct_info* info) {
  return guarded([&]() -> ss_status {
    if (!op || !op->impl) return fail(SS_EINVAL, "null operator");
    DirectStats st;
    const ss_status r = direct_solve_impl(op->impl, f_dev, u_dev, prec, tol, as_stream(stream), &st);
    if (info) {
      info->factor_ms = st.factor_ms;
      info->tiles = st.tiles;
      info->chunks = st.chunks;
      info->refine_steps = st.refine_steps;
      info->rel_residual = st.rel_residual;
    }
    return r;
  });
}

ss_status ss_build_adr(const ss_stamp* st, const ss_op* op, const int32_t* n_b, const int16_t* b_freqs,
                       const double* b_hat, const int32_t* n_c, const int16_t* c_freqs, const double* c_hat,
                       void* stream, ss_adr** out) {
  return guarded([&]() -> ss_status {
    if (!out) return fail(SS_EINVAL, "null output handle");
    *out = nullptr;
    if (!st || !st->impl || !op || !op->impl) return fail(SS_EINVAL, "null stamp or operator");
    AdrImpl* impl = nullptr;
    SS_TRY(adr_build_impl(st->impl, op->impl, n_b, b_freqs, b_hat, n_c, c_freqs, c_hat, as_stream(stream), &impl));
    *out = new ss_adr{impl};
    return SS_OK;
  });
}

ss_status ss_adr_apply(const ss_adr* adr, const void* x_dev, void* y_dev, void* stream) {
  return guarded([&]() -> ss_status {
    if (!adr || !adr->impl) return fail(SS_EINVAL, "null ADR operator");
    return adr_apply_impl(adr->impl, x_dev, y_dev, as_stream(stream));
  });
}

ss_status ss_adr_solve(const ss_adr* adr, const void* f_dev, void* u_dev, double tol, int32_t max_iter,
                       void* stream, ss_solve_info* info) {
  return guarded([&]() -> ss_status {
    if (!adr || !adr->impl) return fail(SS_EINVAL, "null ADR operator");
    return adr_solve_impl(adr->impl, f_dev, u_dev, tol, max_iter, as_stream(stream), info);
  });
}

void ss_free_adr(ss_adr* adr) {
  if (!adr) return;
  adr_free_impl(adr->impl);
  delete adr;
}

ss_status ss_op_class_sizes(const ss_op* op, int64_t cap, int64_t* sizes, int64_t* n_out) {
  return guarded([&]() -> ss_status {
    if (!op || !op->impl || !n_out) return fail(SS_EINVAL, "null argument");
    const std::vector<int64_t>& n = op->impl->cls_n;
    *n_out = (int64_t)n.size();
    if (sizes) {
      if (cap < (int64_t)n.size()) return fail(SS_EINVAL, "sizes holds fewer entries than there are classes");
      std::copy(n.begin(), n.end(), sizes);
    }
    return SS_OK;
  });
}

ss_status ss_solve_op(const ss_op* op, const void* f_dev, void* u_dev, double tol, ss_precision prec,
                      int32_t max_iter, void* stream, ss_solve_info* info) {
  return guarded([&]() -> ss_status {
    if (!op || !op->impl) return fail(SS_EINVAL, "null operator");
    return solve_op_impl(op->impl, f_dev, u_dev, tol, prec, max_iter, as_stream(stream), info);
  });
}

ss_status ss_solve_op_noalloc(const ss_op* op, const void* f_dev, void* u_dev, double tol, ss_precision prec,
                              int32_t max_iter, void* stream, ss_solve_info* info) {
  return guarded([&]() -> ss_status {
    if (!op || !op->impl) return fail(SS_EINVAL, "null operator");
    return solve_op_noalloc_impl(op->impl, f_dev, u_dev, tol, prec, max_iter, as_stream(stream), info);
  });
}

ss_status ss_op_bytes(const ss_op* op, int64_t* bytes) {
  return guarded([&]() -> ss_status {
    if (!op || !op->impl || !bytes) return fail(SS_EINVAL, "null argument");
    *bytes = op_device_bytes(op->impl) + (int64_t)op->impl->ws.bytes;
    return SS_OK;
  });
}

ss_status ss_engine_create(int64_t hbm_budget_bytes, int32_t max_slots, void* stream, ss_engine** out) {
  return guarded([&]() -> ss_status {
    if (!out) return fail(SS_EINVAL, "out is null");
    *out = nullptr;
    if (hbm_budget_bytes < 0 || max_slots < 0) return fail(SS_EINVAL, "negative budget or slot count");
    EngineImpl* e = nullptr;
    SS_TRY(engine_create(hbm_budget_bytes, max_slots, as_stream(stream), &e));
    *out = new ss_engine{e};
    return SS_OK;
  });
}

ss_status ss_engine_submit(ss_engine* e, ss_op* op, const void* f_dev, void* u_dev, double tol, ss_precision prec,
                           int32_t max_iter, int64_t tag) {
  return guarded([&]() -> ss_status {
    if (!e || !e->impl || !op || !op->impl) return fail(SS_EINVAL, "null engine or operator");
    return engine_submit(e->impl, op->impl, f_dev, u_dev, tol, prec, max_iter, tag);
  });
}

ss_status ss_engine_step(ss_engine* e, int32_t iters, int32_t* n_active) {
  return guarded([&]() -> ss_status {
    if (!e || !e->impl) return fail(SS_EINVAL, "null engine");
    return engine_step(e->impl, iters, n_active);
  });
}

ss_status ss_engine_poll(ss_engine* e, int32_t cap, int64_t* tags, int32_t* probs, ss_solve_info* info,
                         int32_t* n_out) {
  return guarded([&]() -> ss_status {
    if (!e || !e->impl || !n_out || cap < 0) return fail(SS_EINVAL, "bad argument");
    return engine_poll(e->impl, cap, tags, probs, info, n_out);
  });
}

ss_status ss_engine_usage(const ss_engine* e, int32_t* n_active_requests, int64_t* bytes) {
  return guarded([&]() -> ss_status {
    if (!e || !e->impl) return fail(SS_EINVAL, "null engine");
    return engine_usage(e->impl, n_active_requests, bytes);
  });
}

void ss_engine_free(ss_engine* e) {
  if (!e) return;
  engine_free(e->impl);
  delete e;
}

void ss_free_op(ss_op* op) {
  if (!op) return;
  free_op_impl(op->impl);
  delete op;
}

ss_status ss_solve_batch(int32_t n_prob, int32_t d, const int32_t* n_a, const int16_t* a_freqs,
                         const double* a_hat, const int32_t* n_f, const int16_t* f_freqs, const double* f_hat,
                         const int32_t* level, double tol, ss_precision prec, int32_t max_iter, uint32_t flags,
                         int32_t n_parts, ss_batch** out, ss_solve_info* info) {
  return guarded([&]() -> ss_status {
    if (!out) return fail(SS_EINVAL, "out is null");
    *out = nullptr;
    if (d < 1 || d > 1024) return fail(SS_EINVAL, "d must be in [1, 1024]");
    if (!(tol > 0) || max_iter < 1) return fail(SS_EINVAL, "tol must be > 0 and max_iter >= 1");
    if (prec != SS_FP64 && prec != SS_FP32_REFINE) return fail(SS_EINVAL, "unknown precision");
    BatchImpl* impl = nullptr;
    const ss_status st = batch_solve_impl(n_prob, d, n_a, a_freqs, a_hat, n_f, f_freqs, f_hat, level, tol, prec,
                                          max_iter, flags, n_parts, info, &impl);
    if (impl) *out = new ss_batch{impl};
    return st;
  });
}

ss_status ss_batch_size(const ss_batch* b, int64_t* n_total, int64_t* offsets) {
  return guarded([&]() -> ss_status {
    if (!b || !b->impl) return fail(SS_EINVAL, "null batch");
    if (n_total) *n_total = b->impl->offsets.back();
    if (offsets) std::memcpy(offsets, b->impl->offsets.data(), b->impl->offsets.size() * 8);
    return SS_OK;
  });
}

ss_status ss_batch_solution(const ss_batch* b, void* u, void* stream) {
  return guarded([&]() -> ss_status {
    if (!b || !b->impl) return fail(SS_EINVAL, "null batch");
    return batch_solution_impl(b->impl, u, as_stream(stream));
  });
}

void ss_free_batch(ss_batch* b) {
  if (!b) return;
  free_batch_impl(b->impl);
  delete b;
}

ss_status ss_solve(int32_t d, int32_t n_a, const int16_t* a_freqs, const double* a_hat, int32_t n_f,
                   const int16_t* f_freqs, const double* f_hat, int32_t level, double tol, ss_precision prec,
                   int32_t max_iter, uint32_t flags, const double* x0, int64_t u_cap, int64_t* n_out, double* u_hat_out,
                   int16_t* keys_out, ss_solve_info* info) {
  return guarded([&]() -> ss_status {
    if (d < 1 || d > 1024) return fail(SS_EINVAL, "d must be in [1, 1024]");
    if (!a_freqs || !a_hat || !f_freqs || !f_hat || n_f < 1 || !n_out)
      return fail(SS_EINVAL, "null or empty argument");
    const auto t0 = std::chrono::steady_clock::now();
    ATable at;
    SS_TRY(canonical_a(d, n_a, a_freqs, a_hat, true, &at));
    const int32_t s = at.size();
    const std::vector<int16_t>& ak = at.keys;
    std::vector<double> ac;
    for (int j = 0; j < s; ++j) {
      ac.push_back(at.coef[j].x);
      ac.push_back(at.coef[j].y);
    }
    // supp(f): exact zeros dropped; a nonzero f_0 makes the problem ill-posed
    std::vector<int16_t> fk;
    std::vector<double> fc;
    for (int32_t i = 0; i < n_f; ++i) {
      const int16_t* k = f_freqs + (int64_t)i * d;
      const double re = f_hat[2 * i], im = f_hat[2 * i + 1];
      if (!std::isfinite(re) || !std::isfinite(im)) return fail(SS_EINVAL, "f_hat is not finite");
      bool zero_k = true;
      for (int t = 0; t < d; ++t) zero_k &= k[t] == 0;
      if (re == 0 && im == 0) continue;
      if (zero_k) return fail(SS_EINVAL, "f_0 must be 0 (the forcing must have mean zero)");
      fk.insert(fk.end(), k, k + d);
      fc.push_back(re);
      fc.push_back(im);
    }
    const int32_t nf = (int32_t)fc.size() / 2;
    if (nf == 0) return fail(SS_EINVAL, "f has no nonzero coefficient");
    ss_stamp* st = nullptr;
    SS_TRY(ss_build_stamp(d, s, ak.data(), nf, fk.data(), level, nullptr, &st));
    std::unique_ptr<ss_stamp, void (*)(ss_stamp*)> stg(st, ss_free_stamp);
    const int64_t n = st->impl->total;
    *n_out = n;
    if (!u_hat_out) return SS_OK;
    if (u_cap < n) return fail(SS_EINVAL, "u_cap is smaller than |S^N| (query the size first)");
    ss_op* op = nullptr;
    SS_TRY(ss_build_op(st, &s, ak.data(), ac.data(), flags, nullptr, &op));
    std::unique_ptr<ss_op, void (*)(ss_op*)> opg(op, ss_free_op);
    std::vector<int64_t> slot(nf);
    SS_TRY(stamp_lookup_impl(st->impl, 0, nf, fk.data(), slot.data(), nullptr));
    std::vector<double> fdense(2 * n, 0.0);
    for (int32_t i = 0; i < nf; ++i) {
      if (slot[i] < 0 || slot[i] >= n) return fail(SS_EINVAL, "internal: forcing frequency not in S^N");
      fdense[2 * slot[i]] = fc[2 * i];
      fdense[2 * slot[i] + 1] = fc[2 * i + 1];
    }
    if (keys_out) SS_HIP(hipMemcpy(keys_out, st->impl->d_keys, (size_t)n * d * 2, hipMemcpyDeviceToHost));
    DevMem fd, ud;
    SS_HIP(pool_alloc((void**)&fd.p, n * 16));
    SS_HIP(pool_alloc((void**)&ud.p, n * 16));
    SS_HIP(hipMemcpy(fd.p, fdense.data(), n * 16, hipMemcpyHostToDevice));
    if (x0) SS_HIP(hipMemcpy(ud.p, x0, n * 16, hipMemcpyHostToDevice));   // warm start
    else SS_HIP(hipMemset(ud.p, 0, n * 16));
    const double t_build = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    ss_solve_info inf{};
    const ss_status rs = solve_op_impl(op->impl, fd.p, ud.p, tol, prec, max_iter, nullptr, &inf);
    if (rs != SS_OK && rs != SS_ENOCONV && rs != SS_EBREAKDOWN) return rs;
    const std::string err = rs == SS_OK ? std::string() : std::string(last_error_cstr());
    SS_HIP(hipMemcpy(u_hat_out, ud.p, n * 16, hipMemcpyDeviceToHost));
    inf.t_build_ms = t_build;
    if (info) *info = inf;
    if (rs != SS_OK) return fail(rs, err);
    return SS_OK;
  });
}

}  // extern "C"
