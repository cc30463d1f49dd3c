// Host backend: sections, reductions and remaps on host memory.
//
// The paper maps each section to the CPU or the GPU of its platform and
// weighs that choice in the shortest path (section 2, third paragraph;
// Table 4 maps the Medical sections to both).  These are the host versions
// of the device kernels, with the same semantics and the same rounding:
// terms are read before any write, folded in the order the section fixes,
// and every floating-point step is a single IEEE operation in the write
// field's type (this file is compiled without contraction into fused
// multiply-adds, and x86-64 evaluates float and double in their own
// precision).  Records are split into contiguous ranges over host threads;
// a reduction adds the threads' tables in thread order, with the device's
// compensated summation.
#include <algorithm>
#include <atomic>
#include <condition_variable>
#include <cstring>
#include <functional>
#include <mutex>
#include <thread>
#include <vector>

#include "adha_impl.h"

namespace adha {

namespace {

// A process-wide pool of host threads, started on first use and kept until
// exit (starting threads per call costs far more than the small sections it
// would run).  One job at a time: its parts are taken from a counter by the
// workers and by the calling thread.  A worker takes its copy of the job
// (function, part count) under the lock and counts itself active; run()
// returns only when every part is done and no worker is active, so no
// worker can still be inside one job, or claim a part of it, once the next
// job has been published.
class HostPool {
 public:
  static HostPool &get() {
    static HostPool pool;
    return pool;
  }
  uint32_t size() const { return (uint32_t)workers_.size() + 1; }
  void run(uint32_t parts, const std::function<void(uint32_t)> &fn) {
    std::lock_guard<std::mutex> one(run_m_);
    {
      std::lock_guard<std::mutex> lk(m_);
      job_ = &fn;
      parts_ = parts;
      next_.store(0);
      done_.store(0);
      ++gen_;
    }
    cv_.notify_all();
    work(fn, parts);
    std::unique_lock<std::mutex> lk(m_);
    done_cv_.wait(lk, [&] { return done_.load() == parts && active_ == 0; });
    job_ = nullptr;
  }
  ~HostPool() {
    {
      std::lock_guard<std::mutex> lk(m_);
      stop_ = true;
    }
    cv_.notify_all();
    for (auto &t : workers_) t.join();
  }

 private:
  HostPool() {
    const uint32_t hw = std::thread::hardware_concurrency();
    const uint32_t n = std::max(1u, std::min(hw ? hw : 1u, 256u)) - 1;
    for (uint32_t k = 0; k < n; ++k) workers_.emplace_back([this] { loop(); });
  }
  void work(const std::function<void(uint32_t)> &fn, uint32_t parts) {
    for (;;) {
      const uint32_t p = next_.fetch_add(1);
      if (p >= parts) return;
      fn(p);
      done_.fetch_add(1);
    }
  }
  void loop() {
    uint64_t seen = 0;
    for (;;) {
      const std::function<void(uint32_t)> *job;
      uint32_t parts;
      {
        std::unique_lock<std::mutex> lk(m_);
        cv_.wait(lk, [&] { return stop_ || (gen_ != seen && job_ != nullptr); });
        if (stop_) return;
        seen = gen_;
        job = job_;
        parts = parts_;
        ++active_;
      }
      work(*job, parts);
      {
        std::lock_guard<std::mutex> lk(m_);
        --active_;
      }
      done_cv_.notify_all();
    }
  }
  std::vector<std::thread> workers_;
  std::mutex m_, run_m_;
  std::condition_variable cv_, done_cv_;
  const std::function<void(uint32_t)> *job_ = nullptr;  // guarded by m_
  uint32_t parts_ = 0;                                  // guarded by m_
  uint32_t active_ = 0;                                 // workers inside work(); guarded by m_
  std::atomic<uint32_t> next_{0}, done_{0};
  uint64_t gen_ = 0;
  bool stop_ = false;
};

// fn(part, begin, end) over `threads` contiguous ranges of [0, n) (fewer for
// small n).
template <class Fn>
void parallel_ranges(int64_t n, uint32_t threads, Fn fn) {
  const uint32_t t = (uint32_t)std::max<int64_t>(1, std::min<int64_t>(threads, (n + 4095) / 4096));
  if (t <= 1) {
    fn(0u, (int64_t)0, n);
    return;
  }
  const std::function<void(uint32_t)> part = [&](uint32_t k) { fn(k, n * k / t, n * (k + 1) / t); };
  HostPool::get().run(t, part);
}

// Reductions sum floating-point columns as the device does: per thread a
// pair (s, c), s the rounded running sum and c collecting the exact rounding
// errors (TwoSum), and the threads' pairs added in thread order as
// double-double numbers; the result is the double nearest the final pair.
inline void two_sum(double a, double b, double *s, double *e) {
  const double t = a + b;
  const double bb = t - a;
  *e = (a - (t - bb)) + (b - bb);
  *s = t;
}

// A host thread's chain is a whole record range, so the pair is renormalised
// after every value (the error then grows with the chain's length, not with
// its square).
inline void comp_add(double &s, double &c, double v) {
  double e;
  two_sum(s, v, &s, &e);
  two_sum(s, c + e, &s, &c);
}

inline void pair_add(double a1, double a2, double b1, double b2, double *hi, double *lo) {
  double s, e, t, f, s2, e3;
  two_sum(a1, b1, &s, &e);
  two_sum(a2, b2, &t, &f);
  two_sum(s, e + t, &s2, &e3);
  two_sum(s2, e3 + f, hi, lo);
}

inline uint64_t read_term(const uint8_t *buf, const LayoutDesc &l, int64_t r, int f) {
  uint64_t v = 0;
  std::memcpy(&v, buf + l.addr(r, f), l.shape.ebytes[f]);
  return v;
}

// The value of an integer term (its element bytes zero-extended in b).
inline int64_t int_value(int32_t dt, uint64_t b) {
  switch (dt) {
    case ADHA_I32: return (int32_t)(uint32_t)b;
    case ADHA_I16: return (int16_t)(uint16_t)b;
    case ADHA_U32: return (uint32_t)b;
    case ADHA_U16: return (uint16_t)b;
    default: return (uint8_t)b;
  }
}

inline float as_f32(int32_t dt, uint64_t b) {
  if (dt == ADHA_F32) {
    float x;
    const uint32_t u = (uint32_t)b;
    std::memcpy(&x, &u, 4);
    return x;
  }
  if (dt == ADHA_F64) {
    double d;
    std::memcpy(&d, &b, 8);
    return (float)d;
  }
  return (float)int_value(dt, b);  // nearest even; exact below 2^24
}

inline double as_f64(int32_t dt, uint64_t b) {
  if (dt == ADHA_F32) return (double)as_f32(ADHA_F32, b);
  if (dt == ADHA_F64) {
    double d;
    std::memcpy(&d, &b, 8);
    return d;
  }
  return (double)int_value(dt, b);
}

inline uint32_t word32(int32_t dt, uint64_t b) {
  if (dt == ADHA_F64) return (uint32_t)b ^ (uint32_t)(b >> 32);
  if (dt == ADHA_F32) return (uint32_t)b;
  return (uint32_t)(uint64_t)int_value(dt, b);
}

struct HAcc {
  float f = 0.0f;
  double d = 0.0;
  uint32_t u = 0;
};

// Write k's accumulator after one more term (GEN and SUM).
inline void fold_term(HAcc &a, int k, int32_t wdt, int32_t tdt, uint64_t t) {
  if (wdt == ADHA_F32) {
    const float v = as_f32(tdt, t);
    if (k == 0) a.f = a.f + v;
    else {
      const float h = a.f * 0.5f;
      a.f = h + v;
    }
  } else if (wdt == ADHA_F64) {
    const double v = as_f64(tdt, t);
    if (k == 0) a.d = a.d + v;
    else {
      const double h = a.d * 0.5;
      a.d = h + v;
    }
  } else {
    const uint32_t u = word32(tdt, t);
    a.u = k == 0 ? a.u + u : (a.u ^ u) * 16777619u;
  }
}

inline void write_acc(uint8_t *buf, const LayoutDesc &l, int64_t r, int f, const HAcc &a) {
  uint8_t *p = buf + l.addr(r, f);
  const int32_t dt = l.shape.dtype[f];
  if (dt == ADHA_F32) std::memcpy(p, &a.f, 4);
  else if (dt == ADHA_F64) std::memcpy(p, &a.d, 8);
  else std::memcpy(p, &a.u, l.shape.ebytes[f]);  // the low bytes (x86-64 is little-endian)
}

}  // namespace

uint32_t host_threads(const Ctx *ctx) {
  if (ctx && ctx->host_threads) return ctx->host_threads;
  const uint32_t hw = std::thread::hardware_concurrency();
  return std::max(1u, std::min(hw ? hw : 1u, 64u));
}

adha_status host_section_run(uint32_t threads, const SectionDesc &sec, const LayoutDesc &l, uint8_t *buf,
                             const int32_t *idx, void *table, uint64_t *bad_out) {
  const int64_t n = l.shape.n;
  const size_t nr = sec.rd.size(), nw = sec.wr.size();
  std::vector<uint64_t> bad(std::max<uint32_t>(1, threads), 0);
  if (sec.op == ADHA_OP_REDUCE) {
    const uint32_t cols = (uint32_t)nr + 1, cells = sec.reduce_cells();
    const uint32_t t = std::max<uint32_t>(1, threads);
    // per thread: compensated pairs (s, c) for floating-point columns (c in
    // cs), uint64 for the rest
    std::vector<std::vector<double>> fs(t, std::vector<double>(cells, 0.0));
    std::vector<std::vector<double>> cs(t, std::vector<double>(cells, 0.0));
    std::vector<std::vector<uint64_t>> us(t, std::vector<uint64_t>(cells, 0));
    parallel_ranges(n, t, [&](uint32_t k, int64_t b, int64_t e) {
      for (int64_t r = b; r < e; ++r) {
        int64_t key = 0;
        if (sec.key >= 0) key = (int32_t)(uint32_t)read_term(buf, l, r, sec.key);
        if (key < 0 || key >= (int64_t)sec.n_keys) {
          ++bad[k];
          continue;
        }
        const size_t row = (size_t)key * cols;
        for (size_t q = 0; q < nr; ++q) {
          const int f = sec.rd[q];
          const uint64_t v = read_term(buf, l, r, f);
          const int32_t dt = l.shape.dtype[f];
          if (dt != ADHA_F32 && dt != ADHA_F64) us[k][row + q] += (uint64_t)int_value(dt, v);
          else comp_add(fs[k][row + q], cs[k][row + q], as_f64(dt, v));
        }
        us[k][row + nr] += 1;
      }
    });
    uint64_t *out = (uint64_t *)table;
    for (uint32_t c = 0; c < cells; ++c) {
      const uint32_t q = c % cols;
      const bool fp = q < nr && (l.shape.dtype[sec.rd[q]] == ADHA_F32 || l.shape.dtype[sec.rd[q]] == ADHA_F64);
      if (fp) {
        double hi = 0.0, lo = 0.0;
        for (uint32_t k = 0; k < t; ++k) pair_add(hi, lo, fs[k][c], cs[k][c], &hi, &lo);
        std::memcpy(&out[c], &hi, 8);
      } else {
        uint64_t s = 0;
        for (uint32_t k = 0; k < t; ++k) s += us[k][c];
        out[c] = s;
      }
    }
  } else {
    const int32_t w0 = nw > 0 ? l.shape.dtype[sec.wr[0]] : ADHA_F32;
    const int32_t w1 = nw > 1 ? l.shape.dtype[sec.wr[1]] : ADHA_F32;
    parallel_ranges(n, threads, [&](uint32_t k, int64_t b, int64_t e) {
      std::vector<uint64_t> tv(nr);
      for (int64_t r = b; r < e; ++r) {
        HAcc acc[2];
        if (sec.degree == 0) {
          for (size_t q = 0; q < nr; ++q) tv[q] = read_term(buf, l, r, sec.rd[q]);
          if (sec.op == ADHA_OP_GEN || sec.op == ADHA_OP_SUM) {
            for (size_t q = 0; q < nr; ++q) {
              const int32_t dt = l.shape.dtype[sec.rd[q]];
              fold_term(acc[0], 0, w0, dt, tv[q]);
              if (nw > 1) fold_term(acc[1], 1, w1, dt, tv[q]);
            }
          } else {
            const int32_t d0 = l.shape.dtype[sec.rd[0]], d1 = l.shape.dtype[sec.rd[1]];
            if (w0 == ADHA_F32) {
              const float x = as_f32(d0, tv[0]), y = as_f32(d1, tv[1]);
              if (sec.op == ADHA_OP_MULADD3) {
                const float m = x * y;
                acc[0].f = m + as_f32(l.shape.dtype[sec.rd[2]], tv[2]);
              } else {
                acc[0].f = x - y;
              }
            } else {
              const double x = as_f64(d0, tv[0]), y = as_f64(d1, tv[1]);
              if (sec.op == ADHA_OP_MULADD3) {
                const double m = x * y;
                acc[0].d = m + as_f64(l.shape.dtype[sec.rd[2]], tv[2]);
              } else {
                acc[0].d = x - y;
              }
            }
          }
        } else {
          const int32_t *row = sec.stencil ? nullptr : idx + (uint64_t)r * sec.degree;
          int64_t x = 0, y = 0, z = 0;
          if (sec.stencil) {
            x = r % sec.nx;
            y = (r / sec.nx) % sec.ny;
            z = r / ((int64_t)sec.nx * sec.ny);
          }
          for (uint32_t j = 0; j < sec.degree; ++j) {
            int64_t nb;
            if (sec.stencil) {
              const int64_t xx = x + sec.offsets[3 * j], yy = y + sec.offsets[3 * j + 1],
                            zz = z + sec.offsets[3 * j + 2];
              if (xx < 0 || xx >= sec.nx || yy < 0 || yy >= sec.ny || zz < 0 || zz >= sec.nz) continue;  // off the grid
              nb = xx + (int64_t)sec.nx * (yy + (int64_t)sec.ny * zz);
            } else {
              nb = row[j];
            }
            if (nb < 0 || nb >= n) {
              ++bad[k];
              continue;
            }
            for (size_t q = 0; q < nr; ++q) {
              const int f = sec.rd[q];
              const uint64_t t = read_term(buf, l, nb, f);
              fold_term(acc[0], 0, w0, l.shape.dtype[f], t);
              if (nw > 1) fold_term(acc[1], 1, w1, l.shape.dtype[f], t);
            }
          }
        }
        write_acc(buf, l, r, sec.wr[0], acc[0]);
        if (nw > 1) write_acc(buf, l, r, sec.wr[1], acc[1]);
      }
    });
  }
  if (bad_out) {
    uint64_t s = 0;
    for (uint64_t b : bad) s += b;
    *bad_out = s;
  }
  return ADHA_OK;
}

adha_status host_remap(uint32_t threads, const LayoutDesc &a, const uint8_t *src, const LayoutDesc &b,
                       uint8_t *dst) {
  const int64_t n = a.shape.n;
  const int F = a.shape.nfields();
  // padding is zero: clear the destination, then place every element
  parallel_ranges((int64_t)b.nbytes, threads, [&](uint32_t, int64_t s, int64_t e) {
    std::memset(dst + s, 0, (size_t)(e - s));
  });
  parallel_ranges(n, threads, [&](uint32_t, int64_t s, int64_t e) {
    for (int64_t r = s; r < e; ++r)
      for (int f = 0; f < F; ++f) std::memcpy(dst + b.addr(r, f), src + a.addr(r, f), a.shape.ebytes[f]);
  });
  return ADHA_OK;
}

}  // namespace adha

using namespace adha;

extern "C" {

adha_status adha_host_section_run(const adha_section *sec, const adha_layout *l, void *buf, uint64_t buf_cap,
                                  const int32_t *idx, uint64_t idx_count, void *table, uint64_t table_cap,
                                  uint32_t threads, uint64_t *bad) {
  if (!sec || !l) return fail(ADHA_ERR_INVALID, "NULL argument");
  if (!sec->d.shape.same(l->d.shape)) return fail(ADHA_ERR_INVALID, "section and layout describe different structs");
  const int64_t n = l->d.shape.n;
  if (n > 0 && (!buf || buf_cap < l->d.nbytes))
    return fail(ADHA_ERR_INVALID, "host buffer is NULL or holds %llu bytes, the layout needs %llu",
                (unsigned long long)buf_cap, (unsigned long long)l->d.nbytes);
  if (sec->d.degree > 0 && !sec->d.stencil && n > 0 && (!idx || idx_count < (uint64_t)n * sec->d.degree))
    return fail(ADHA_ERR_INVALID, "gather section needs a host index array of N*d entries");
  if (sec->d.op == ADHA_OP_REDUCE && (!table || table_cap < (uint64_t)sec->d.reduce_cells() * 8))
    return fail(ADHA_ERR_INVALID, "reduction needs a host table of %u cells", sec->d.reduce_cells());
  if (threads == 0) threads = host_threads(nullptr);
  uint64_t nbad = 0;
  ADHA_TRY(host_section_run(threads, sec->d, l->d, (uint8_t *)buf, idx, table, &nbad));
  if (bad) *bad = nbad;
  return ADHA_OK;
}

adha_status adha_host_remap(const adha_layout *src_l, const void *src, uint64_t src_cap, const adha_layout *dst_l,
                            void *dst, uint64_t dst_cap, uint32_t threads) {
  if (!src_l || !dst_l) return fail(ADHA_ERR_INVALID, "layout is NULL");
  if (!src_l->d.shape.same(dst_l->d.shape))
    return fail(ADHA_ERR_INVALID, "source and destination layouts describe different structs");
  if (src_l->d.nbytes && (!src || src_cap < src_l->d.nbytes)) return fail(ADHA_ERR_INVALID, "src too small");
  if (dst_l->d.nbytes && (!dst || dst_cap < dst_l->d.nbytes)) return fail(ADHA_ERR_INVALID, "dst too small");
  const uintptr_t x = (uintptr_t)src, y = (uintptr_t)dst;
  if (src_l->d.nbytes && dst_l->d.nbytes && x < y + dst_l->d.nbytes && y < x + src_l->d.nbytes)
    return fail(ADHA_ERR_INVALID, "src and dst overlap (remaps are out of place)");
  if (threads == 0) threads = host_threads(nullptr);
  return host_remap(threads, src_l->d, (const uint8_t *)src, dst_l->d, (uint8_t *)dst);
}

}  // extern "C"
