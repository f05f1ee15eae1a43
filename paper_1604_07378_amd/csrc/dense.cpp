// Dense building blocks of the host factorisation: a small persistent thread
// pool and a register-blocked C -= A B^T update (the Schur-complement and
// left-looking updates of the supernodal Cholesky factorisation).
#include <algorithm>
#include <atomic>
#include <condition_variable>
#include <cstdlib>
#include <functional>
#include <mutex>
#include <thread>
#include <vector>

#include "host.hpp"

namespace qn {

namespace {

class Pool {
 public:
  explicit Pool(int n) : nthreads_(n) {
    for (int i = 1; i < n; ++i) workers_.emplace_back([this, i] { loop(i); });
  }
  ~Pool() {
    {
      std::lock_guard<std::mutex> g(mu_);
      stop_ = true;
      ++gen_;
    }
    cv_.notify_all();
    for (auto& t : workers_) t.join();
  }
  int size() const { return nthreads_; }

  // Runs fn(chunk) for chunk in [0, nchunks) on all threads; returns when done.
  void run(int64_t nchunks, const std::function<void(int64_t)>& fn) {
    std::unique_lock<std::mutex> call_lock(call_mu_);
    {
      std::lock_guard<std::mutex> g(mu_);
      fn_ = &fn;
      nchunks_ = nchunks;
      next_.store(0);
      busy_ = nthreads_ - 1;
      ++gen_;
    }
    cv_.notify_all();
    work();
    std::unique_lock<std::mutex> g(mu_);
    done_cv_.wait(g, [this] { return busy_ == 0; });
    fn_ = nullptr;
  }

 private:
  void work() {
    for (;;) {
      int64_t c = next_.fetch_add(1);
      if (c >= nchunks_) break;
      (*fn_)(c);
    }
  }
  void loop(int) {
    uint64_t seen = 0;
    for (;;) {
      {
        std::unique_lock<std::mutex> g(mu_);
        cv_.wait(g, [&] { return gen_ != seen; });
        seen = gen_;
        if (stop_) return;
      }
      work();
      {
        std::lock_guard<std::mutex> g(mu_);
        if (--busy_ == 0) done_cv_.notify_all();
      }
    }
  }

  int nthreads_;
  std::vector<std::thread> workers_;
  std::mutex mu_, call_mu_;
  std::condition_variable cv_, done_cv_;
  uint64_t gen_ = 0;
  bool stop_ = false;
  int busy_ = 0;
  const std::function<void(int64_t)>* fn_ = nullptr;
  int64_t nchunks_ = 0;
  std::atomic<int64_t> next_{0};
};

Pool& pool() {
  static Pool p([] {
    int n = (int)std::thread::hardware_concurrency();
    if (const char* e = std::getenv("OMP_NUM_THREADS")) {
      int v = std::atoi(e);
      if (v > 0) n = v;
    }
    return std::max(1, std::min(n, 16));
  }());
  return p;
}

}  // namespace

int host_threads() { return pool().size(); }

void parallel_for(int64_t n, int64_t grain, const void* ctx,
                  void (*fn)(const void* ctx, int64_t lo, int64_t hi)) {
  if (n <= 0) return;
  grain = std::max<int64_t>(1, grain);
  int64_t nchunks = (n + grain - 1) / grain;
  if (nchunks == 1 || pool().size() == 1) {
    fn(ctx, 0, n);
    return;
  }
  std::function<void(int64_t)> body = [&](int64_t c) {
    int64_t lo = c * grain, hi = std::min(n, lo + grain);
    fn(ctx, lo, hi);
  };
  pool().run(nchunks, body);
}

// ---------------------------------------------------------------------------
// C -= A B^T with an 8 x 4 register tile (GCC/clang vector extensions).
// ---------------------------------------------------------------------------
typedef double v4d __attribute__((vector_size(32), aligned(8)));

static inline v4d load4(const double* p) {
  v4d v;
  __builtin_memcpy(&v, p, sizeof(v));
  return v;
}
static inline void store4(double* p, v4d v) { __builtin_memcpy(p, &v, sizeof(v)); }

// Full 8x4 tile: rows a0..a0+7 of A, rows b0..b0+3 of B.
static void tile8x4(int kk, const double* A, int lda, const double* B, int ldb, double* C,
                    int ldc) {
  v4d c00 = {0, 0, 0, 0}, c01 = c00, c02 = c00, c03 = c00;
  v4d c10 = c00, c11 = c00, c12 = c00, c13 = c00;
  for (int k = 0; k < kk; ++k) {
    const double* a = A + (int64_t)k * lda;
    const double* b = B + (int64_t)k * ldb;
    v4d a0 = load4(a), a1 = load4(a + 4);
    double b0 = b[0], b1 = b[1], b2 = b[2], b3 = b[3];
    c00 += a0 * b0; c10 += a1 * b0;
    c01 += a0 * b1; c11 += a1 * b1;
    c02 += a0 * b2; c12 += a1 * b2;
    c03 += a0 * b3; c13 += a1 * b3;
  }
  double* c;
  c = C + 0 * (int64_t)ldc; store4(c, load4(c) - c00); store4(c + 4, load4(c + 4) - c10);
  c = C + 1 * (int64_t)ldc; store4(c, load4(c) - c01); store4(c + 4, load4(c + 4) - c11);
  c = C + 2 * (int64_t)ldc; store4(c, load4(c) - c02); store4(c + 4, load4(c + 4) - c12);
  c = C + 3 * (int64_t)ldc; store4(c, load4(c) - c03); store4(c + 4, load4(c + 4) - c13);
}

static void tile_generic(int ma, int nb, int kk, const double* A, int lda, const double* B,
                         int ldb, double* C, int ldc, int a_base, int b_base, bool lower) {
  for (int b = 0; b < nb; ++b) {
    for (int a = 0; a < ma; ++a) {
      if (lower && (a + a_base) < (b + b_base)) continue;
      double s = 0.0;
      for (int k = 0; k < kk; ++k) s += A[a + (int64_t)k * lda] * B[b + (int64_t)k * ldb];
      C[a + (int64_t)b * ldc] -= s;
    }
  }
}

namespace {
struct GemmArgs {
  int ma, nb, kk, lda, ldb, ldc;
  const double *A, *B;
  double* C;
  bool lower;
  int ntile_b;
};
constexpr int TA = 64, TB = 64;

void gemm_tiles(const void* vctx, int64_t lo, int64_t hi) {
  const GemmArgs& g = *static_cast<const GemmArgs*>(vctx);
  for (int64_t t = lo; t < hi; ++t) {
    int ta = (int)(t / g.ntile_b), tb = (int)(t % g.ntile_b);
    int a0 = ta * TA, b0 = tb * TB;
    if (g.lower && b0 > a0 + TA - 1) continue;
    int ma = std::min(TA, g.ma - a0), nb = std::min(TB, g.nb - b0);
    for (int bb = 0; bb < nb; bb += 4) {
      int nbb = std::min(4, nb - bb);
      for (int aa = 0; aa < ma; aa += 8) {
        int maa = std::min(8, ma - aa);
        int ga = a0 + aa, gb = b0 + bb;
        const double* Ap = g.A + ga;
        const double* Bp = g.B + gb;
        double* Cp = g.C + ga + (int64_t)gb * g.ldc;
        bool full = (maa == 8 && nbb == 4);
        bool below = !g.lower || (ga >= gb + 3);
        if (full && below)
          tile8x4(g.kk, Ap, g.lda, Bp, g.ldb, Cp, g.ldc);
        else if (!g.lower || ga + maa - 1 >= gb)
          tile_generic(maa, nbb, g.kk, Ap, g.lda, Bp, g.ldb, Cp, g.ldc, ga, gb, g.lower);
      }
    }
  }
}
}  // namespace

void gemm_nt_sub(int ma, int nb, int kk, const double* A, int lda, const double* B, int ldb,
                 double* C, int ldc, bool lower_only) {
  if (ma <= 0 || nb <= 0 || kk <= 0) return;
  GemmArgs g{ma, nb, kk, lda, ldb, ldc, A, B, C, lower_only, (nb + TB - 1) / TB};
  int64_t ntiles = (int64_t)((ma + TA - 1) / TA) * g.ntile_b;
  double work = (double)ma * nb * kk;
  int64_t grain = work < 2e6 ? ntiles : 1;
  parallel_for(ntiles, grain, &g, gemm_tiles);
}

namespace {
struct GramArgs {
  int n, nt;
  const double* LT;  // transpose of Linv: LT[a + k n] = Linv[k, a]
  double* S;
};
constexpr int TG = 64;

void gram_tiles(const void* vctx, int64_t lo, int64_t hi) {
  const GramArgs& g = *static_cast<const GramArgs*>(vctx);
  const int n = g.n;
  for (int64_t t = lo; t < hi; ++t) {
    const int ta = (int)(t / g.nt), tb = (int)(t % g.nt);
    if (tb > ta) continue;
    const int a0 = ta * TG, b0 = tb * TG;
    const int ma = std::min(TG, n - a0), nb = std::min(TG, n - b0);
    const int k0 = a0;  // Linv[k, a] = 0 for k < a, and a >= a0 >= b0
    const int kk = n - k0;
    for (int bb = 0; bb < nb; bb += 4) {
      const int nbb = std::min(4, nb - bb);
      for (int aa = 0; aa < ma; aa += 8) {
        const int maa = std::min(8, ma - aa);
        const int ga = a0 + aa, gb = b0 + bb;
        const double* Ap = g.LT + ga + (int64_t)k0 * n;
        const double* Bp = g.LT + gb + (int64_t)k0 * n;
        double* Cp = g.S + ga + (int64_t)gb * n;
        if (maa == 8 && nbb == 4)
          tile8x4(kk, Ap, n, Bp, n, Cp, n);
        else
          tile_generic(maa, nbb, kk, Ap, n, Bp, n, Cp, n, ga, gb, false);
      }
    }
  }
}

struct TransArgs {
  int n;
  const double* src;
  double* dst;
};
void transpose_cols(const void* vctx, int64_t lo, int64_t hi) {
  const TransArgs& a = *static_cast<const TransArgs*>(vctx);
  for (int64_t c = lo; c < hi; ++c)
    for (int i = 0; i < a.n; ++i) a.dst[c + (int64_t)i * a.n] = a.src[i + c * a.n];
}

void mirror_cols(const void* vctx, int64_t lo, int64_t hi) {
  const TransArgs& a = *static_cast<const TransArgs*>(vctx);
  double* S = a.dst;
  // lower part holds -S; write S to both triangles (column c: rows >= c)
  for (int64_t c = lo; c < hi; ++c)
    for (int i = (int)c; i < a.n; ++i) S[i + c * a.n] = -S[i + c * a.n];
}
void mirror_upper(const void* vctx, int64_t lo, int64_t hi) {
  const TransArgs& a = *static_cast<const TransArgs*>(vctx);
  double* S = a.dst;
  for (int64_t c = lo; c < hi; ++c)
    for (int i = 0; i < (int)c; ++i) S[i + c * a.n] = S[c + (int64_t)i * a.n];
}
}  // namespace

void gram_of_lower_inverse(int n, const double* Linv, double* S) {
  if (n <= 0) return;
  std::vector<double> LT((size_t)n * n);
  TransArgs tr{n, Linv, LT.data()};
  parallel_for(n, 16, &tr, transpose_cols);
  std::fill(S, S + (size_t)n * n, 0.0);
  GramArgs g{n, (n + TG - 1) / TG, LT.data(), S};
  parallel_for((int64_t)g.nt * g.nt, 1, &g, gram_tiles);
  TransArgs m{n, nullptr, S};
  parallel_for(n, 16, &m, mirror_cols);
  parallel_for(n, 16, &m, mirror_upper);
}

}  // namespace qn
