// Internal device-side tensor-train handles, memory pool and TT algebra.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <functional>
#include <thread>
#include <mutex>
#include <exception>
#include <condition_variable>
#include <map>
#include <stdexcept>
#include <string>
#include <unordered_map>
#include <vector>

#include "kernels.h"

namespace sgtt {

struct SgttError : std::runtime_error {
  int code;
  SgttError(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define SGTT_HIP(x)                                                                                  \
  do {                                                                                               \
    hipError_t e_ = (x);                                                                             \
    if (e_ != hipSuccess)                                                                            \
      throw ::sgtt::SgttError(-2, std::string(#x) + ": " + hipGetErrorString(e_) + " at " __FILE__); \
  } while (0)

// Caching device allocator: blocks are reused stream-ordered on one stream.
// With a reservation (reserve), blocks are first carved out of one arena
// allocated up front (first fit, freed blocks coalesce), so that work done
// after the reservation allocates no device memory while the arena suffices;
// blocks beyond it come from hipMalloc and are cached as before.
class Pool {
 public:
  ~Pool();
  double* get(size_t ndoubles);
  void put(double* p);
  // allocate an arena of ndoubles (replaces an empty earlier one; fails if
  // blocks of the old arena are in use)
  void reserve(size_t ndoubles);
  size_t bytes_held() const { return held_; }
  size_t arena_bytes() const { return arena_n_ * sizeof(double); }
  size_t arena_peak_bytes() const { return arena_peak_ * sizeof(double); }
  long device_allocs() const { return device_allocs_; }   // hipMalloc calls so far

 private:
  std::unordered_map<double*, size_t> size_;
  std::multimap<size_t, double*> free_;
  size_t held_ = 0;
  long device_allocs_ = 0;
  // arena: [arena_, arena_ + arena_n_), free ranges by offset (doubles)
  double* arena_ = nullptr;
  size_t arena_n_ = 0, arena_used_ = 0, arena_peak_ = 0;
  std::map<size_t, size_t> arena_free_;
  std::unordered_map<double*, size_t> arena_size_;
  double* arena_get(size_t n);
  bool arena_put(double* p);
};

// Device TT: core1 n1 x r1 (ld r1), core2 r1 x n2 x r2, core3 n3 x r2 (ld r2).
struct TT {
  int n1 = 0, n2 = 0, n3 = 0, r1 = 0, r2 = 0;
  double *c1 = nullptr, *c2 = nullptr, *c3 = nullptr;
  Pool* pool = nullptr;   // owning pool, or nullptr for a view
  TT() = default;
  TT(const TT&) = delete;
  TT& operator=(const TT&) = delete;
  TT(TT&& o) noexcept { *this = std::move(o); }
  TT& operator=(TT&& o) noexcept;
  ~TT() { release(); }
  void release();
  long n_c1() const { return (long)n1 * r1; }
  long n_c2() const { return (long)r1 * n2 * r2; }
  long n_c3() const { return (long)n3 * r2; }
};

// A vector of the all-at-once system: 1 (velocity only) or 2 (u, p) TTs.
struct Vec {
  TT c[2];
  int nc = 2;
};

struct SideLane;

struct Ctx {
  hipStream_t s = nullptr;
  Pool pool;
  // second stream and host thread for the pressure TT of a vector pair
  // (see pair_run); created on first use, owned by this context
  SideLane* side = nullptr;
  // a second lane for the solver's own overlap (the solution and residual of
  // one outer iteration beside the next iteration's preconditioner)
  SideLane* sol = nullptr;
  int device = 0;
  bool side_enabled = true;
  // scratch (grown on demand)
  double* ws = nullptr;
  size_t ws_n = 0;
  double* ws2 = nullptr;
  size_t ws2_n = 0;
  int* dint = nullptr;         // small device int scratch (64)
  int* dpiv = nullptr;         // pivots of the last truncation's first stage (96)
  double* dscal = nullptr;     // small device double scratch (256)
  int* hint = nullptr;         // pinned host mirror (64)
  double* hdbl = nullptr;      // pinned host mirror (256)
  long syncs = 0;
  long roundings = 0;
  double* scratch(size_t n);   // general scratch for gram partials
  double* scratch2(size_t n);  // trunc L + dwork
  void sync();
  ~Ctx();
};

// A second context (own stream, pool and scratch) driven by its own host
// thread: post() hands it one job at a time, wait() joins it and returns
// the job's exception (null if none).  fork_ev / join_ev order its stream
// against the caller's; `held` and `keep` hold results that live in its pool
// until its next job releases them (on its own thread).
struct SideLane {
  Ctx c;
  std::thread th;
  std::mutex mu;
  std::condition_variable cv;
  std::function<void()> job;
  bool has_job = false, done = true, quit = false;
  std::exception_ptr err;
  hipEvent_t fork_ev = nullptr, join_ev = nullptr;
  TT held;   // the last result, in this lane's pool until the next job
  std::vector<TT> keep;   // more results of the last job, released likewise

  explicit SideLane(int device) {
    c.device = device;
    c.side_enabled = false;
    SGTT_HIP(hipSetDevice(device));
    SGTT_HIP(hipStreamCreateWithFlags(&c.s, hipStreamNonBlocking));
    SGTT_HIP(hipEventCreateWithFlags(&fork_ev, hipEventDisableTiming));
    SGTT_HIP(hipEventCreateWithFlags(&join_ev, hipEventDisableTiming));
    SGTT_HIP(hipHostMalloc((void**)&c.hint, 64 * sizeof(int), hipHostMallocDefault));
    SGTT_HIP(hipHostMalloc((void**)&c.hdbl, 256 * sizeof(double), hipHostMallocDefault));
    c.dint = (int*)c.pool.get(64);
    c.dscal = c.pool.get(256);
    th = std::thread([this, device]() {
      (void)hipSetDevice(device);
      std::unique_lock<std::mutex> lk(mu);
      for (;;) {
        cv.wait(lk, [this] { return has_job || quit; });
        if (quit) return;
        std::function<void()> f = std::move(job);
        has_job = false;
        lk.unlock();
        std::exception_ptr e;
        try {
          f();
        } catch (...) {
          e = std::current_exception();
        }
        lk.lock();
        err = e;
        done = true;
        cv.notify_all();
      }
    });
  }
  ~SideLane() {
    {
      std::lock_guard<std::mutex> lk(mu);
      quit = true;
    }
    cv.notify_all();
    if (th.joinable()) th.join();
    (void)hipStreamSynchronize(c.s);
    held.release();
    if (fork_ev) (void)hipEventDestroy(fork_ev);
    if (join_ev) (void)hipEventDestroy(join_ev);
    // the pool and pinned mirrors go with c; the stream last
    hipStream_t s = c.s;
    c.s = nullptr;
    if (s) {
      splitk_release(s);
      (void)hipStreamDestroy(s);
    }
  }
  void post(std::function<void()> f) {
    std::lock_guard<std::mutex> lk(mu);
    job = std::move(f);
    has_job = true;
    done = false;
    err = nullptr;
    cv.notify_all();
  }
  // waits for the posted job; returns its exception (null if none)
  std::exception_ptr wait() {
    std::unique_lock<std::mutex> lk(mu);
    cv.wait(lk, [this] { return done; });
    return err;
  }
};


// Runs fu on this thread and context (its stream) and fp on the context's
// side lane (a second stream driven by a second host thread, with its own
// memory pool and scratch), concurrently: the two TTs of a vector pair are
// rounded side by side, so that the one-workgroup eigen stages of the
// velocity and pressure truncations overlap and each waits on its own
// stream only.  The side stream starts after everything queued on c's
// stream so far and c's stream resumes after the side work; fp's result is
// copied into c's pool (its own memory is recycled on the side lane).  The
// calling thread's product precision and profiler phase carry over.  With
// c.side_enabled false both run here, one after the other.
void pair_run(Ctx& c, const std::function<TT(Ctx&)>& fu, const std::function<TT(Ctx&)>& fp, TT& out_u, TT& out_p);
// device allocations and roundings of the side lane so far (0 without one)
long side_device_allocs(const Ctx& c);
long side_roundings(const Ctx& c);
void side_release(Ctx& c);   // joins the side thread and frees its stream and memory

TT tt_new(Ctx& c, int n1, int n2, int n3, int r1, int r2);
TT tt_view(int n1, int n2, int n3, int r1, int r2, double* c1, double* c2, double* c3);
TT tt_copy(Ctx& c, const TT& x);

// sum_i coef_i x_i by concatenation; coefficient i = hcoef[i] * (dcoef ? dcoef[i] : 1)
TT tt_concat(Ctx& c, const std::vector<const TT*>& xs, const double* dcoef, const std::vector<double>& hcoef);
// <x, y> into *dout (device); accumulate if acc.  If k3_out is given, the
// core-3 cross Gram X3^T Y3 (x.r2 x y.r2, row-major) is left there.
void tt_dot(Ctx& c, const TT& x, const TT& y, double* dout, int acc, double* k3_out = nullptr);

// One term of a sum of TTs: coefficient = hcoef * (dcoef ? *dcoef : 1).
struct Term {
  const TT* t;
  const double* dcoef;
  double hcoef;
};
constexpr int RANK_CAP = 512;         // first bond (single-workgroup truncation)
constexpr int RANK_CAP_LARGE = 4096;  // second bond (blocked pivoted Cholesky + skeleton)
// T_eps(sum_i c_i t_i) (Gram-based, FP64), exploiting the block structure of
// the concatenated cores.  cache (k*k, row-major, may be null or hold nulls):
// cache[i*k + j] for i <= j = device block t_i.core3^T t_j.core3 (row-major).
// Writes ||sum||^2 to *d_normsq and the squared norm of the result to
// *d_kept (device) when non-null.
TT tt_round_sum(Ctx& c, const std::vector<Term>& terms, double eps, double* d_normsq, double* d_kept,
                const std::vector<const double*>* cache = nullptr, int maxrank = RANK_CAP_LARGE);
TT tt_round(Ctx& c, const TT& x, double eps, double* d_normsq, double* d_kept, int maxrank = RANK_CAP_LARGE);
// TT-SVD (Alg. 4.1) of a full n1 x n2 x n3 tensor (device, C order)
TT tt_from_full(Ctx& c, const double* X, int n1, int n2, int n3, double eps, double* d_normsq,
                int maxrank = RANK_CAP_LARGE);
// full tensor (device buffer of n1*n2*n3)
void tt_expand(Ctx& c, const TT& x, double* out);
// scale core3 by *dscale (inv: 1 / *dscale)
void tt_scale3(Ctx& c, TT& x, const double* dscale, int inv);

}  // namespace sgtt
