// Host build of the device driver's state machine (csrc/driver.hpp) for the
// CPU tests: the test supplies every evaluation from the oracle, so the
// control flow of the estimator is checked without a GPU.
//
// drv_step runs the state machine with one thread as the team.  drv_step_lanes
// runs it with W threads in lockstep as the team, the way a wave runs it on
// the device: each lane holds its own copy of the scalar state and steps the
// components and candidates strided over the lanes; team reductions exchange
// the lanes' values through a shared array between barriers and combine them
// in one fixed order, so every lane receives the same bits.  After the step
// the lanes' states must be bitwise identical (the device stores lane 0's);
// a lane that took a decision from its own partial value instead of the
// team's shows up as a difference.
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <mutex>
#include <cstdint>
#include <cstring>
#include <thread>
#include <vector>
#define SFLS_HD
#include "driver.hpp"

namespace {

// A barrier for W threads that breaks (and stays broken) when a wait lasts
// longer than a second: lanes that diverged may call it different numbers of
// times, and the step then reports the divergence instead of hanging.
struct Barrier {
  explicit Barrier(int w) : W(w) {}
  void arrive_and_wait() {
    std::unique_lock<std::mutex> lk(m);
    if (broken) return;
    const long gen = generation;
    if (++count == W) {
      count = 0;
      ++generation;
      cv.notify_all();
      return;
    }
    if (!cv.wait_for(lk, std::chrono::seconds(1), [&] { return generation != gen || broken; })) {
      broken = true;
      cv.notify_all();
    }
  }
  int W, count = 0;
  long generation = 0;
  bool broken = false;
  std::mutex m;
  std::condition_variable cv;
};

struct LaneShared {
  int W = 1;
  Barrier* bar = nullptr;
  std::vector<double> dv;
  std::vector<int> iv;
};
LaneShared* g_ls = nullptr;
thread_local int tl_lane = 0;

struct LockstepTeam {
  static int lane() { return tl_lane; }
  static int width() { return g_ls->W; }
  template <typename F>
  static double fold_d(double v, F f) {
    g_ls->bar->arrive_and_wait();
    g_ls->dv[tl_lane] = v;
    g_ls->bar->arrive_and_wait();
    double r = g_ls->dv[0];
    for (int i = 1; i < g_ls->W; ++i) r = f(r, g_ls->dv[i]);
    return r;
  }
  static double sum(double v) { return fold_d(v, [](double a, double b) { return a + b; }); }
  static double max(double v) { return fold_d(v, [](double a, double b) { return fmax(a, b); }); }
  static double min(double v) { return fold_d(v, [](double a, double b) { return fmin(a, b); }); }
  static int imin(int v) {
    g_ls->bar->arrive_and_wait();
    g_ls->iv[tl_lane] = v;
    g_ls->bar->arrive_and_wait();
    int r = g_ls->iv[0];
    for (int i = 1; i < g_ls->W; ++i) r = g_ls->iv[i] < r ? g_ls->iv[i] : r;
    return r;
  }
  static bool any(bool b) { return imin(b ? 0 : 1) == 0; }
  static void sync() { g_ls->bar->arrive_and_wait(); }
};

}  // namespace

extern "C" {
int drv_sizes(int* out) {
  out[0] = (int)sizeof(sfls::DrvParams);
  out[1] = (int)sizeof(sfls::DrvState);
  out[2] = (int)sizeof(sfls::DrvArrays);
  return 3;
}
void drv_step(const sfls::DrvParams* P, sfls::DrvState* S, const sfls::DrvArrays* A) {
  sfls::Driver<sfls::SerialTeam> d(*P, *S, *A);
  d.step();
}
// W lanes in lockstep; returns the number of lanes whose state differs from
// lane 0's after the step (0: all agree; W: the lanes did not even meet at
// the same barriers), and stores lane 0's state in S.
int drv_step_lanes(const sfls::DrvParams* P, sfls::DrvState* S, const sfls::DrvArrays* A,
                   int W) {
  Barrier bar(W);
  LaneShared ls;
  ls.W = W;
  ls.bar = &bar;
  ls.dv.assign((size_t)W, 0.0);
  ls.iv.assign((size_t)W, 0);
  g_ls = &ls;
  std::vector<sfls::DrvState> st((size_t)W, *S);
  std::vector<std::thread> th;
  for (int l = 0; l < W; ++l)
    th.emplace_back([&, l] {
      tl_lane = l;
      sfls::Driver<LockstepTeam> d(*P, st[(size_t)l], *A);
      d.step();
      // a lane's last writes are in place before the caller reads the arrays
      bar.arrive_and_wait();
    });
  for (auto& t : th) t.join();
  g_ls = nullptr;
  if (bar.broken) {
    *S = st[0];
    return W;
  }
  int diff = 0;
  for (int l = 1; l < W; ++l)
    if (std::memcmp(&st[0], &st[(size_t)l], sizeof(sfls::DrvState)) != 0) ++diff;
  *S = st[0];
  return diff;
}
}
