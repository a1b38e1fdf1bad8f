// Host-only stress test of the continuous-batching fit server (sb_server.cpp),
// built with g++ against tests/host/fake_hip and run under the thread or
// address sanitizer.  The device is replaced by a fake fit launch that runs in
// the scheduler thread: it moves an admitted request's observations from the
// inbox into the arena as the kernel does, advances each fit's iteration count,
// and sets its chi-square to sum_i data_i / sigma_i^2 over the fit's arena
// range, so every result shows whether the fit saw exactly its own observations.
// Submitter threads, a poller and a canceller then race the scheduler thread.
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <map>
#include <mutex>
#include <random>
#include <thread>
#include <vector>

#include "sb_server.h"

// ---------------------------------------------------------------- library pieces the server uses
namespace sbh {
thread_local std::string g_err;
sb_status set_error(sb_status st, const std::string& msg) {
  g_err = msg;
  return st;
}
double now_seconds() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}
}  // namespace sbh

namespace sbk {
// The fit kernel's effect on slots, arena and results (see the file comment).
hipError_t launch_fit(const KModel&, const KTables&, const KFit& f, hipStream_t) {
  for (int b = 0; b < f.n_active; ++b) {
    FitSlot* sl = f.slots + f.active[b];
    FitSlot st{};
    if (f.admit[b] >= 0) {
      const AdmitHeader& h = f.hdr[f.admit[b]];
      for (int i = 0; i < h.n_obs; ++i) {
        f.t[h.arena_off + i] = f.in_t[h.src_off + i];
        f.band[h.arena_off + i] = f.in_band[h.src_off + i];
        f.data[h.arena_off + i] = f.in_data[h.src_off + i];
        f.w[h.arena_off + i] = f.in_w[h.src_off + i];
      }
      st.obs_off = h.arena_off;
      st.n_obs = h.n_obs;
      st.status = SB_OK;
      st.free_mask = h.free_mask;
      st.z = h.z;
      st.q[0] = h.t0;
      st.q[1] = h.lnx0;
      st.q[2] = h.x1;
      st.q[3] = h.c;
    } else {
      st = *sl;
    }
    for (int it = 0; it < f.iters && st.iter < f.fit_iters; ++it) st.iter += 1;
    double c2 = 0.0;
    for (int i = 0; i < st.n_obs; ++i) c2 += (double)f.data[st.obs_off + i] * (double)f.w[st.obs_off + i];
    st.chi2 = (float)c2;
    st.n_accept = st.iter;
    *sl = st;
    if (f.out_idx[b] >= 0) f.results[f.out_idx[b]] = st;
  }
  return hipSuccess;
}
}  // namespace sbk

// ---------------------------------------------------------------- the test
namespace {

struct Req {
  std::vector<float> t, data, sigma;
  std::vector<int> band;
  float expect;   // sum data / sigma^2 as the fake kernel computes it
};

Req make_req(std::mt19937& g) {
  std::uniform_int_distribution<int> nob(1, 64);
  std::uniform_real_distribution<float> u(0.5f, 2.0f);
  Req r;
  const int n = nob(g);
  double c2 = 0.0;
  for (int i = 0; i < n; ++i) {
    r.t.push_back(10.0f * i);
    r.band.push_back(i % 2);
    r.data.push_back(u(g));
    r.sigma.push_back(u(g));
    const float w = (float)(1.0 / ((double)r.sigma.back() * r.sigma.back()));
    c2 += (double)r.data.back() * (double)w;
  }
  r.expect = (float)c2;
  return r;
}

}  // namespace

int main(int argc, char** argv) {
  const int per_thread = argc > 1 ? std::atoi(argv[1]) : 300;
  const int n_threads = 4;
  sb_ctx ctx;
  sb_config_default(&ctx.cfg);
  ctx.cfg.max_slots = 16;                  // few slots and a small budget: requests queue
  ctx.cfg.hbm_budget_bytes = 24 * 1024;
  ctx.cfg.iters_per_tick = 7;
  ctx.n_bands = 2;
  ctx.band_lo = {4000.0, 5000.0};
  ctx.band_hi = {4800.0, 5800.0};
  ctx.wave_lo = 2000.0;
  ctx.wave_hi = 9200.0;
  static int err_flag = 0;
  ctx.d_err = &err_flag;
  sbh::Server* server = new sbh::Server(&ctx);
  if (server->start() != SB_OK) {
    std::printf("FAIL start: %s\n", sbh::g_err.c_str());
    return 1;
  }
  std::mutex mu;
  std::map<uint64_t, float> expect;        // ticket -> expected chi2
  std::vector<uint64_t> tickets;
  std::atomic<bool> done_submitting{false};
  std::atomic<int> failures{0};
  std::vector<std::thread> th;
  for (int k = 0; k < n_threads; ++k)
    th.emplace_back([&, k] {
      std::mt19937 g(1234 + k);
      for (int i = 0; i < per_thread; ++i) {
        Req r = make_req(g);
        sb_fit_request q{};
        q.n_obs = (int)r.t.size();
        q.t = r.t.data();
        q.band = r.band.data();
        q.data = r.data.data();
        q.sigma = r.sigma.data();
        q.z = 0.1f;
        q.t0 = 1.0f;
        q.x0 = 1e-5f;
        q.x1 = 0.0f;
        q.c = 0.0f;
        uint64_t tk = 0;
        if (server->submit(&q, &tk) != SB_OK) {
          ++failures;
          continue;
        }
        std::lock_guard<std::mutex> lk(mu);
        expect[tk] = r.expect;
        tickets.push_back(tk);
        if (i % 17 == 0) std::this_thread::yield();
      }
    });
  // a canceller racing the scheduler
  std::thread canceller([&] {
    std::mt19937 g(99);
    while (!done_submitting) {
      uint64_t tk = 0;
      {
        std::lock_guard<std::mutex> lk(mu);
        if (!tickets.empty()) tk = tickets[g() % tickets.size()];
      }
      if (tk && g() % 4 == 0) (void)server->cancel(tk);
      std::this_thread::sleep_for(std::chrono::microseconds(50));
    }
  });
  // a statistics reader
  std::thread stats_reader([&] {
    while (!done_submitting) {
      sb_stats_t s{};
      server->stats(&s);
      if (s.completed + s.cancelled > s.submitted) ++failures;
      std::this_thread::sleep_for(std::chrono::microseconds(100));
    }
  });
  for (auto& t : th) t.join();
  done_submitting = true;
  canceller.join();
  stats_reader.join();
  // collect: every ticket ends exactly once, ok or cancelled; ok results carry their own chi2
  int ok = 0, cancelled = 0;
  for (uint64_t tk : tickets) {
    sb_fit_result res{};
    const sb_status st = server->wait(tk, 30.0, &res);
    if (st != SB_OK) {
      std::printf("FAIL ticket %llu: wait returned %d\n", (unsigned long long)tk, st);
      ++failures;
      continue;
    }
    if (res.status == SB_OK) {
      ++ok;
      if (res.chi2 != expect[tk] || res.iters != ctx.cfg.fit_iters) {
        std::printf("FAIL ticket %llu: chi2 %g expected %g, iters %d\n", (unsigned long long)tk, res.chi2,
                    expect[tk], res.iters);
        ++failures;
      }
    } else if (res.status == SB_CANCELLED) {
      ++cancelled;
    } else {
      std::printf("FAIL ticket %llu: status %d\n", (unsigned long long)tk, res.status);
      ++failures;
    }
    if (server->poll(tk, &res) != SB_ERR_NOTFOUND) ++failures;   // a result is handed out once
  }
  sb_stats_t s{};
  server->stats(&s);
  const bool consistent = s.submitted == (int64_t)tickets.size() && s.completed == ok &&
                          s.cancelled == cancelled && s.active_slots == 0 && s.queue_depth == 0 &&
                          s.bytes_in_use == 0;
  int64_t hist = 0;
  for (int k = 0; k < SB_LATENCY_BINS; ++k) hist += s.latency_hist[k];
  // shutting down with fits still queued cancels them
  std::mt19937 g(7);
  std::vector<uint64_t> late;
  for (int i = 0; i < 50; ++i) {
    Req r = make_req(g);
    sb_fit_request q{};
    q.n_obs = (int)r.t.size();
    q.t = r.t.data();
    q.band = r.band.data();
    q.data = r.data.data();
    q.sigma = r.sigma.data();
    q.z = 0.1f;
    q.x0 = 1e-5f;
    uint64_t tk = 0;
    if (server->submit(&q, &tk) == SB_OK) late.push_back(tk);
  }
  delete server;
  std::printf("submitted %zu ok %d cancelled %d failures %d consistent %d histogram %lld ticks %lld\n",
              tickets.size(), ok, cancelled, failures.load(), (int)consistent, (long long)hist, (long long)s.ticks);
  return (failures == 0 && consistent && hist == ok && ok > 0 && cancelled > 0) ? 0 : 1;
}

// sb_config_default lives in sb_host.cpp, which needs the device code; the test links this copy.
extern "C" void sb_config_default(sb_config* cfg) {
  cfg->max_spacing = 5.0;
  cfg->max_obs_per_fit = 256;
  cfg->max_slots = 1024;
  cfg->hbm_budget_bytes = 256ll << 20;
  cfg->iters_per_tick = 5;
  cfg->fit_iters = 50;
  cfg->lm_lambda0 = 1e-3;
  cfg->quad_rule = SB_QUAD_TRAPEZOID;
  cfg->lds_limit_bytes = 0;
  cfg->solver = SB_SOLVER_LM;
  cfg->lbfgs_m = 5;
}
