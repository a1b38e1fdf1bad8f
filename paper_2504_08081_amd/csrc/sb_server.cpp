// Continuous-batching fit server.
//
// A host thread runs "ticks".  Each tick it (1) admits queued requests into
// free device slots while the byte budget, the slot count and the arena
// allow, (2) packs the tick's active slot list and the admitted requests into
// one pinned blob and copies it to a device inbox, (3) launches the fit
// kernel over every resident fit (the workgroup of a newly admitted fit first
// moves its observations from the inbox into the arena), and (4) copies the
// states of the fits that finish in this tick back to pinned memory.  Ticks
// are pipelined one deep: while tick n runs, the thread publishes the results
// of tick n-1 and prepares tick n+1.  Everything is on one stream, so stream
// order keeps the slot and arena reuse safe.
#include "sb_server.h"

#include <algorithm>
#include <cmath>
#include <cstring>

namespace sbh {

namespace {
constexpr int kInboxObs = 1 << 16;   // observations admitted per tick at most
size_t align256(size_t x) { return (x + 255) & ~size_t(255); }
}  // namespace

// ------------------------------------------------------------------ arena

void Arena::reset(int capacity) {
  cap_ = capacity;
  free_.clear();
  if (capacity > 0) free_[0] = capacity;
}

int Arena::alloc(int n) {
  for (auto it = free_.begin(); it != free_.end(); ++it) {
    if (it->second >= n) {
      const int off = it->first, len = it->second;
      free_.erase(it);
      if (len > n) free_[off + n] = len - n;
      return off;
    }
  }
  return -1;
}

void Arena::release(int off, int n) {
  auto next = free_.lower_bound(off);
  int start = off, len = n;
  if (next != free_.begin()) {
    auto prev = std::prev(next);
    if (prev->first + prev->second == off) {
      start = prev->first;
      len += prev->second;
      free_.erase(prev);
    }
  }
  if (next != free_.end() && next->first == off + n) {
    len += next->second;
    free_.erase(next);
  }
  free_[start] = len;
}

// ------------------------------------------------------------------ server

Server::Server(sb_ctx* ctx) : ctx_(ctx) {}

sb_status Server::start() {
  const sb_config& cfg = ctx_->cfg;
  hipError_t e = hipSetDevice(ctx_->device);
  const int ns = cfg.max_slots;
  const int64_t cap64 = std::max<int64_t>(1, cfg.hbm_budget_bytes / 16);
  const int cap = (int)std::min<int64_t>(cap64, 1 << 30);
  inbox_obs_ = kInboxObs;
  inbox_bytes_ = 3 * align256((size_t)ns * sizeof(int)) + align256((size_t)ns * sizeof(sbk::AdmitHeader)) +
                 4 * align256((size_t)inbox_obs_ * 4) + 1024;
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&stream_, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&ev_[0], hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&ev_[1], hipEventDisableTiming);
  if (e == hipSuccess) e = hipMalloc(&d_slots_, (size_t)ns * sizeof(sbk::FitSlot));
  if (e == hipSuccess) e = hipMalloc(&d_results_, (size_t)ns * sizeof(sbk::FitSlot));
  if (e == hipSuccess) e = hipMalloc(&d_t_, (size_t)cap * 4);
  if (e == hipSuccess) e = hipMalloc(&d_band_, (size_t)cap * 4);
  if (e == hipSuccess) e = hipMalloc(&d_data_, (size_t)cap * 4);
  if (e == hipSuccess) e = hipMalloc(&d_w_, (size_t)cap * 4);
  if (e == hipSuccess) e = hipMalloc(&d_inbox_, inbox_bytes_);
  for (int p = 0; p < 2 && e == hipSuccess; ++p) {
    e = hipHostMalloc((void**)&h_inbox_[p], inbox_bytes_, hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc((void**)&h_res_[p], (size_t)ns * sizeof(sbk::FitSlot), hipHostMallocDefault);
  }
  if (e != hipSuccess) return set_error(SB_ERR_NOMEM, std::string("fit server: ") + hipGetErrorString(e));
  slots_.assign(ns, Slot());
  free_slots_.clear();
  for (int s = ns - 1; s >= 0; --s) free_slots_.push_back(s);
  arena_.reset(cap);
  th_ = std::thread([this] { loop(); });
  started_ = true;
  return SB_OK;
}

Server::~Server() {
  {
    std::lock_guard<std::mutex> lk(mu_);
    stop_ = true;
  }
  cv_work_.notify_all();
  if (th_.joinable()) th_.join();
  {
    std::lock_guard<std::mutex> lk(mu_);
    for (auto& kv : tickets_)
      if (kv.second.state != DONE) {
        kv.second.state = DONE;
        kv.second.res.status = SB_CANCELLED;
      }
  }
  cv_done_.notify_all();
  (void)hipSetDevice(ctx_->device);
  if (stream_) (void)hipStreamSynchronize(stream_);
  for (int p = 0; p < 2; ++p) {
    if (h_inbox_[p]) (void)hipHostFree(h_inbox_[p]);
    if (h_res_[p]) (void)hipHostFree(h_res_[p]);
    if (ev_[p]) (void)hipEventDestroy(ev_[p]);
  }
  if (d_slots_) (void)hipFree(d_slots_);
  if (d_results_) (void)hipFree(d_results_);
  if (d_t_) (void)hipFree(d_t_);
  if (d_band_) (void)hipFree(d_band_);
  if (d_data_) (void)hipFree(d_data_);
  if (d_w_) (void)hipFree(d_w_);
  if (d_inbox_) (void)hipFree(d_inbox_);
  if (stream_) (void)hipStreamDestroy(stream_);
}

sb_status Server::submit(const sb_fit_request* r, uint64_t* ticket) {
  const sb_config& cfg = ctx_->cfg;
  if (!r || !ticket) return set_error(SB_ERR_ARG, "sb_fit_submit: NULL argument");
  if (r->n_obs < 1 || r->n_obs > cfg.max_obs_per_fit)
    return set_error(SB_ERR_ARG, "sb_fit_submit: n_obs outside [1, max_obs_per_fit]");
  if (!r->t || !r->band || !r->data || !r->sigma) return set_error(SB_ERR_ARG, "sb_fit_submit: NULL array");
  if (!std::isfinite(r->z) || !(r->z > -1.f) || !std::isfinite(r->t0) || !std::isfinite(r->x1) ||
      !std::isfinite(r->c) || !std::isfinite(r->x0) || !(r->x0 > 0.f))
    return set_error(SB_ERR_ARG, "sb_fit_submit: bad starting parameters");
  if (r->free_mask & ~(uint32_t)SB_FREE_ALL) return set_error(SB_ERR_ARG, "sb_fit_submit: unknown free_mask bits");
  const double opz = 1.0 + (double)r->z;
  for (int i = 0; i < r->n_obs; ++i) {
    const int b = r->band[i];
    if (b < 0 || b >= ctx_->n_bands) return set_error(SB_ERR_ARG, "sb_fit_submit: band id out of range");
    if (ctx_->band_lo[b] / opz < ctx_->wave_lo || ctx_->band_hi[b] / opz > ctx_->wave_hi)
      return set_error(SB_ERR_ARG, "sb_fit_submit: band rest window outside the surface grid");
    if (!std::isfinite(r->t[i]) || !std::isfinite(r->data[i]) || !std::isfinite(r->sigma[i]) || !(r->sigma[i] > 0.f))
      return set_error(SB_ERR_ARG, "sb_fit_submit: non-finite observation or sigma <= 0");
  }
  // bounds of q = (t0, ln x0, x1, c)
  float qlo[4], qhi[4];
  for (int i = 0; i < 4; ++i) {
    qlo[i] = -INFINITY;
    qhi[i] = INFINITY;
  }
  if (r->has_bounds) {
    if (cfg.solver != SB_SOLVER_LBFGSB)
      return set_error(SB_ERR_ARG, "sb_fit_submit: bounds need the L-BFGS-B solver (sb_config.solver)");
    for (int i = 0; i < 4; ++i) {
      const float a = r->lower[i], b = r->upper[i];
      if (std::isnan(a) || std::isnan(b) || !(a <= b)) return set_error(SB_ERR_ARG, "sb_fit_submit: bounds");
      qlo[i] = a;
      qhi[i] = b;
    }
    if (!(r->upper[1] > 0.f)) return set_error(SB_ERR_ARG, "sb_fit_submit: x0 upper bound must be > 0");
    qlo[1] = r->lower[1] > 0.f ? (float)std::log((double)r->lower[1]) : -INFINITY;
    qhi[1] = std::isinf(r->upper[1]) ? INFINITY : (float)std::log((double)r->upper[1]);
  }
  const int64_t bytes = (int64_t)r->n_obs * 16 + (int64_t)sizeof(sbk::FitSlot);
  if (bytes > cfg.hbm_budget_bytes || r->n_obs > arena_.capacity())
    return set_error(SB_ERR_BUDGET, "sb_fit_submit: request larger than the serving budget");
  Request q;
  q.t.assign(r->t, r->t + r->n_obs);
  q.band.assign(r->band, r->band + r->n_obs);
  q.data.assign(r->data, r->data + r->n_obs);
  q.w.resize(r->n_obs);
  for (int i = 0; i < r->n_obs; ++i) {
    const double sg = r->sigma[i];
    q.w[i] = (float)(1.0 / (sg * sg));
  }
  q.z = r->z;
  q.t0 = r->t0;
  q.x0 = r->x0;
  q.x1 = r->x1;
  q.c = r->c;
  q.free_mask = r->free_mask == 0 ? SB_FREE_ALL : (int)r->free_mask;
  for (int i = 0; i < 4; ++i) {
    q.lo[i] = qlo[i];
    q.hi[i] = qhi[i];
  }
  q.bytes = bytes;
  q.t_submit = now_seconds();
  {
    std::lock_guard<std::mutex> lk(mu_);
    if (poisoned_ != SB_OK) return set_error(poisoned_, poison_msg_);
    q.ticket = next_ticket_++;
    Entry& en = tickets_[q.ticket];
    en.res.status = SB_PENDING;
    en.res.t_submit = q.t_submit;
    *ticket = q.ticket;
    queue_.push_back(std::move(q));
    ++n_submitted_;
  }
  cv_work_.notify_one();
  return SB_OK;
}

sb_status Server::poll(uint64_t ticket, sb_fit_result* out) {
  if (!out) return set_error(SB_ERR_ARG, "sb_fit_poll: NULL result");
  std::lock_guard<std::mutex> lk(mu_);
  auto it = tickets_.find(ticket);
  if (it == tickets_.end()) return set_error(SB_ERR_NOTFOUND, "sb_fit_poll: unknown ticket");
  if (it->second.state != DONE) return SB_PENDING;
  *out = it->second.res;
  tickets_.erase(it);
  return SB_OK;
}

sb_status Server::wait(uint64_t ticket, double timeout_s, sb_fit_result* out) {
  if (!out) return set_error(SB_ERR_ARG, "sb_fit_wait: NULL result");
  std::unique_lock<std::mutex> lk(mu_);
  auto done = [&] {
    auto it = tickets_.find(ticket);
    return it == tickets_.end() || it->second.state == DONE;
  };
  const auto dl = std::chrono::steady_clock::now() + std::chrono::duration<double>(std::max(0.0, timeout_s));
  cv_done_.wait_until(lk, dl, done);
  auto it = tickets_.find(ticket);
  if (it == tickets_.end()) return set_error(SB_ERR_NOTFOUND, "sb_fit_wait: unknown ticket");
  if (it->second.state != DONE) return SB_PENDING;
  *out = it->second.res;
  tickets_.erase(it);
  return SB_OK;
}

sb_status Server::cancel(uint64_t ticket) {
  std::lock_guard<std::mutex> lk(mu_);
  auto it = tickets_.find(ticket);
  if (it == tickets_.end()) return set_error(SB_ERR_NOTFOUND, "sb_fit_cancel: unknown ticket");
  Entry& en = it->second;
  if (en.state == DONE) return SB_OK;
  if (en.state == QUEUED) {
    for (auto q = queue_.begin(); q != queue_.end(); ++q)
      if (q->ticket == ticket) {
        queue_.erase(q);
        break;
      }
    en.state = DONE;
    en.res.status = SB_CANCELLED;
    en.res.t_done = now_seconds();
    ++n_cancelled_;
    cv_done_.notify_all();
    return SB_OK;
  }
  en.cancel = true;   // the scheduler drops it from the next launch
  cv_work_.notify_one();
  return SB_OK;
}

void Server::stats(sb_stats_t* out) {
  std::lock_guard<std::mutex> lk(mu_);
  out->submitted = n_submitted_;
  out->admitted = n_admitted_;
  out->completed = n_completed_;
  out->cancelled = n_cancelled_;
  out->rejected = n_rejected_;
  out->ticks = n_ticks_;
  out->queue_depth = (int32_t)queue_.size();
  out->active_slots = n_active_slots_;
  out->bytes_in_use = bytes_in_use_;
  out->budget_bytes = ctx_->cfg.hbm_budget_bytes;
  out->busy_seconds = busy_s_;
  out->slot_ticks = n_slot_ticks_;
  for (int k = 0; k < SB_LATENCY_BINS; ++k) out->latency_hist[k] = lat_hist_[k];
}

void Server::release_slot(int s) {
  Slot& sl = slots_[s];
  arena_.release(sl.arena_off, sl.n_obs);
  bytes_in_use_ -= sl.bytes;
  sl = Slot();
  free_slots_.push_back(s);
  --n_active_slots_;
}

// Build the blob of one tick (called with mu_ held).  Returns false if there is
// nothing to launch or retire.
bool Server::prepare_tick(int parity, std::vector<Retire>& retire, size_t& blob_bytes, int& n_active,
                          int& n_fin) {
  const sb_config& cfg = ctx_->cfg;
  const int ticks_per_fit = std::max(1, (cfg.fit_iters + cfg.iters_per_tick - 1) / cfg.iters_per_tick);
  retire.clear();
  // cancelled resident fits leave now; their slots free once this tick completes
  for (int s = 0; s < (int)slots_.size(); ++s) {
    Slot& sl = slots_[s];
    if (!sl.used || sl.ticks_left <= 0) continue;
    auto it = tickets_.find(sl.ticket);
    if (it != tickets_.end() && it->second.cancel) {
      sl.ticks_left = 0;
      retire.push_back({s, -1});
    }
  }
  // admissions (first come, first served)
  std::vector<int> admitted;
  std::vector<Request> adm_req;
  int adm_obs = 0;
  while (!queue_.empty()) {
    Request& q = queue_.front();
    const int n = (int)q.t.size();
    if (free_slots_.empty() || bytes_in_use_ + q.bytes > cfg.hbm_budget_bytes || adm_obs + n > inbox_obs_) break;
    const int off = arena_.alloc(n);
    if (off < 0) break;
    const int s = free_slots_.back();
    free_slots_.pop_back();
    Slot& sl = slots_[s];
    sl.used = true;
    sl.ticket = q.ticket;
    sl.arena_off = off;
    sl.n_obs = n;
    sl.ticks_left = ticks_per_fit;
    sl.bytes = q.bytes;
    sl.free_mask = q.free_mask;
    sl.x0 = q.x0;
    bytes_in_use_ += q.bytes;
    ++n_active_slots_;
    ++n_admitted_;
    Entry& en = tickets_[q.ticket];
    en.state = ACTIVE;
    en.slot = s;
    en.res.t_admit = now_seconds();
    admitted.push_back(s);
    adm_obs += n;
    adm_req.push_back(std::move(q));
    queue_.pop_front();
  }
  // the tick's active list
  std::vector<int> act, outi, admi;
  std::vector<sbk::AdmitHeader> hdr;
  size_t adm_pos = 0;
  int src = 0;
  n_fin = 0;
  for (int s = 0; s < (int)slots_.size(); ++s) {
    Slot& sl = slots_[s];
    if (!sl.used || sl.ticks_left <= 0) continue;
    act.push_back(s);
    int ai = -1;
    if (adm_pos < admitted.size()) {
      for (size_t a = 0; a < admitted.size(); ++a)
        if (admitted[a] == s) {
          ai = (int)a;
          break;
        }
    }
    admi.push_back(ai);
    sl.ticks_left -= 1;
    if (sl.ticks_left == 0) {
      outi.push_back(n_fin);
      retire.push_back({s, n_fin});
      ++n_fin;
    } else {
      outi.push_back(-1);
    }
  }
  n_active = (int)act.size();
  for (size_t a = 0; a < admitted.size(); ++a) {
    const Request& q = adm_req[a];
    const Slot& sl = slots_[admitted[a]];
    sbk::AdmitHeader h{};
    h.slot = admitted[a];
    h.arena_off = sl.arena_off;
    h.n_obs = sl.n_obs;
    h.src_off = src;
    h.z = q.z;
    h.t0 = q.t0;
    h.lnx0 = (float)std::log((double)q.x0);
    h.x1 = q.x1;
    h.c = q.c;
    h.free_mask = q.free_mask;
    for (int i = 0; i < 4; ++i) {
      h.lo[i] = q.lo[i];
      h.hi[i] = q.hi[i];
    }
    hdr.push_back(h);
    src += sl.n_obs;
  }
  if (n_active == 0 && retire.empty()) return false;
  // pack the blob
  char* B = h_inbox_[parity];
  size_t o = 0;
  off_active_ = o; o = align256(o + act.size() * sizeof(int));
  off_out_ = o;    o = align256(o + outi.size() * sizeof(int));
  off_admit_ = o;  o = align256(o + admi.size() * sizeof(int));
  off_hdr_ = o;    o = align256(o + hdr.size() * sizeof(sbk::AdmitHeader));
  off_t_ = o;      o = align256(o + (size_t)src * 4);
  off_band_ = o;   o = align256(o + (size_t)src * 4);
  off_data_ = o;   o = align256(o + (size_t)src * 4);
  off_w_ = o;      o = align256(o + (size_t)src * 4);
  blob_bytes = o;
  if (!act.empty()) std::memcpy(B + off_active_, act.data(), act.size() * sizeof(int));
  if (!outi.empty()) std::memcpy(B + off_out_, outi.data(), outi.size() * sizeof(int));
  if (!admi.empty()) std::memcpy(B + off_admit_, admi.data(), admi.size() * sizeof(int));
  if (!hdr.empty()) std::memcpy(B + off_hdr_, hdr.data(), hdr.size() * sizeof(sbk::AdmitHeader));
  size_t p = 0;
  for (const Request& q : adm_req) {
    const size_t n = q.t.size();
    std::memcpy(B + off_t_ + p * 4, q.t.data(), n * 4);
    std::memcpy(B + off_band_ + p * 4, q.band.data(), n * 4);
    std::memcpy(B + off_data_ + p * 4, q.data.data(), n * 4);
    std::memcpy(B + off_w_ + p * 4, q.w.data(), n * 4);
    p += n;
  }
  return true;
}

void Server::finish_tick(int parity) {
  Tick& tk = ticks_[parity];
  hipError_t e = hipEventSynchronize(ev_[parity]);
  const double now = now_seconds();
  {
    std::lock_guard<std::mutex> lk(mu_);
    for (const Retire& r : tk.retire) {
      const uint64_t ticket = slots_[r.slot].ticket;
      auto it = tickets_.find(ticket);
      if (it != tickets_.end()) {
        Entry& en = it->second;
        sb_fit_result& res = en.res;
        if (e != hipSuccess) {
          res.status = SB_ERR_DEVICE;
        } else if (en.cancel || r.out_idx < 0) {
          res.status = SB_CANCELLED;
          ++n_cancelled_;
        } else {
          const sbk::FitSlot& st = h_res_[parity][r.out_idx];
          res.status = st.status;
          res.z = st.z;
          res.t0 = st.q[0];
          res.x0 = (slots_[r.slot].free_mask & SB_FREE_X0) ? std::exp(st.q[1]) : slots_[r.slot].x0;
          res.x1 = st.q[2];
          res.c = st.q[3];
          res.chi2 = st.chi2;
          res.iters = st.iter < 0 ? 0 : st.iter;
          res.n_accept = st.n_accept;
          ++n_completed_;
          // latency histogram: bin k holds [2^k, 2^(k+1)) microseconds
          const double us = (now - res.t_submit) * 1e6;
          int bin = 0;
          while (bin < SB_LATENCY_BINS - 1 && us >= (double)(2ll << bin)) ++bin;
          ++lat_hist_[bin];
        }
        res.t_done = now;
        en.state = DONE;
      }
      release_slot(r.slot);
    }
    tk.retire.clear();
    tk.pending = false;
  }
  cv_done_.notify_all();
  if (e != hipSuccess) fail_all(SB_ERR_DEVICE, std::string("fit server: ") + hipGetErrorString(e));
}

void Server::fail_all(sb_status st, const std::string& msg) {
  std::lock_guard<std::mutex> lk(mu_);
  poisoned_ = st;
  poison_msg_ = msg;
  for (auto& kv : tickets_)
    if (kv.second.state != DONE) {
      kv.second.state = DONE;
      kv.second.res.status = st;
    }
  queue_.clear();
  cv_done_.notify_all();
}

void Server::loop() {
  (void)hipSetDevice(ctx_->device);
  const sb_config& cfg = ctx_->cfg;
  int parity = 0;
  for (;;) {
    std::vector<Retire> retire;
    size_t blob = 0;
    int n_active = 0, n_fin = 0;
    bool launch = false;
    double t_prep = 0;
    {
      std::unique_lock<std::mutex> lk(mu_);
      cv_work_.wait(lk, [&] {
        return stop_ || ticks_[1 - parity].pending ||
               (poisoned_ == SB_OK && (!queue_.empty() || n_active_slots_ > 0));
      });
      if (stop_ && !ticks_[1 - parity].pending) break;
      if (!stop_ && poisoned_ == SB_OK) launch = prepare_tick(parity, retire, blob, n_active, n_fin);
      t_prep = now_seconds();
    }
    if (launch) {
      hipError_t e = hipSuccess;
      if (n_active > 0) {
        e = hipMemcpyAsync(d_inbox_, h_inbox_[parity], blob, hipMemcpyHostToDevice, stream_);
        sbk::KFit f{};
        f.slots = d_slots_;
        f.results = d_results_;
        f.active = (const int*)(d_inbox_ + off_active_);
        f.out_idx = (const int*)(d_inbox_ + off_out_);
        f.admit = (const int*)(d_inbox_ + off_admit_);
        f.hdr = (const sbk::AdmitHeader*)(d_inbox_ + off_hdr_);
        f.in_t = (const float*)(d_inbox_ + off_t_);
        f.in_band = (const int*)(d_inbox_ + off_band_);
        f.in_data = (const float*)(d_inbox_ + off_data_);
        f.in_w = (const float*)(d_inbox_ + off_w_);
        f.n_active = n_active;
        f.iters = cfg.iters_per_tick;
        f.fit_iters = cfg.fit_iters;
        f.lambda0 = (float)cfg.lm_lambda0;
        f.solver = cfg.solver;
        f.lbfgs_m = cfg.lbfgs_m;
        f.t = d_t_;
        f.band = d_band_;
        f.data = d_data_;
        f.w = d_w_;
        f.err = ctx_->d_err;
        if (e == hipSuccess) e = sbk::launch_fit(ctx_->km, ctx_->tables(), f, stream_);
        if (e == hipSuccess && n_fin > 0)
          e = hipMemcpyAsync(h_res_[parity], d_results_, (size_t)n_fin * sizeof(sbk::FitSlot),
                             hipMemcpyDeviceToHost, stream_);
      }
      if (e == hipSuccess) e = hipEventRecord(ev_[parity], stream_);
      if (e != hipSuccess) {
        fail_all(SB_ERR_DEVICE, std::string("fit server launch: ") + hipGetErrorString(e));
        std::lock_guard<std::mutex> lk(mu_);
        for (const Retire& r : retire) release_slot(r.slot);
        continue;
      }
      {
        std::lock_guard<std::mutex> lk(mu_);
        ticks_[parity].pending = true;
        ticks_[parity].retire = std::move(retire);
        ++n_ticks_;
        n_slot_ticks_ += n_active;
      }
    }
    if (ticks_[1 - parity].pending) finish_tick(1 - parity);
    if (launch) {
      std::lock_guard<std::mutex> lk(mu_);
      if (n_active > 0) busy_s_ += now_seconds() - t_prep;
      parity = 1 - parity;
    }
  }
}

}  // namespace sbh

// ------------------------------------------------------------------ C ABI

extern "C" {

sb_status sb_fit_submit(sb_ctx* ctx, const sb_fit_request* req, uint64_t* ticket) {
  if (!ctx) return sbh::set_error(SB_ERR_ARG, "sb_fit_submit: NULL context");
  if (ctx->n_bands == 0) return sbh::set_error(SB_ERR_STATE, "sb_fit_submit: no band registered");
  {
    std::lock_guard<std::mutex> lk(ctx->mu);
    if (!ctx->server) {
      sbh::Server* s = new sbh::Server(ctx);
      sb_status st = s->start();
      if (st != SB_OK) {
        delete s;
        return st;
      }
      ctx->server = s;
    }
  }
  return ctx->server->submit(req, ticket);
}

sb_status sb_fit_poll(sb_ctx* ctx, uint64_t ticket, sb_fit_result* out) {
  if (!ctx) return sbh::set_error(SB_ERR_ARG, "sb_fit_poll: NULL context");
  if (!ctx->server) return sbh::set_error(SB_ERR_NOTFOUND, "sb_fit_poll: no fit submitted");
  return ctx->server->poll(ticket, out);
}

sb_status sb_fit_wait(sb_ctx* ctx, uint64_t ticket, double timeout_s, sb_fit_result* out) {
  if (!ctx) return sbh::set_error(SB_ERR_ARG, "sb_fit_wait: NULL context");
  if (!ctx->server) return sbh::set_error(SB_ERR_NOTFOUND, "sb_fit_wait: no fit submitted");
  return ctx->server->wait(ticket, timeout_s, out);
}

sb_status sb_fit_cancel(sb_ctx* ctx, uint64_t ticket) {
  if (!ctx) return sbh::set_error(SB_ERR_ARG, "sb_fit_cancel: NULL context");
  if (!ctx->server) return sbh::set_error(SB_ERR_NOTFOUND, "sb_fit_cancel: no fit submitted");
  return ctx->server->cancel(ticket);
}

sb_status sb_stats(sb_ctx* ctx, sb_stats_t* out) {
  if (!ctx || !out) return sbh::set_error(SB_ERR_ARG, "sb_stats: NULL argument");
  std::memset(out, 0, sizeof(*out));
  out->budget_bytes = ctx->cfg.hbm_budget_bytes;
  if (ctx->server) ctx->server->stats(out);
  return SB_OK;
}

}  // extern "C"
