// Continuous-batching fit server: a host scheduler thread that owns a HIP
// stream, a slot array and an observation arena on the device.
#pragma once

#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "sb_ctx.h"

namespace sbh {

// First-fit allocator over [0, capacity) observation units.
class Arena {
 public:
  explicit Arena(int capacity = 0) { reset(capacity); }
  void reset(int capacity);
  int alloc(int n);          // offset, or -1
  void release(int off, int n);
  int capacity() const { return cap_; }

 private:
  int cap_ = 0;
  std::map<int, int> free_;  // offset -> length, non-adjacent
};

class Server {
 public:
  explicit Server(sb_ctx* ctx);
  ~Server();
  sb_status start();
  sb_status submit(const sb_fit_request* req, uint64_t* ticket);
  sb_status poll(uint64_t ticket, sb_fit_result* out);
  sb_status wait(uint64_t ticket, double timeout_s, sb_fit_result* out);
  sb_status cancel(uint64_t ticket);
  void stats(sb_stats_t* out);

 private:
  struct Request {
    uint64_t ticket;
    std::vector<float> t, data, w;
    std::vector<int> band;
    float z, t0, x0, x1, c;
    int free_mask;
    float lo[4], hi[4];   // bounds of (t0, ln x0, x1, c); +-inf when none
    double t_submit;
    int64_t bytes;
  };
  enum State { QUEUED, ACTIVE, DONE };
  struct Entry {
    State state = QUEUED;
    int slot = -1;
    bool cancel = false;
    sb_fit_result res{};
  };
  struct Slot {
    bool used = false;
    uint64_t ticket = 0;
    int arena_off = 0;
    int n_obs = 0;
    int ticks_left = 0;
    int64_t bytes = 0;
    int free_mask = SB_FREE_ALL;
    float x0 = 0.f;     // starting x0, reported as given when x0 is held fixed
  };
  struct Retire {       // slot to release once its last launch has completed
    int slot;
    int out_idx;        // -1: no result to publish (cancelled)
  };
  struct Tick {
    bool pending = false;
    std::vector<Retire> retire;
  };

  void loop();
  bool prepare_tick(int parity, std::vector<Retire>& retire, size_t& blob_bytes, int& n_active, int& n_fin);
  void finish_tick(int parity);
  void fail_all(sb_status st, const std::string& msg);
  void release_slot(int s);

  sb_ctx* ctx_;
  std::mutex mu_;
  std::condition_variable cv_work_, cv_done_;
  std::thread th_;
  bool stop_ = false;
  bool started_ = false;
  sb_status poisoned_ = SB_OK;
  std::string poison_msg_;

  std::deque<Request> queue_;
  std::unordered_map<uint64_t, Entry> tickets_;
  uint64_t next_ticket_ = 1;
  std::vector<Slot> slots_;
  std::vector<int> free_slots_;
  Arena arena_;
  int64_t bytes_in_use_ = 0;

  // stats
  int64_t n_submitted_ = 0, n_admitted_ = 0, n_completed_ = 0, n_cancelled_ = 0, n_rejected_ = 0, n_ticks_ = 0,
          n_slot_ticks_ = 0;
  int n_active_slots_ = 0;
  double busy_s_ = 0.0;
  int64_t lat_hist_[SB_LATENCY_BINS] = {};

  // device side
  hipStream_t stream_ = nullptr;
  hipEvent_t ev_[2] = {nullptr, nullptr};
  sbk::FitSlot* d_slots_ = nullptr;
  sbk::FitSlot* d_results_ = nullptr;
  float* d_t_ = nullptr;
  int* d_band_ = nullptr;
  float* d_data_ = nullptr;
  float* d_w_ = nullptr;
  char* d_inbox_ = nullptr;
  char* h_inbox_[2] = {nullptr, nullptr};
  sbk::FitSlot* h_res_[2] = {nullptr, nullptr};
  size_t inbox_bytes_ = 0;
  int inbox_obs_ = 0;
  Tick ticks_[2];
  // layout of the inbox for the current tick
  size_t off_active_ = 0, off_out_ = 0, off_admit_ = 0, off_hdr_ = 0, off_t_ = 0, off_band_ = 0,
         off_data_ = 0, off_w_ = 0;
};

}  // namespace sbh
