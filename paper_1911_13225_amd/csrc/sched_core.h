// Device-independent core of the serving loop: the request queue, tickets,
// admission of pooled resources (contiguous ray-slot ranges, image slots, a
// latent slot and the device buffers a backend charges against its budget),
// the per-tick table of images that start rays (the coarse-to-fine schedule
// of Sec. 3.2: the coarsest level at step 0, one finer level after every
// third step), completion, failure and cancellation.  A Backend does the
// device work; the HIP server is one backend, and a null-device backend
// drives the same state machine on the CPU (tests, ThreadSanitizer).
//
// Threads: submit() and poll() may be called from any thread; one scheduler
// thread (start()) owns admission, the running list and every backend call.
// The queue, the ticket map and the published results are guarded by mu.
#pragma once

#include <chrono>
#include <condition_variable>
#include <cstdint>
#include <deque>
#include <iterator>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "dist.h"

namespace dist {
namespace sched {

using Clock = std::chrono::steady_clock;

// First-fit allocator of contiguous ray-slot ranges.
struct SlotAlloc {
  std::map<int, int> free_;     // begin -> count
  void init(int cap) { free_.clear(); free_[0] = cap; }
  int alloc(int n) {
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= n) {
        const int b = it->first, c = it->second;
        free_.erase(it);
        if (c > n) free_[b + n] = c - n;
        return b;
      }
    }
    return -1;
  }
  void release(int b, int n) {
    auto it = free_.emplace(b, n).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
};

// A request as the scheduler sees it; a backend derives its own type with
// the device buffers.
struct Job {
  virtual ~Job() = default;
  uint64_t ticket = 0;
  int kind = DIST_REQ_RENDER;
  int n_views = 0, H = 0, W = 0, hw = 0, levels = 0, spi = 0, max_steps = 0, iters = 1;
  // pooled resources
  int slot_base = -1;
  std::vector<int> imgs;        // image slots, view order
  int lat = -1;
  // progress (scheduler thread)
  int step = 0, iter = 0;
  std::vector<char> img_done;
  bool finished = false;        // render / optimisation complete
  int error = DIST_OK;          // set by the backend: the job ends with this code (e.g. DIST_ENUMERIC)
  // published result (under mu)
  bool done = false;
  int status = DIST_OK;
  int64_t queries = 0;
  float final_loss = 0.f;
  Clock::time_point t_submit, t_done;
  // restart the render from step 0 (a z-opt job's next iteration)
  void restart() {
    step = 0;
    img_done.assign(n_views, 0);
  }
};

// An image that starts rays this tick: its level, whether its rays come from
// a split of the coarser level, and where its new rays go in the tick's list.
struct TickEntry {
  int img, lvl, step, split, begin, count;
};

struct Backend {
  virtual ~Backend() = default;
  // device buffers of a job beyond its pooled slots (charged against the
  // backend's budget); false: not now (the job waits in the queue)
  virtual bool acquire(Job* j) = 0;
  virtual void release(Job* j) = 0;
  // the job holds its ray slots, image slots and latent: descriptors,
  // latent code, optimiser state, first render
  virtual void begin(Job* j) = 0;
  // one tick: start the table's rays, march every pooled active ray, and
  // make active(img) / queries(img) current; DIST_OK or an error code
  virtual int tick(const std::vector<TickEntry>& table, int n_new) = 0;
  virtual int active(int img) const = 0;
  virtual int64_t queries(int img) const = 0;
  // every image of j is done: outputs (render) or loss, gradient and the
  // optimiser step (z-opt); sets j->finished, or restarts the job's render;
  // may set j->error (the job then ends with that code)
  virtual void complete(Job* j) = 0;
  // before j's result is published: its device work has drained and
  // j->final_loss is set
  virtual void settle(Job* j) = 0;
  // after a failed tick: no ray of a failed job may stay in the pooled lists
  virtual void drop_rays() = 0;
  // the loop found nothing to run; wait briefly for resources to free up
  virtual void idle() { std::this_thread::sleep_for(std::chrono::microseconds(200)); }
  // first thing the scheduler thread does (select the device)
  virtual void thread_init() {}
};

class Core {
 public:
  Core(Backend* be, int cap_rays, int cap_imgs, int cap_lat, int max_pending)
      : be_(be), cap_rays_(cap_rays), max_pending_(max_pending) {
    slots_.init(cap_rays);
    for (int i = cap_imgs - 1; i >= 0; --i) free_imgs_.push_back(i);
    for (int i = cap_lat - 1; i >= 0; --i) free_lats_.push_back(i);
  }
  ~Core() {
    shutdown();
    for (auto& kv : tickets_) delete kv.second;
  }
  int cap_rays() const { return cap_rays_; }

  void start() { th_ = std::thread([this] { run(); }); }

  // Queue a job (ownership passes to the core); DIST_EBUSY when the queue is full.
  int submit(Job* j, uint64_t* ticket) {
    std::lock_guard<std::mutex> lk(mu_);
    if (stop_) {
      delete j;
      return DIST_ECANCELLED;
    }
    if ((int)pending_.size() >= max_pending_) {
      delete j;
      return DIST_EBUSY;
    }
    j->ticket = next_ticket_++;
    j->t_submit = Clock::now();
    tickets_[j->ticket] = j;
    pending_.push_back(j);
    *ticket = j->ticket;
    cv_sub_.notify_all();
    return DIST_OK;
  }

  // DIST_OK with *res filled (the ticket is then released), DIST_PENDING,
  // or DIST_ENOTFOUND.  timeout_us < 0 waits until the job is done.
  int poll(uint64_t ticket, dist_result* res, int64_t timeout_us) {
    std::unique_lock<std::mutex> lk(mu_);
    auto it = tickets_.find(ticket);
    if (it == tickets_.end()) return DIST_ENOTFOUND;
    Job* j = it->second;
    auto done = [&] { return j->done; };
    if (!done()) {
      if (timeout_us == 0) return DIST_PENDING;
      // a system-clock deadline (pthread_cond_timedwait, which ThreadSanitizer
      // follows; the steady-clock wait of wait_for is not intercepted there)
      if (timeout_us < 0) cv_done_.wait(lk, done);
      else if (!cv_done_.wait_until(lk, std::chrono::system_clock::now() + std::chrono::microseconds(timeout_us), done))
        return DIST_PENDING;
    }
    res->status = j->status;
    res->latency_ns = std::chrono::duration_cast<std::chrono::nanoseconds>(j->t_done - j->t_submit).count();
    res->queries = j->queries;
    res->final_loss = j->final_loss;
    tickets_.erase(it);
    delete j;
    return DIST_OK;
  }

  // Stop the scheduler thread; jobs still queued or running finish with
  // DIST_ECANCELLED (their tickets stay pollable).
  void shutdown() {
    {
      std::lock_guard<std::mutex> lk(mu_);
      stop_ = true;
    }
    cv_sub_.notify_all();
    if (th_.joinable()) th_.join();
  }

 private:
  bool try_admit(Job* j) {
    const int need = j->n_views * j->spi;
    if ((int)free_imgs_.size() < j->n_views || free_lats_.empty()) return false;
    if (!be_->acquire(j)) return false;
    const int base = slots_.alloc(need);
    if (base < 0) {
      be_->release(j);
      return false;
    }
    j->slot_base = base;
    j->lat = free_lats_.back();
    free_lats_.pop_back();
    j->imgs.resize(j->n_views);
    for (int v = 0; v < j->n_views; ++v) {
      j->imgs[v] = free_imgs_.back();
      free_imgs_.pop_back();
    }
    j->restart();
    be_->begin(j);
    return true;
  }

  void release(Job* j) {
    if (j->slot_base >= 0) {
      slots_.release(j->slot_base, j->n_views * j->spi);
      be_->release(j);
    }
    j->slot_base = -1;
    for (int i : j->imgs) free_imgs_.push_back(i);
    j->imgs.clear();
    if (j->lat >= 0) free_lats_.push_back(j->lat);
    j->lat = -1;
  }

  void finish(Job* j, int status) {
    if (j->slot_base >= 0) be_->settle(j);
    release(j);
    std::lock_guard<std::mutex> lk(mu_);
    j->status = status == DIST_OK && j->error != DIST_OK ? j->error : status;
    j->t_done = Clock::now();
    j->finished = true;
    j->done = true;
    cv_done_.notify_all();
  }

  void run() {
    be_->thread_init();
    while (true) {
      // admission
      {
        std::unique_lock<std::mutex> lk(mu_);
        if (stop_) break;
        if (running_.empty() && pending_.empty()) {
          cv_sub_.wait(lk, [&] { return stop_ || !pending_.empty(); });
          if (stop_) break;
        }
      }
      while (true) {
        Job* j = nullptr;
        {
          std::lock_guard<std::mutex> lk(mu_);
          if (pending_.empty()) break;
          j = pending_.front();
        }
        if (!try_admit(j)) break;
        std::lock_guard<std::mutex> lk(mu_);
        pending_.pop_front();
        running_.push_back(j);
      }
      if (running_.empty()) {
        be_->idle();
        continue;
      }
      // the tick's table of images that start rays
      table_.clear();
      int n_new = 0;
      for (Job* j : running_) {
        const int L = j->levels;
        int lvl = -1, split = 0;
        if (j->step == 0) {
          lvl = L;
        } else if (j->step % 3 == 0 && j->step / 3 <= L) {
          lvl = L - j->step / 3;
          split = 1;
        }
        if (lvl < 0) continue;
        for (int v = 0; v < j->n_views; ++v) {
          const int count = (j->H >> lvl) * (j->W >> lvl);
          table_.push_back(TickEntry{j->imgs[v], lvl, j->step, split, n_new, count});
          n_new += count;
        }
      }
      if (be_->tick(table_, n_new) != DIST_OK) {
        // device failure: fail every running job
        std::vector<Job*> js;
        js.swap(running_);
        for (Job* j : js) finish(j, DIST_EHIP);
        be_->drop_rays();
        continue;
      }
      // progress and completion
      std::vector<Job*> keep;
      for (Job* j : running_) {
        j->step += 1;
        bool all = true;
        for (int v = 0; v < j->n_views; ++v) {
          if (!j->img_done[v]) {
            const bool no_more_splits = j->step > 3 * j->levels;
            if (j->step >= j->max_steps || (no_more_splits && be_->active(j->imgs[v]) == 0)) j->img_done[v] = 1;
          }
          all = all && j->img_done[v];
        }
        if (!all) {
          keep.push_back(j);
          continue;
        }
        be_->complete(j);
        if (j->finished) {
          int64_t q = 0;
          for (int img : j->imgs) q += be_->queries(img);
          j->queries = q;
          finish(j, DIST_OK);
        } else {
          keep.push_back(j);
        }
      }
      running_.swap(keep);
    }
    // cancel what is left
    std::vector<Job*> rest;
    {
      std::lock_guard<std::mutex> lk(mu_);
      rest.swap(running_);
      for (Job* j : pending_) rest.push_back(j);
      pending_.clear();
    }
    for (Job* j : rest) finish(j, DIST_ECANCELLED);
  }

  Backend* be_;
  int cap_rays_, max_pending_;
  std::thread th_;
  std::mutex mu_;
  std::condition_variable cv_sub_, cv_done_;
  bool stop_ = false;
  std::deque<Job*> pending_;
  std::map<uint64_t, Job*> tickets_;
  uint64_t next_ticket_ = 1;
  // scheduler thread
  std::vector<Job*> running_;
  std::vector<TickEntry> table_;
  SlotAlloc slots_;
  std::vector<int> free_imgs_, free_lats_;
};

}  // namespace sched
}  // namespace dist
