// The serving loop's scheduler core driven by a null device on the CPU: the
// same queue, tickets, admission, coarse-to-fine tick table and completion /
// failure / cancellation paths as the HIP server, with a device model in
// which each started image stays active for a fixed number of ticks.  Built
// with ThreadSanitizer by tests/test_sched_null.py; each scenario prints
// "ok <name>" and exits 0, or prints the failed check and exits 1.
#include <atomic>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <random>
#include <set>
#include <string>
#include <thread>
#include <vector>

#include "sched_core.h"

using namespace dist::sched;

#define CHECK(c)                                                              \
  do {                                                                        \
    if (!(c)) {                                                               \
      std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c);    \
      std::exit(1);                                                           \
    }                                                                         \
  } while (0)

struct NullJob : Job {
  int life = 1;                 // ticks an image stays active after its rays start
  size_t bytes = 0;             // device buffers the backend charges
};

// The device model.  Every method runs on the scheduler thread only, so the
// backend holds no lock; ThreadSanitizer reports it if the core ever calls it
// from another thread.
struct NullBackend : Backend {
  explicit NullBackend(int cap_imgs, size_t budget)
      : remaining(cap_imgs, 0), act(cap_imgs, 0), q(cap_imgs, 0), owner(cap_imgs, 0), budget(budget) {}
  std::vector<int> remaining, act;
  std::vector<int64_t> q;
  std::vector<uint64_t> owner;             // ticket holding each image slot (0: free)
  std::map<int, std::pair<int, uint64_t>> ranges;   // live ray-slot ranges: begin -> (count, ticket)
  std::map<uint64_t, int> life_of;
  size_t budget, used = 0;
  int acquire_calls = 0, fail_acquire_every = 0, ticks = 0, fail_tick_at = -1;
  int numeric_every = 0;                   // every n-th ticket's render meets a non-finite query
  bool block = false;
  int tick_failures = 0, max_running_imgs = 0;

  bool acquire(Job* j) override {
    ++acquire_calls;
    if (block) return false;
    if (fail_acquire_every && acquire_calls % fail_acquire_every == 0) return false;   // injected failure
    NullJob* n = static_cast<NullJob*>(j);
    if (used + n->bytes > budget) return false;
    used += n->bytes;
    return true;
  }
  void release(Job* j) override {
    NullJob* n = static_cast<NullJob*>(j);
    CHECK(used >= n->bytes);
    used -= n->bytes;
  }
  void begin(Job* j) override {
    NullJob* n = static_cast<NullJob*>(j);
    // every image slot and ray-slot range is held by one job at a time
    for (int img : j->imgs) {
      CHECK(owner[img] == 0);
      owner[img] = j->ticket;
    }
    const int cnt = j->n_views * j->spi;
    auto nx = ranges.lower_bound(j->slot_base);
    if (nx != ranges.end()) CHECK(j->slot_base + cnt <= nx->first);
    if (nx != ranges.begin()) {
      auto pv = std::prev(nx);
      CHECK(pv->first + pv->second.first <= j->slot_base);
    }
    ranges[j->slot_base] = {cnt, j->ticket};
    life_of[j->ticket] = n->life;
    CHECK(j->step == 0 && (int)j->img_done.size() == j->n_views);
  }
  int tick(const std::vector<TickEntry>& table, int n_new) override {
    ++ticks;
    if (ticks == fail_tick_at) {
      ++tick_failures;
      return DIST_EHIP;
    }
    int sum = 0;
    for (const TickEntry& e : table) {
      CHECK(owner[e.img] != 0);
      CHECK(e.begin == sum);
      sum += e.count;
      if (e.step == 0) remaining[e.img] = life_of[owner[e.img]];   // the coarsest level's rays start
    }
    CHECK(sum == n_new);
    int running = 0;
    for (size_t i = 0; i < remaining.size(); ++i) {
      if (remaining[i] > 0) {
        q[i] += remaining[i];
        --remaining[i];
        ++running;
      }
      act[i] = remaining[i];
    }
    max_running_imgs = std::max(max_running_imgs, running);
    return DIST_OK;
  }
  int active(int img) const override { return act[img]; }
  int64_t queries(int img) const override { return q[img]; }
  void complete(Job* j) override {
    CHECK(j->imgs.size() == (size_t)j->n_views);
    if (numeric_every && j->ticket % numeric_every == 0) {
      j->error = DIST_ENUMERIC;
      j->finished = true;
      return;
    }
    if (j->kind == DIST_REQ_ZOPT) {
      ++j->iter;
      if (j->iter >= j->iters) j->finished = true;
      else {
        for (int img : j->imgs) q[img] = 0;
        j->restart();
      }
    } else {
      j->finished = true;
    }
  }
  void settle(Job* j) override {
    if (j->kind == DIST_REQ_ZOPT && j->iter > 0) j->final_loss = 1.f / (1.f + j->iter);
    for (int img : j->imgs) {
      CHECK(owner[img] == j->ticket);
      owner[img] = 0;
      remaining[img] = 0;
      act[img] = 0;
      q[img] = 0;
    }
    auto it = ranges.find(j->slot_base);
    CHECK(it != ranges.end() && it->second.second == j->ticket);
    ranges.erase(it);
  }
  void drop_rays() override {
    std::fill(remaining.begin(), remaining.end(), 0);
    std::fill(act.begin(), act.end(), 0);
  }
  void idle() override { std::this_thread::sleep_for(std::chrono::microseconds(50)); }
};

static NullJob* make_job(std::mt19937& g, int kind) {
  NullJob* j = new NullJob();
  j->kind = kind;
  j->n_views = 1 + (int)(g() % 4);
  const int sizes[4] = {8, 16, 32, 64};
  j->H = j->W = sizes[g() % 4];
  j->hw = j->H * j->W;
  j->levels = (int)(g() % 3);
  // slots of an image: every coarse-to-fine level
  int spi = 0;
  for (int l = 0; l <= j->levels; ++l) spi += (j->H >> l) * (j->W >> l);
  j->spi = spi;
  j->max_steps = 10 + (int)(g() % 30);
  j->iters = kind == DIST_REQ_ZOPT ? 1 + (int)(g() % 3) : 1;
  j->life = 1 + (int)(g() % 25);
  j->bytes = (size_t)j->n_views * j->hw * 64;
  return j;
}

// Many submitters and pollers at once; transient allocation failures; tight
// image and ray-slot pools so jobs wait for each other.
static void mixed() {
  NullBackend be(24, (size_t)8 << 20);
  be.fail_acquire_every = 5;
  Core core(&be, 40000, 24, 16, 4096);
  core.start();
  const int T = 6, N = 120;
  std::atomic<int> ok{0}, zopt_ok{0};
  std::vector<std::thread> th;
  std::vector<std::vector<uint64_t>> seen(T);
  for (int t = 0; t < T; ++t) {
    th.emplace_back([&, t] {
      std::mt19937 g(1000 + t);
      std::vector<std::pair<uint64_t, int>> mine;      // ticket, iters of a z-opt job (0: render)
      for (int i = 0; i < N; ++i) {
        const int kind = g() % 4 == 0 ? DIST_REQ_ZOPT : DIST_REQ_RENDER;
        NullJob* j = make_job(g, kind);
        const int iters = kind == DIST_REQ_ZOPT ? j->iters : 0;
        uint64_t tk = 0;
        CHECK(core.submit(j, &tk) == DIST_OK);
        mine.push_back({tk, iters});
        seen[t].push_back(tk);
      }
      for (auto& [tk, iters] : mine) {
        dist_result r{};
        int rc;
        const int64_t timeouts[3] = {0, 200, -1};
        int k = 0;
        while ((rc = core.poll(tk, &r, timeouts[k++ % 3])) == DIST_PENDING) {
        }
        CHECK(rc == DIST_OK);
        CHECK(r.status == DIST_OK);
        CHECK(r.queries > 0);
        CHECK(r.latency_ns >= 0);
        if (iters) {
          CHECK(r.final_loss == 1.f / (1.f + iters));
          zopt_ok++;
        }
        ok++;
        CHECK(core.poll(tk, &r, 0) == DIST_ENOTFOUND);       // a ticket is released once read
      }
    });
  }
  for (auto& x : th) x.join();
  core.shutdown();
  CHECK(ok == T * N);
  CHECK(zopt_ok > 0);
  std::set<uint64_t> all;
  for (auto& v : seen) all.insert(v.begin(), v.end());
  CHECK((int)all.size() == T * N);                            // tickets are unique
  CHECK(be.used == 0);                                        // every buffer returned
  CHECK(be.ranges.empty());
  CHECK(be.max_running_imgs <= 24);
  dist_result r{};
  CHECK(core.poll(987654321ull, &r, 0) == DIST_ENOTFOUND);
}

// A full queue answers DIST_EBUSY; shutting down cancels what is queued.
static void busy() {
  NullBackend be(8, 1 << 20);
  be.block = true;                                            // no job is ever admitted
  Core core(&be, 1 << 16, 8, 8, 16);
  core.start();
  std::mt19937 g(7);
  std::vector<uint64_t> tks;
  int busy = 0;
  for (int i = 0; i < 20; ++i) {
    uint64_t tk = 0;
    const int rc = core.submit(make_job(g, DIST_REQ_RENDER), &tk);
    if (rc == DIST_OK) tks.push_back(tk);
    else {
      CHECK(rc == DIST_EBUSY);
      ++busy;
    }
  }
  CHECK(tks.size() == 16 && busy == 4);
  dist_result r{};
  CHECK(core.poll(tks[0], &r, 1000) == DIST_PENDING);
  core.shutdown();
  for (uint64_t tk : tks) {
    CHECK(core.poll(tk, &r, -1) == DIST_OK);
    CHECK(r.status == DIST_ECANCELLED);
  }
  uint64_t tk = 0;
  CHECK(core.submit(make_job(g, DIST_REQ_RENDER), &tk) == DIST_ECANCELLED);
}

// Shutdown while jobs run: each ends DIST_OK or DIST_ECANCELLED, and a
// poller blocked on a running job is woken.
static void cancel() {
  NullBackend be(64, (size_t)64 << 20);
  Core core(&be, 1 << 18, 64, 64, 4096);
  core.start();
  std::mt19937 g(11);
  std::vector<uint64_t> tks;
  for (int i = 0; i < 80; ++i) {
    NullJob* j = make_job(g, i % 2 ? DIST_REQ_ZOPT : DIST_REQ_RENDER);
    j->life = 1 << 20;                  // still marching when the server stops
    j->max_steps = 1 << 30;
    uint64_t tk = 0;
    CHECK(core.submit(j, &tk) == DIST_OK);
    tks.push_back(tk);
  }
  std::atomic<int> woke{0};
  std::thread waiter([&] {
    dist_result r{};
    CHECK(core.poll(tks.back(), &r, -1) == DIST_OK);
    CHECK(r.status == DIST_OK || r.status == DIST_ECANCELLED);
    woke++;
  });
  std::this_thread::sleep_for(std::chrono::milliseconds(20));
  core.shutdown();
  waiter.join();
  CHECK(woke == 1);
  int cancelled = 0;
  for (size_t i = 0; i + 1 < tks.size(); ++i) {
    dist_result r{};
    CHECK(core.poll(tks[i], &r, 0) == DIST_OK);
    CHECK(r.status == DIST_OK || r.status == DIST_ECANCELLED);
    cancelled += r.status == DIST_ECANCELLED;
  }
  CHECK(cancelled > 0);
  CHECK(be.used == 0 && be.ranges.empty());
}

// A failed tick fails every running job with DIST_EHIP and drops the pooled
// rays; jobs admitted afterwards complete.
static void tickfail() {
  NullBackend be(16, (size_t)16 << 20);
  be.fail_tick_at = 4;
  Core core(&be, 1 << 16, 16, 16, 4096);
  core.start();
  std::mt19937 g(5);
  std::vector<uint64_t> tks;
  for (int i = 0; i < 40; ++i) {
    uint64_t tk = 0;
    NullJob* j = make_job(g, DIST_REQ_RENDER);
    j->life = 8;
    CHECK(core.submit(j, &tk) == DIST_OK);
    tks.push_back(tk);
  }
  int failed = 0, ok = 0;
  for (uint64_t tk : tks) {
    dist_result r{};
    CHECK(core.poll(tk, &r, -1) == DIST_OK);
    CHECK(r.status == DIST_OK || r.status == DIST_EHIP);
    failed += r.status == DIST_EHIP;
    ok += r.status == DIST_OK;
  }
  core.shutdown();
  CHECK(be.tick_failures == 1);
  CHECK(failed > 0 && ok > 0);
  CHECK(be.used == 0 && be.ranges.empty());
}

// A job whose render met a non-finite query ends with DIST_ENUMERIC; the
// others complete.
static void numeric() {
  NullBackend be(16, (size_t)16 << 20);
  be.numeric_every = 3;
  Core core(&be, 1 << 16, 16, 16, 4096);
  core.start();
  std::mt19937 g(9);
  std::vector<uint64_t> tks;
  for (int i = 0; i < 30; ++i) {
    uint64_t tk = 0;
    CHECK(core.submit(make_job(g, i % 2 ? DIST_REQ_ZOPT : DIST_REQ_RENDER), &tk) == DIST_OK);
    tks.push_back(tk);
  }
  for (uint64_t tk : tks) {
    dist_result r{};
    CHECK(core.poll(tk, &r, -1) == DIST_OK);
    CHECK(r.status == (tk % 3 == 0 ? DIST_ENUMERIC : DIST_OK));
  }
  core.shutdown();
  CHECK(be.used == 0 && be.ranges.empty());
}

int main(int argc, char** argv) {
  const std::string s = argc > 1 ? argv[1] : "all";
  if (s == "mixed" || s == "all") { mixed(); std::printf("ok mixed\n"); }
  if (s == "busy" || s == "all") { busy(); std::printf("ok busy\n"); }
  if (s == "cancel" || s == "all") { cancel(); std::printf("ok cancel\n"); }
  if (s == "tickfail" || s == "all") { tickfail(); std::printf("ok tickfail\n"); }
  if (s == "numeric" || s == "all") { numeric(); std::printf("ok numeric\n"); }
  return 0;
}
