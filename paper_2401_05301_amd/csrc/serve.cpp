// Serving loop: quench requests of different L, chi_max and couplings are
// admitted by device-memory footprint and run concurrently, each on its own
// handle, stream and host thread, until their horizon.  Requests that arrive
// while others run are admitted as soon as a slot and enough of the memory
// budget are free (first come, first served), so their work overlaps on the
// device with the requests already running.
//
// Every request is evolved exactly as tebd_step / measure_local would evolve
// it alone: handles share no state, so the result of a request does not
// depend on the mix it ran in.
//
// With continuous batching (tebd_serve_opts.batched) one scheduler thread
// instead steps all admitted requests together: each Strang layer of all of
// them is one fused batch (tebd_step_many), so their small SVDs share one
// batched Jacobi and one host read-back per sweep.  Arrivals are admitted
// and finished requests retired between steps; results are again those of
// each request alone.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "engine.hpp"

namespace {

using Clock = std::chrono::steady_clock;

double seconds_since(Clock::time_point t0) {
  return std::chrono::duration<double>(Clock::now() - t0).count();
}

int64_t gates_per_step(int L) {
  // layers (0, 1, 2, 1, 0): gates j = g, g + 3, ... <= L - 3
  auto count = [L](int g) { return g <= L - 3 ? (int64_t)((L - 3 - g) / 3 + 1) : 0; };
  return 2 * count(0) + 2 * count(1) + count(2);
}

}  // namespace

extern "C" tebd_status tebd_serve(const tebd_request* req, int32_t n, const tebd_serve_opts* so,
                                  tebd_serve_result* res, double* n_out, double* cnn_out, double* cnnn_out) {
  if (n < 0 || (n > 0 && (!req || !so || !res))) {
    ptebd::set_last_error("tebd_serve: bad arguments");
    return TEBD_EINVAL;
  }
  if (n == 0) return TEBD_OK;
  // validate every request and size its footprint before anything runs
  std::vector<size_t> footprint(n);
  std::vector<int64_t> off_n(n + 1, 0), off_c(n + 1, 0), off_d(n + 1, 0);
  std::vector<tebd_opts> opts(n);
  for (int i = 0; i < n; ++i) {
    const tebd_request& r = req[i];
    if (!(r.dt == r.dt) || r.steps < 0 || !(r.arrival >= 0.0) || (r.first_occupied != 0 && r.first_occupied != 1)) {
      ptebd::set_last_error("tebd_serve: request " + std::to_string(i) + " has a bad dt, steps, arrival or parity");
      return TEBD_EINVAL;
    }
    tebd_opts& o = opts[i];
    tebd_opts_default(&o);
    o.chi_max = r.chi_max;
    o.trunc_weight = so->trunc_weight;
    o.trunc_rel = so->trunc_rel;
    o.prec = so->prec;
    o.svd = so->svd;
    o.u1 = so->u1;
    o.fuse = so->batched ? 1 : 0;
    o.workers = so->workers_per_request > 0 ? so->workers_per_request : (so->batched ? 0 : 1);
    tebd_status st = mps_footprint(&r.model, &o, &footprint[i]);
    if (st) return st;   // message set by mps_footprint
    off_n[i + 1] = off_n[i] + r.model.L;
    off_c[i + 1] = off_c[i] + 2 * (r.model.L - 1);
    off_d[i + 1] = off_d[i] + 2 * (r.model.L - 2);
  }
  size_t budget = so->hbm_budget > 0 ? (size_t)so->hbm_budget : 0;
  if (budget == 0) {
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) {
      (void)hipGetLastError();
      ptebd::set_last_error("tebd_serve: hipMemGetInfo failed");
      return TEBD_EDEVICE;
    }
    budget = (size_t)(0.85 * (double)free_b);
  }
  for (int i = 0; i < n; ++i)
    if (footprint[i] > budget) {
      ptebd::set_last_error("tebd_serve: request " + std::to_string(i) + " needs " + std::to_string(footprint[i]) +
                            " bytes, above the budget of " + std::to_string(budget));
      return TEBD_ENOMEM;
    }
  const int slots = so->max_active > 0 ? so->max_active : 8;
  if (so->batched != 0 && so->batched != 1) {
    ptebd::set_last_error("tebd_serve: batched must be 0 or 1");
    return TEBD_EINVAL;
  }

  // arrival order (stable for equal times)
  std::vector<int> order(n);
  for (int i = 0; i < n; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return req[a].arrival < req[b].arrival; });

  if (so->batched) {
    // Continuous batching: admitted requests are stepped together, one
    // fused batch per Strang layer; requests join and leave between steps.
    struct Live {
      int i;
      tebd_mps* M;
      int done;
    };
    std::vector<Live> live;
    size_t reserved = 0;
    const Clock::time_point t0 = Clock::now();
    const int every = so->measure_every;
    auto measure = [&](int i, tebd_mps* M) {
      return measure_local(M, n_out ? n_out + off_n[i] : nullptr, cnn_out ? cnn_out + off_c[i] : nullptr,
                           cnnn_out ? cnnn_out + off_d[i] : nullptr);
    };
    auto finish = [&](int i, tebd_mps* M, tebd_status st) {
      if (!st) st = measure(i, M);
      double w = 0.0;
      if (!st) st = mps_discarded_weight(M, &w);
      if (M) mps_free(M);
      res[i].status = st;
      res[i].discarded_weight = w;
      res[i].gate_updates = st ? 0 : (int64_t)req[i].steps * gates_per_step(req[i].model.L);
      res[i].finished = seconds_since(t0);
      reserved -= footprint[i];
    };
    int next = 0;
    while (next < n || !live.empty()) {
      while (next < n) {   // admit, first come first served, while a slot and the memory are free
        const int i = order[next];
        if (seconds_since(t0) < req[i].arrival || (int)live.size() >= slots || reserved + footprint[i] > budget)
          break;
        res[i].arrival = req[i].arrival;
        res[i].admitted = seconds_since(t0);
        reserved += footprint[i];
        ++next;
        tebd_mps* M = nullptr;
        tebd_status st = mps_init_cdw(&req[i].model, &opts[i], req[i].first_occupied, &M);
        if (!st) st = tebd_prepare(M, req[i].dt);
        if (st || req[i].steps == 0)
          finish(i, M, st);
        else
          live.push_back(Live{i, M, 0});
      }
      if (live.empty()) {
        if (next < n) {
          const double wait = req[order[next]].arrival - seconds_since(t0);
          if (wait > 0) std::this_thread::sleep_for(std::chrono::duration<double>(wait));
        }
        continue;
      }
      std::vector<tebd_mps*> hs;
      std::vector<double> dts;
      for (const Live& x : live) {
        hs.push_back(x.M);
        dts.push_back(req[x.i].dt);
      }
      const tebd_status st = tebd_step_many(hs.data(), (int32_t)hs.size(), dts.data());
      std::vector<Live> keep;
      for (Live& x : live) {
        tebd_status sx = st;
        ++x.done;
        if (!sx && every > 0 && x.done % every == 0 && x.done < req[x.i].steps) sx = measure(x.i, x.M);
        if (sx || x.done == req[x.i].steps)
          finish(x.i, x.M, sx);
        else
          keep.push_back(x);
      }
      live.swap(keep);
    }
    tebd_status first = TEBD_OK;
    for (int i = 0; i < n && !first; ++i) first = (tebd_status)res[i].status;
    if (first) ptebd::set_last_error("tebd_serve: at least one request failed (see the per-request status)");
    return first;
  }

  std::mutex mu;
  std::condition_variable cv;
  int active = 0;
  size_t reserved = 0;
  std::vector<std::thread> threads;
  threads.reserve(n);
  const Clock::time_point t0 = Clock::now();

  auto run = [&](int i) {
    const tebd_request& r = req[i];
    tebd_serve_result& out = res[i];
    tebd_mps* M = nullptr;
    tebd_status st = mps_init_cdw(&r.model, &opts[i], r.first_occupied, &M);
    if (!st) st = tebd_prepare(M, r.dt);
    const int every = so->measure_every;
    for (int k = 0; !st && k < r.steps; ++k) {
      st = tebd_step(M, r.dt);
      if (!st && every > 0 && (k + 1) % every == 0 && k + 1 < r.steps)
        st = measure_local(M, n_out ? n_out + off_n[i] : nullptr, cnn_out ? cnn_out + off_c[i] : nullptr,
                           cnnn_out ? cnnn_out + off_d[i] : nullptr);
    }
    if (!st)
      st = measure_local(M, n_out ? n_out + off_n[i] : nullptr, cnn_out ? cnn_out + off_c[i] : nullptr,
                         cnnn_out ? cnnn_out + off_d[i] : nullptr);
    double w = 0.0;
    if (!st) st = mps_discarded_weight(M, &w);
    if (M) mps_free(M);
    out.status = st;
    out.discarded_weight = w;
    out.gate_updates = st ? 0 : (int64_t)r.steps * gates_per_step(r.model.L);
    {
      std::lock_guard<std::mutex> lk(mu);
      out.finished = seconds_since(t0);
      --active;
      reserved -= footprint[i];
    }
    cv.notify_all();
  };

  int next = 0;   // next request in arrival order to admit
  {
    std::unique_lock<std::mutex> lk(mu);
    while (next < n) {
      const int i = order[next];
      const double now = seconds_since(t0);
      if (now < req[i].arrival) {
        cv.wait_for(lk, std::chrono::duration<double>(req[i].arrival - now));
        continue;
      }
      if (active < slots && reserved + footprint[i] <= budget) {
        ++active;
        reserved += footprint[i];
        res[i].admitted = seconds_since(t0);
        res[i].arrival = req[i].arrival;
        threads.emplace_back(run, i);
        ++next;
        continue;
      }
      cv.wait(lk);   // a request finished: slot or memory may be free now
    }
  }
  for (auto& t : threads) t.join();
  tebd_status first = TEBD_OK;
  for (int i = 0; i < n && !first; ++i) first = (tebd_status)res[i].status;
  if (first) ptebd::set_last_error("tebd_serve: at least one request failed (see the per-request status)");
  return first;
}
