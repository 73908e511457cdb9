// Batched serving (include/mm.h, second part): many simulations resident in
// one engine, each a segment of the shared launches, a slot pool holding
// their positions, charges and mesh velocities, first-fit placement of each
// simulation's slot range, admission by device footprint, and a first-come,
// first-served serving loop over a request trace.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "../../include/mm.h"
#include "mm_engine.h"
#include "mm_internal.h"

using namespace mm;

namespace {

constexpr int64_t kPoolBytesPerSlot = 8 * (3 + 5 + 3) + 4;   // pos, Q, w, slot segment
constexpr int64_t kPoolSlotsPerCell = 2;                      // slot pool over-provisioned against fragmentation
constexpr int64_t kMinPoints = 3;

struct Sim {
  bool used = false;
  int64_t base = 0, n = 0;
  mm_params p{};
  double dt_max = INFINITY;
  int fresh = 0;
  int64_t steps = 0;
  double t = 0.0;
  int status = MM_OK;   // sticky: a failed simulation is parked
  mm_sim_info last{};
};

thread_local std::string g_batch_create_err;

}  // namespace

struct mm_batch {
  Engine E;
  int precision = MM_FP64;
  int max_sims = 0;
  int64_t slot_cap = 0;
  double *pos = nullptr, *Q = nullptr, *w = nullptr;
  int32_t* slot_seg = nullptr;
  std::vector<Sim> sims;                                  // by id
  std::vector<std::pair<int64_t, int64_t>> free_ranges;   // [start, length), sorted by start
  int64_t cells = 0;
  bool layout_dirty = true;                               // slot segments must be rewritten
  std::vector<int> order;                                 // ids of the simulations stepped, in segment order
  std::string err;

  mm_status fail(mm_status code, const std::string& msg) {
    err = msg;
    return code;
  }
};

namespace {

int64_t per_cell_bytes(int precision) {
  return engine_bytes_per_cell(precision) + kPoolSlotsPerCell * kPoolBytesPerSlot;
}

// First fit of n slots; -1 if no free range is long enough.
int64_t take_range(mm_batch* b, int64_t n) {
  for (size_t k = 0; k < b->free_ranges.size(); ++k) {
    auto& r = b->free_ranges[k];
    if (r.second >= n) {
      const int64_t start = r.first;
      r.first += n;
      r.second -= n;
      if (r.second == 0) b->free_ranges.erase(b->free_ranges.begin() + (long)k);
      return start;
    }
  }
  return -1;
}

void give_range(mm_batch* b, int64_t start, int64_t n) {
  auto& fr = b->free_ranges;
  auto it = std::lower_bound(fr.begin(), fr.end(), std::make_pair(start, (int64_t)0));
  it = fr.insert(it, {start, n});
  // Merge with the next and the previous range.
  if (it + 1 != fr.end() && it->first + it->second == (it + 1)->first) {
    it->second += (it + 1)->second;
    fr.erase(it + 1);
  }
  if (it != fr.begin() && (it - 1)->first + (it - 1)->second == it->first) {
    (it - 1)->second += it->second;
    fr.erase(it);
  }
}

int64_t slot_high(const mm_batch* b) {
  int64_t hi = 0;
  for (const Sim& s : b->sims)
    if (s.used) hi = std::max(hi, s.base + s.n);
  return hi;
}

double now_s(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

double quantile(std::vector<double> v, double q) {
  if (v.empty()) return 0.0;
  std::sort(v.begin(), v.end());
  const double x = q * (double)(v.size() - 1);
  const size_t i = (size_t)std::floor(x);
  const size_t j = std::min(i + 1, v.size() - 1);
  return v[i] + (x - (double)i) * (v[j] - v[i]);
}

}  // namespace

extern "C" {

int64_t mm_batch_footprint(int32_t precision, int64_t n) {
  if (n < 0) return 0;
  return n * per_cell_bytes(precision) + (int64_t)(sizeof(SegDesc) + sizeof(SegStatus) + 16 * 8);
}

const char* mm_batch_last_error(const mm_batch* b) { return b ? b->err.c_str() : g_batch_create_err.c_str(); }

mm_status mm_batch_create(mm_batch** out, int32_t precision, int64_t hbm_budget, int32_t max_sims,
                          void* hip_stream) {
  if (!out) {
    g_batch_create_err = "out is NULL";
    return MM_EINVAL;
  }
  *out = nullptr;
  if (precision != MM_FP64 && precision != MM_MIXED) {
    g_batch_create_err = "precision must be MM_FP64 or MM_MIXED";
    return MM_EINVAL;
  }
  if (max_sims < 1 || max_sims > (1 << 16)) {
    g_batch_create_err = "max_sims must be in [1, 65536]";
    return MM_EINVAL;
  }
  const int64_t ncap = hbm_budget / per_cell_bytes(precision);
  if (ncap < kMinPoints || ncap > (1ll << 26)) {
    g_batch_create_err = "hbm_budget must hold between 3 and 2^26 points";
    return MM_EINVAL;
  }
  mm_batch* b = new (std::nothrow) mm_batch();
  if (!b) {
    g_batch_create_err = "host allocation failed";
    return MM_ENOMEM;
  }
  b->precision = precision;
  b->max_sims = max_sims;
  b->slot_cap = kPoolSlotsPerCell * ncap;
  mm_status r = b->E.init(precision, ncap, b->slot_cap, kFacesPerCell * ncap, max_sims, (hipStream_t)hip_stream);
  bool ok = r == MM_OK;
  if (ok) {
    ok &= hipMalloc((void**)&b->pos, sizeof(double) * 3 * b->slot_cap) == hipSuccess;
    ok &= hipMalloc((void**)&b->Q, sizeof(double) * 5 * b->slot_cap) == hipSuccess;
    ok &= hipMalloc((void**)&b->w, sizeof(double) * 3 * b->slot_cap) == hipSuccess;
    ok &= hipMalloc((void**)&b->slot_seg, sizeof(int32_t) * b->slot_cap) == hipSuccess;
    if (!ok) r = MM_ENOMEM;
  }
  if (!ok) {
    g_batch_create_err = r == MM_ENOMEM ? "device allocation failed" : b->E.err;
    mm_batch_destroy(b);
    return r;
  }
  b->sims.resize(max_sims);
  b->free_ranges.push_back({0, b->slot_cap});
  *out = b;
  return MM_OK;
}

mm_status mm_batch_destroy(mm_batch* b) {
  if (!b) return MM_EINVAL;
  if (b->E.stream || b->pos) (void)hipStreamSynchronize(b->E.stream);
  void* ptrs[] = {b->pos, b->Q, b->w, b->slot_seg};
  for (void* q : ptrs)
    if (q) (void)hipFree(q);
  b->E.release();
  delete b;
  return MM_OK;
}

mm_status mm_batch_admit(mm_batch* b, const mm_params* p, int64_t n, const double* pos, const double* prim,
                         double dt_max, int32_t* sim) {
  if (!b) return MM_EINVAL;
  if (!p || !pos || !prim || !sim) return b->fail(MM_EINVAL, "NULL argument");
  std::string why;
  if (!params_ok(p, why)) return b->fail(MM_EINVAL, why);
  if (p->precision != b->precision) return b->fail(MM_EINVAL, "precision differs from the batch's");
  if (p->half_step_mesh) return b->fail(MM_EINVAL, "half_step_mesh is available for single simulations only");
  if (p->mach_threshold != 0.0) return b->fail(MM_EINVAL, "the entropy switch is available for single simulations only");
  if (!(dt_max > 0.0)) return b->fail(MM_EINVAL, "dt_max must be positive");
  if (n < kMinPoints) return b->fail(MM_EINVAL, "n must be at least 3");
  if (n > b->E.ncap) return b->fail(MM_ECAPACITY, "n exceeds the batch's point capacity");
  int id = -1;
  for (int k = 0; k < b->max_sims; ++k)
    if (!b->sims[k].used) {
      id = k;
      break;
    }
  if (id < 0) return b->fail(MM_EFULL, "every simulation slot is in use");
  if (b->cells + n > b->E.ncap) return b->fail(MM_EFULL, "not enough device room for the simulation now");
  const int64_t base = take_range(b, n);
  if (base < 0) return b->fail(MM_EFULL, "no free slot range long enough now");
  hipStream_t st = b->E.stream;
  hipError_t e = hipMemcpyAsync(b->pos + 3 * base, pos, sizeof(double) * 3 * n, hipMemcpyDefault, st);
  // Until the first step the charge rows hold the primitives; that step
  // turns them into charges once the cells are known.
  if (e == hipSuccess) e = hipMemcpyAsync(b->Q + 5 * base, prim, sizeof(double) * 5 * n, hipMemcpyDefault, st);
  // The caller may release its buffers once this returns.
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) {
    give_range(b, base, n);
    return b->fail(MM_EHIP, std::string("admission copy: ") + hipGetErrorString(e));
  }
  Sim& s = b->sims[id];
  s = Sim();
  s.used = true;
  s.base = base;
  s.n = n;
  s.p = *p;
  s.dt_max = dt_max;
  s.fresh = 1;
  b->cells += n;
  b->layout_dirty = true;
  *sim = id;
  return MM_OK;
}

mm_status mm_batch_step(mm_batch* b, mm_sim_info* info, int32_t info_cap, int32_t* n_info) {
  if (!b) return MM_EINVAL;
  if (n_info) *n_info = 0;
  Engine& E = b->E;
  // Segments: the healthy resident simulations in slot order.
  if (b->layout_dirty) {
    b->order.clear();
    for (int k = 0; k < b->max_sims; ++k)
      if (b->sims[k].used && b->sims[k].status == MM_OK) b->order.push_back(k);
    std::sort(b->order.begin(), b->order.end(),
              [&](int x, int y) { return b->sims[x].base < b->sims[y].base; });
  }
  const int nseg = (int)b->order.size();
  if (nseg == 0) return MM_OK;
  SegDesc* d = E.staging();
  int64_t nbt = 0, n = 0;
  bool any_fresh = false;
  for (int k = 0; k < nseg; ++k) {
    const Sim& s = b->sims[b->order[k]];
    d[k].g = make_grid(s.p, s.n, E.rfac, nbt);
    d[k].hp = hydro_params(s.p);
    d[k].dt_max = s.dt_max;
    d[k].fresh = s.fresh;
    d[k].pad = 0;
    nbt += d[k].g.nbt;
    n += s.n;
    any_fresh |= s.fresh != 0;
  }
  if (mm_status r = E.upload(nseg)) return b->fail(r, E.err);
  const int64_t hi = slot_high(b);
  if (b->layout_dirty) {
    launch_fill_i32(b->slot_seg, -1, hi, E.stream);
    for (int k = 0; k < nseg; ++k) {
      const Sim& s = b->sims[b->order[k]];
      launch_fill_i32(b->slot_seg + s.base, k, s.n, E.stream);
    }
    b->layout_dirty = false;
  }
  E.n = n;
  E.enqueue_step(b->pos, b->w, b->Q, hi, b->slot_seg, n, nbt, any_fresh);
  if (mm_status r = E.readback()) return b->fail(r, E.err);
  E.finish_timing();
  const DevStatus& g = *E.st_host;
  const bool global_cap = (g.flags & F_FACECAP) != 0;
  std::string msg;
  int out = 0;
  for (int k = 0; k < nseg; ++k) {
    Sim& s = b->sims[b->order[k]];
    const SegStatus& ss = E.segst_host[k];
    int flags = ss.flags | (global_cap ? F_FACECAP : 0);
    const mm_status r = E.check_flags(flags, ss.bad_cell, msg);
    const double dt = std::min(dt_from_bits(ss.dt_bits), s.dt_max);
    mm_sim_info& I = s.last;
    I.sim = b->order[k];
    I.status = r;
    I.n = s.n;
    I.dt = dt;
    for (int q = 0; q < 4; ++q) I.floor_hits[q] = (int64_t)ss.floor_hits[q];
    I.flags = flags;
    I.reserved = 0;
    if (r == MM_OK) {
      s.steps += 1;
      s.t += dt;
      s.fresh = 0;
    } else {
      s.status = r;           // parked until evicted
      b->layout_dirty = true;
      b->err = msg;
    }
    I.steps = s.steps;
    I.t = s.t;
    if (info && out < info_cap) info[out++] = I;
  }
  if (n_info) *n_info = out;
  return global_cap ? b->fail(MM_ECAPACITY, "more unique faces than the batch's face capacity") : MM_OK;
}

mm_status mm_batch_read(mm_batch* b, int32_t sim, double* pos, double* Q, double* w) {
  if (!b) return MM_EINVAL;
  if (sim < 0 || sim >= b->max_sims || !b->sims[sim].used) return b->fail(MM_EINVAL, "no such simulation");
  const Sim& s = b->sims[sim];
  if (s.fresh) return b->fail(MM_ESTATE, "the simulation has not taken a step yet");
  hipStream_t st = b->E.stream;
  hipError_t e = hipSuccess;
  if (pos) e = hipMemcpyAsync(pos, b->pos + 3 * s.base, sizeof(double) * 3 * s.n, hipMemcpyDefault, st);
  if (Q && e == hipSuccess) e = hipMemcpyAsync(Q, b->Q + 5 * s.base, sizeof(double) * 5 * s.n, hipMemcpyDefault, st);
  if (w && e == hipSuccess) e = hipMemcpyAsync(w, b->w + 3 * s.base, sizeof(double) * 3 * s.n, hipMemcpyDefault, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return b->fail(MM_EHIP, std::string("read: ") + hipGetErrorString(e));
  return MM_OK;
}

mm_status mm_batch_evict(mm_batch* b, int32_t sim) {
  if (!b) return MM_EINVAL;
  if (sim < 0 || sim >= b->max_sims || !b->sims[sim].used) return b->fail(MM_EINVAL, "no such simulation");
  Sim& s = b->sims[sim];
  give_range(b, s.base, s.n);
  b->cells -= s.n;
  s = Sim();
  b->layout_dirty = true;
  return MM_OK;
}

mm_status mm_batch_usage(const mm_batch* b, int64_t* cells, int64_t* cell_capacity, int32_t* sims) {
  if (!b) return MM_EINVAL;
  if (cells) *cells = b->cells;
  if (cell_capacity) *cell_capacity = b->E.ncap;
  if (sims) {
    int k = 0;
    for (const Sim& s : b->sims) k += s.used ? 1 : 0;
    *sims = k;
  }
  return MM_OK;
}

mm_status mm_serve(mm_batch* b, const mm_request* req, int32_t n_req, mm_request_result* res,
                   mm_serve_stats* stats) {
  if (!b) return MM_EINVAL;
  if (n_req < 0 || (n_req > 0 && (!req || !res)) || !stats) return b->fail(MM_EINVAL, "bad request arrays");
  for (int k = 0; k < b->max_sims; ++k)
    if (b->sims[k].used) return b->fail(MM_ESTATE, "mm_serve needs an empty batch");
  for (int32_t k = 1; k < n_req; ++k)
    if (req[k].arrival < req[k - 1].arrival) return b->fail(MM_EINVAL, "arrival times must not decrease");
  std::memset(stats, 0, sizeof *stats);
  for (int32_t k = 0; k < n_req; ++k) {
    res[k] = mm_request_result{};
    res[k].status = MM_ESTATE;
  }
  std::vector<int32_t> req_of(b->max_sims, -1);   // request held by each simulation id
  std::vector<double> step_ms;                    // one entry per simulation step
  std::vector<double> turnaround;
  int32_t next = 0, done = 0, resident = 0;
  std::vector<mm_sim_info> info(b->max_sims);
  const auto t0 = std::chrono::steady_clock::now();
  double last_finish = 0.0;

  auto finish = [&](int32_t sim, int status) {
    const int32_t r = req_of[sim];
    const Sim& s = b->sims[sim];
    if (status == MM_OK && !s.fresh && (req[r].pos_out || req[r].Q_out))
      status = mm_batch_read(b, sim, req[r].pos_out, req[r].Q_out, nullptr);
    res[r].status = status;
    res[r].steps = (int32_t)s.steps;
    res[r].t = s.t;
    res[r].finished = now_s(t0);
    last_finish = res[r].finished;
    turnaround.push_back(res[r].finished - req[r].arrival);
    mm_batch_evict(b, sim);
    req_of[sim] = -1;
    --resident;
    ++done;
  };

  while (done < n_req) {
    // Admission: arrived requests in order, while they fit.
    while (next < n_req && req[next].arrival <= now_s(t0)) {
      const mm_request& q = req[next];
      int32_t sim = -1;
      const mm_status r = mm_batch_admit(b, &q.params, q.n, q.pos, q.prim, q.dt_max, &sim);
      if (r == MM_EFULL && resident > 0) break;   // wait for room
      if (r != MM_OK) {
        // Cannot run even in an empty batch, or invalid.
        res[next].status = r == MM_EFULL ? MM_ECAPACITY : r;
        res[next].admitted = res[next].finished = now_s(t0);
        turnaround.push_back(res[next].finished - q.arrival);
        ++done;
        ++next;
        continue;
      }
      res[next].admitted = now_s(t0);
      req_of[sim] = next;
      ++resident;
      ++next;
      stats->max_resident = std::max(stats->max_resident, resident);
      if (q.steps <= 0) finish(sim, MM_OK);
    }
    if (resident == 0) {
      if (next < n_req) {
        const double wait = req[next].arrival - now_s(t0);
        if (wait > 0) std::this_thread::sleep_for(std::chrono::duration<double>(wait));
      }
      continue;
    }
    const auto ts = std::chrono::steady_clock::now();
    int32_t n_info = 0;
    const mm_status r = mm_batch_step(b, info.data(), (int32_t)info.size(), &n_info);
    const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - ts).count();
    if (r != MM_OK && r != MM_ECAPACITY) return r;
    ++stats->batch_steps;
    for (int32_t k = 0; k < n_info; ++k) {
      const mm_sim_info& I = info[k];
      const int32_t rq = req_of[I.sim];
      if (I.status == MM_OK) {
        step_ms.push_back(ms);
        stats->sim_steps += 1;
        stats->cell_updates += I.n;
        if (I.steps >= req[rq].steps) finish(I.sim, MM_OK);
      } else {
        finish(I.sim, I.status);
      }
    }
  }
  stats->wall = last_finish;
  stats->cell_updates_per_s = stats->wall > 0 ? (double)stats->cell_updates / stats->wall : 0.0;
  stats->step_p50 = quantile(step_ms, 0.5);
  stats->step_p99 = quantile(step_ms, 0.99);
  double sum = 0.0;
  for (double v : step_ms) sum += v;
  stats->step_mean = step_ms.empty() ? 0.0 : sum / (double)step_ms.size();
  stats->turnaround_p50 = quantile(turnaround, 0.5);
  stats->turnaround_p99 = quantile(turnaround, 0.99);
  return MM_OK;
}

}  // extern "C"
