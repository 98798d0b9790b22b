// libmdeos serving: continuous batching of EOS queries at chunk granularity.
//
// The continuum side calls the material model at every quadrature point on
// every time step (Sec. III); here each call is a query (cell, rho, e). A
// scheduler thread admits queries into resident slots as capacity allows,
// advances every admitted cell by one chunk of MD steps per round in one
// persistent launch per size bucket (a replayed HIP graph), and retires cells
// whose schedule finished. A cell keeps its particle state resident between
// queries: the next query of the same cell warm-starts from it (dilation to
// the new density and an energy re-pin) instead of lifting from the lattice.
// Queries of one cell run in arrival order; resident state is evicted
// least-recently-used when the HBM budget would be exceeded.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <sstream>

#include "mdeos.h"
#include "mdeos_host.h"

using namespace mdeos;

static double mono_now() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

// ---------------------------------------------------------------------------
// tune cache: one JSON object {"key": [block, apt, ext, list_lds], ...}

void Ctx::load_tune_cache() {
  if (tune_cache.empty()) return;
  std::ifstream f(tune_cache);
  if (!f) return;
  std::stringstream ss;
  ss << f.rdbuf();
  std::string s = ss.str();
  size_t i = 0;
  while ((i = s.find('"', i)) != std::string::npos) {
    size_t j = s.find('"', i + 1);
    if (j == std::string::npos) break;
    std::string key = s.substr(i + 1, j - i - 1);
    size_t lb = s.find('[', j), rb = s.find(']', j);
    if (lb == std::string::npos || rb == std::string::npos) break;
    Variant v{};
    const int nf = sscanf(s.c_str() + lb + 1, "%d , %d , %d , %d , %d , %d , %d , %d", &v.block, &v.apt, &v.ext,
                          &v.list_lds, &v.wpe, &v.mi, &v.nvt, &v.eam);
    if (nf >= 6 && variant_available(v))
      tuned[key] = v;
    i = rb + 1;
  }
}

void Ctx::save_tune_cache() {
  if (tune_cache.empty()) return;
  std::string tmp = tune_cache + ".tmp";
  {
    std::ofstream f(tmp);
    if (!f) return;
    f << "{\n";
    size_t k = 0;
    for (auto& kv : tuned) {
      f << "  \"" << kv.first << "\": [" << kv.second.block << ", " << kv.second.apt << ", " << kv.second.ext << ", "
        << kv.second.list_lds << ", " << kv.second.wpe << ", " << kv.second.mi << ", " << kv.second.nvt << ", "
        << kv.second.eam << "]"
        << (++k < tuned.size() ? "," : "") << "\n";
    }
    f << "}\n";
  }
  std::rename(tmp.c_str(), tune_cache.c_str());
}

// ---------------------------------------------------------------------------
// serving

static Ctx* C_(mdeos_ctx* c) { return reinterpret_cast<Ctx*>(c); }

static bool sched_has0(const mdeos_schedule& q) {
  for (int i = 0; i < q.n_rescale; ++i)
    if (q.rescale_steps[i] == 0) return true;
  return false;
}

extern "C" mdeos_status mdeos_serve_start(mdeos_ctx* ctx, const mdeos_serve_config* cfg) {
  Ctx* c = C_(ctx);
  if (!c || !cfg) return MDEOS_INVALID_ARG;
  if (cfg->chunk_steps < 1 || !(cfg->rc > 0.f) || !(cfg->dt > 0.f)) return MDEOS_INVALID_ARG;
  mdeos_cell_spec probe{0.8, 1.0, 4, cfg->rc, cfg->dt, cfg->seed, 0};
  if (mdeos_validate(&probe, &cfg->cold) != MDEOS_OK || mdeos_validate(&probe, &cfg->warm) != MDEOS_OK)
    return MDEOS_INVALID_ARG;
  if (!sched_has0(cfg->warm)) return MDEOS_INVALID_ARG;
  // the context lock first, as the scheduler thread takes them
  std::lock_guard<std::recursive_mutex> g(c->mu);
  std::lock_guard<std::mutex> lk(c->serve_mu);
  if (c->serving) return MDEOS_INVALID_ARG;
  // the resident cells of an earlier session stay until now (a stop keeps
  // them); this session starts with none, so they are released here
  std::vector<int> idx;
  for (auto& kv : c->serve_cells)
    if (kv.second.slot >= 0) idx.push_back(kv.second.slot);
  c->free_cells(idx);
  c->serve_cfg = *cfg;
  c->serve_stop_flag = false;
  c->serve_drain = true;
  c->serve_queue.clear();
  c->serve_done.clear();
  c->serve_cells.clear();
  memset(&c->serve_stats, 0, sizeof(c->serve_stats));
  c->serve_t0 = mono_now();
  c->serving = true;
  c->serve_thread = std::thread([c] { c->serve_loop(); });
  return MDEOS_OK;
}

extern "C" double mdeos_serve_now(mdeos_ctx* ctx) {
  Ctx* c = C_(ctx);
  return c ? mono_now() - c->serve_t0 : 0.0;
}

extern "C" mdeos_status mdeos_serve_submit(mdeos_ctx* ctx, long long cell_id, double rho, double e, int n_c,
                                           double t_arrival, long long* ticket) {
  Ctx* c = C_(ctx);
  if (!c) return MDEOS_INVALID_ARG;
  mdeos_cell_spec sp{rho, e, n_c, c->serve_cfg.rc, c->serve_cfg.dt, c->serve_cfg.seed, cell_id};
  if (mdeos_validate(&sp, nullptr) != MDEOS_OK) return MDEOS_INVALID_ARG;
  CellPlan p;
  if (plan_cell(sp, c->cell_skin(sp), p) != MDEOS_OK) return MDEOS_INVALID_ARG;
  std::lock_guard<std::mutex> lk(c->serve_mu);
  if (!c->serving || c->serve_stop_flag) return MDEOS_NOT_READY;
  ServeQuery q{c->next_ticket++, cell_id, rho, e, n_c, t_arrival};
  c->serve_queue.push_back(q);
  c->serve_stats.submitted += 1;
  if (ticket) *ticket = q.ticket;
  c->serve_cv.notify_one();
  return MDEOS_OK;
}

extern "C" mdeos_status mdeos_serve_poll(mdeos_ctx* ctx, int max, long long* tickets, mdeos_result* out,
                                         double* t_done, int* n_out) {
  Ctx* c = C_(ctx);
  if (!c || max < 0 || !n_out) return MDEOS_INVALID_ARG;
  std::lock_guard<std::mutex> lk(c->serve_mu);
  int k = 0;
  while (k < max && !c->serve_done.empty()) {
    ServeDone& d = c->serve_done.front();
    if (tickets) tickets[k] = d.ticket;
    if (out) out[k] = d.res;
    if (t_done) t_done[k] = d.t_done;
    c->serve_done.pop_front();
    ++k;
  }
  *n_out = k;
  return MDEOS_OK;
}

extern "C" mdeos_status mdeos_serve_stats_get(mdeos_ctx* ctx, mdeos_serve_stats* out) {
  Ctx* c = C_(ctx);
  if (!c || !out) return MDEOS_INVALID_ARG;
  std::lock_guard<std::mutex> lk(c->serve_mu);
  *out = c->serve_stats;
  return MDEOS_OK;
}

extern "C" mdeos_status mdeos_serve_stop(mdeos_ctx* ctx, int drain) {
  Ctx* c = C_(ctx);
  if (!c) return MDEOS_INVALID_ARG;
  {
    std::lock_guard<std::mutex> lk(c->serve_mu);
    if (!c->serving) return MDEOS_OK;
    c->serve_stop_flag = true;
    c->serve_drain = drain != 0;
    c->serve_cv.notify_all();
  }
  if (c->serve_thread.joinable()) c->serve_thread.join();
  std::lock_guard<std::mutex> lk(c->serve_mu);
  c->serving = false;
  return MDEOS_OK;
}

void Ctx::serve_shutdown() {
  mdeos_serve_stop(reinterpret_cast<mdeos_ctx*>(this), 0);
  // free resident serving cells
  std::vector<int> idx;
  for (auto& kv : serve_cells)
    if (kv.second.slot >= 0) idx.push_back(kv.second.slot);
  std::lock_guard<std::recursive_mutex> g(mu);
  free_cells(idx);
  serve_cells.clear();
}

namespace {
struct Active {
  int slot;
  long long cell_id;
  long long ticket;
  int n_steps;
  int step;
  bool cold;
};
}  // namespace

void Ctx::serve_loop() {
  (void)hipSetDevice(device);
  const mdeos_serve_config cfg = serve_cfg;
  const hipStream_t s = own_stream;
  std::deque<ServeQuery> waiting;  // arrival order
  std::vector<Active> active;
  std::vector<Active> pending;     // admitted while a chunk ran; in the next one
  long long round = 0;
  size_t resident_bytes = 0;
  long long resident = 0;

  auto finish_all = [&](bool drop) {
    if (drop) waiting.clear();
  };

  for (;;) {
    bool stop = false, drain = true;
    {
      std::unique_lock<std::mutex> lk(serve_mu);
      if (active.empty() && pending.empty() && waiting.empty() && serve_queue.empty() && !serve_stop_flag)
        serve_cv.wait_for(lk, std::chrono::milliseconds(2));
      while (!serve_queue.empty()) {
        waiting.push_back(serve_queue.front());
        serve_queue.pop_front();
      }
      stop = serve_stop_flag;
      drain = serve_drain;
      serve_stats.queued = (long long)waiting.size();
    }
    if (stop && !drain) finish_all(true);
    if (stop && waiting.empty() && active.empty() && pending.empty()) break;
    if (stop && !drain && active.empty() && pending.empty()) break;

    std::lock_guard<std::recursive_mutex> g(mu);
    ++round;
    // Admits waiting queries into `into`, in arrival order, as slots and
    // memory allow (a query whose plan fails is answered at once).
    auto admit = [&](std::vector<Active>& into) {
      const size_t max_active = cfg.max_slots > 0 ? (size_t)cfg.max_slots : (size_t)1 << 30;
      for (auto it = waiting.begin(); it != waiting.end() && active.size() + into.size() < max_active;) {
        ServeCell& sc = serve_cells[it->cell_id];
        if (sc.busy) {
          ++it;
          continue;
        }
        const ServeQuery q = *it;
        mdeos_cell_spec sp{q.rho, q.e, q.n_c, cfg.rc, cfg.dt, cfg.seed, q.cell_id};
        CellPlan p;
        const mdeos_status pst = plan_cell(sp, cell_skin(sp), p);
        p.nvt = cfg.warm.ensemble == MDEOS_NVT_LANGEVIN ? 1 : 0;  // used by warm starts (cold ones re-plan)
        if (pst != MDEOS_OK) {
          ServeDone d{q.ticket, {}, mono_now() - serve_t0};
          d.res.status = MDEOS_CELL_OVERFLOW;
          d.res.P = d.res.T = NAN;
          std::lock_guard<std::mutex> lk(serve_mu);
          serve_done.push_back(d);
          serve_stats.completed += 1;
          it = waiting.erase(it);
          continue;
        }
        bool warm = sc.slot >= 0 && h_cells[sc.slot].n_c == q.n_c;
        if (sc.slot >= 0 && !warm) {
          resident_bytes -= mdeos_cell_bytes(h_cells[sc.slot].n_c);
          resident -= 1;
          free_cells({sc.slot});
          sc.slot = -1;
        }
        if (!warm) {
          const size_t need = mdeos_cell_bytes(q.n_c);
          // evict idle resident cells, least recently used first
          while (resident_bytes + need > hbm_budget) {
            long long victim = -1, oldest = 1LL << 62;
            for (auto& kv : serve_cells)
              if (kv.second.slot >= 0 && !kv.second.busy && kv.first != q.cell_id && kv.second.last_use < oldest) {
                oldest = kv.second.last_use;
                victim = kv.first;
              }
            if (victim < 0) break;
            ServeCell& vc = serve_cells[victim];
            resident_bytes -= mdeos_cell_bytes(h_cells[vc.slot].n_c);
            resident -= 1;
            free_cells({vc.slot});
            vc.slot = -1;
            std::lock_guard<std::mutex> lk(serve_mu);
            serve_stats.evictions += 1;
          }
          if (resident_bytes + need > hbm_budget) break;  // wait for capacity
          std::vector<int> idx;
          if (alloc_cells(1, &sp, cfg.cold, idx) != MDEOS_OK) break;
          sc.slot = idx[0];
          resident_bytes += need;
          resident += 1;
        } else {
          CellRec& r = h_cells[sc.slot];
          const double Lold = r.Lw;
          const int off = r.atom_off, query = r.query;
          fill_record(r, sp, cfg.warm, p, off);
          r.warm_scale = p.Lw / Lold;
          r.query = query + 1;
          r.phase = PH_WARM;
          cell_plan[sc.slot] = p;
        }
        sc.busy = true;
        sc.last_use = round;
        const mdeos_schedule& qs = warm ? cfg.warm : cfg.cold;
        into.push_back(Active{sc.slot, q.cell_id, q.ticket, qs.n_steps, 0, !warm});
        {
          std::lock_guard<std::mutex> lk(serve_mu);
          if (warm) serve_stats.warm += 1;
          else serve_stats.cold += 1;
        }
        it = waiting.erase(it);
      }
    };
    // ---- admission: the queries admitted while the last chunk ran, then the
    // ones that arrived since; their records go up before the launch
    std::vector<Active> fresh;
    fresh.swap(pending);
    admit(fresh);
    std::vector<int> upload;
    for (const Active& a : fresh) upload.push_back(a.slot);
    if (!upload.empty() && upload_records(upload, s) != MDEOS_OK) {
      fprintf(stderr, "mdeos serve: record upload failed: %s\n", mdeos_last_error());
      break;
    }
    active.insert(active.end(), fresh.begin(), fresh.end());
    if (active.empty()) continue;

    // ---- one chunk for every admitted cell ------------------------------
    std::vector<int> slots_now;
    slots_now.reserve(active.size());
    for (const Active& a : active) slots_now.push_back(a.slot);
    std::vector<Bucket> b;
    make_buckets(slots_now, b, cfg.chunk_steps, true);
    if (run_buckets(b, cfg.chunk_steps, s, true) != MDEOS_OK) {
      fprintf(stderr, "mdeos serve: launch failed: %s\n", mdeos_last_error());
      break;
    }
    // while the chunk runs: take the queries that arrived meanwhile and plan
    // their admission (host work that would otherwise leave the device idle
    // between chunks); they join the next chunk
    {
      std::lock_guard<std::mutex> lk(serve_mu);
      while (!serve_queue.empty()) {
        waiting.push_back(serve_queue.front());
        serve_queue.pop_front();
      }
      serve_stats.queued = (long long)waiting.size();
    }
    admit(pending);
    double atom_steps = 0.0;
    std::vector<int> finished;
    std::vector<size_t> fin_pos;
    for (size_t i = 0; i < active.size(); ++i) {
      Active& a = active[i];
      const int adv = std::min(cfg.chunk_steps, a.n_steps - a.step);
      a.step += adv;
      atom_steps += (double)adv * h_cells[a.slot].N;
      if (a.step >= a.n_steps) {
        finished.push_back(a.slot);
        fin_pos.push_back(i);
      }
    }
    std::vector<mdeos_result> res(finished.size());
    if (!finished.empty()) {
      if (restrict_cells(finished, res.data(), s) != MDEOS_OK) {
        fprintf(stderr, "mdeos serve: restrict failed: %s\n", mdeos_last_error());
        break;
      }
    } else if (hipStreamSynchronize(s) != hipSuccess) {
      break;
    }
    const double t_done = mono_now() - serve_t0;
    {
      std::lock_guard<std::mutex> lk(serve_mu);
      serve_stats.chunks += 1;
      serve_stats.atom_steps += atom_steps;
      for (size_t k = 0; k < finished.size(); ++k) {
        const Active& a = active[fin_pos[k]];
        ServeDone d{a.ticket, res[k], t_done};
        if (res[k].status & MDEOS_CELL_COLD_RELIFT) serve_stats.relifts += 1;
        serve_done.push_back(d);
        serve_stats.completed += 1;
        serve_cells[a.cell_id].busy = false;
      }
    }
    // drop finished entries (positions ascending) in one pass, keeping the order
    {
      size_t w = 0, f = 0;
      for (size_t i = 0; i < active.size(); ++i) {
        if (f < fin_pos.size() && fin_pos[f] == i) {
          ++f;
          continue;
        }
        active[w++] = active[i];
      }
      active.resize(w);
    }
    {
      std::lock_guard<std::mutex> lk(serve_mu);
      serve_stats.active = (long long)active.size();
      serve_stats.resident = resident;
      serve_stats.resident_bytes = resident_bytes;
    }
  }
  std::lock_guard<std::mutex> lk(serve_mu);
  serve_stats.active = 0;
}
