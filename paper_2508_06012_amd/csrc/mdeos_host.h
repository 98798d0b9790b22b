// Host-side internals of libmdeos: the context, the device arena allocator,
// per-cell plans, launch buckets and the serving state.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "mdeos.h"
#include "mdeos_dev.h"

namespace mdeos {

constexpr int kLdsMax = 160 * 1024;
constexpr int kAux = 4;
constexpr int kMaxBuckets = 64;

double box_length(int n_c, double rho);
int ring_for(int gmax);
void set_last_error(const char* msg);   // message of mdeos_last_error (this thread)
hipError_t noalloc_init(int device);    // the no-alloc workspace's address on `device` (current)

struct CellPlan {
  int N = 0;
  double Lw = 0.0;
  float L = 0.f, rl = 0.f;
  int stencil = 1, nce = 0, ncell = 0;
  int ext_need = 0, ext = 0;
  int list_cap = 0;
  int list_in_lds = 0;
  int lds_bytes = 0;
  int multi_image = 0;
  int minimg = 0;  // 1: minimum-image variant (no ghosts)
  int nvt = 0;     // 1: Langevin integration (set from the schedule, not by plan_cell)
};

mdeos_status plan_cell(const mdeos_cell_spec& s, float skin, CellPlan& out);
mdeos_status finish_plan(CellPlan& out);

// First-fit allocator of integer ranges with coalescing.
class RangeAlloc {
 public:
  int alloc(int n);
  void release(int off, int n);
  void grow(int old_cap, int new_cap);
  bool has_room(int n) const {
    for (auto& kv : free_)
      if (kv.second >= n) return true;
    return false;
  }
  long long used() const { return used_; }

 private:
  void release_raw(int off, int n);
  std::map<int, int> free_;
  long long used_ = 0;
};

struct Bucket {
  Variant v{};
  Caps caps{0, 0, 0, 0, 0};
  int lds = 0;
  int grid = 1;
  int work_off = 0;
  size_t gl_off = 0;
  std::vector<int> cells;
  CellPlan plan{};  // merged capacities of the cells (what the launch shape must fit)
};

struct GraphEntry {
  hipGraphExec_t exec = nullptr;
};

// Kernel helpers implemented in kernels.hip.
hipError_t init_kernel_attributes();
int occupancy(const Variant& v, int lds_bytes);

struct ServeQuery {
  long long ticket;
  long long cell_id;
  double rho, e;
  int n_c;
  double t_arrival;
};

struct ServeDone {
  long long ticket;
  mdeos_result res;
  double t_done;
};

struct ServeCell {
  int slot = -1;           // resident slot, -1 if none
  bool busy = false;       // a query of this cell is advancing
  long long last_use = 0;  // scheduling round of the last query
  std::deque<ServeQuery> pending;
};

struct Ctx {
  int device = 0;
  int n_cu = 256;
  float skin = 0.f;  // Verlet skin set by the caller, or 0: the default of cell_skin
  size_t hbm_budget = 0;
  int autotune = 0;
  int tune_runs = 0;  // buckets timed by the autotuner so far
  int precision = MDEOS_PREC_FP64;
  int potential = MDEOS_POT_LJTS;  // material of every cell of the context
  double eam_c = 39.432;           // embedding strength of MDEOS_POT_EAM
  float prune_skin = 0.f;          // inner-list skin (0: no inner lists)
  // Inner lists are kept for the device-memory lists of the embedded-atom
  // shapes only; the compensated FP32 sums would fold their zero terms
  // differently, so that mode keeps none.
  // Verlet skin of a cell: the caller's, else the measured best of the
  // potential. For LJTS, 0 (plan_cell's per-size default). For the
  // embedded-atom form: 0.5 a up to 1000 atoms, and 0.3 a above, where the
  // ghost-extended boxes at 0.5 outgrow their launch shapes.
  float cell_skin(const mdeos_cell_spec& s) const {
    if (skin > 0.f) return skin;
    if (potential != MDEOS_POT_EAM) return 0.f;
    return 4L * s.n_c * s.n_c * s.n_c <= 1000 ? 0.5f : 0.3f;
  }
  bool prune_lists() const {
    return prune_skin > 0.f && precision != MDEOS_PREC_KAHAN && potential == MDEOS_POT_EAM;
  }
  std::string arch = "gfx950";  // device architecture (tune-cache key)
  std::string tune_cache;
  std::recursive_mutex mu;

  hipStream_t own_stream = nullptr;
  hipStream_t aux[kAux] = {};
  hipEvent_t ev_fork = nullptr, ev_join[kAux] = {}, ev_t0 = nullptr, ev_t1 = nullptr;

  // atom arena: 6 FP64 arrays (x, v) and 6 FP32 arrays (F, build positions)
  std::vector<void*> arena_ptrs;
  AtomArena arena{};
  int atom_cap = 0;
  RangeAlloc atoms;

  // cells
  CellRec* d_cells = nullptr;
  int cell_cap = 0;
  RangeAlloc slots;
  std::vector<CellRec> h_cells;
  std::vector<unsigned> gen;
  std::vector<char> live;
  std::unordered_map<int, CellPlan> cell_plan;

  // launch scratch
  int* d_work = nullptr;
  size_t work_cap = 0;
  int* d_counters = nullptr;
  size_t counters_cap = 0;
  uint16_t* d_gl = nullptr;
  size_t gl_cap = 0, gl_cap_elems = 0;
  DevResult* d_results = nullptr;
  size_t res_cap = 0;
  int* d_idx = nullptr;
  size_t idx_cap = 0;
  DevResult* h_results = nullptr;
  size_t h_results_cap = 0;
  unsigned char* h_stage = nullptr;
  size_t stage_cap = 0;

  std::map<std::string, GraphEntry> graphs;
  std::map<std::string, Variant> tuned;
  Variant forced_variant{0, 0, 0, 0, 0, 0};  // MDEOS_FORCE_VARIANT="block,apt,ext,lds,wpe,mi" (tuning)
  bool tune_log = false;  // MDEOS_TUNE_LOG=1: the autotuner prints each candidate's timings to stderr
  // MDEOS_SHRINK_CAPS=1: eval_batch / eval_plain plan every cell with an
  // 8-entry neighbour list, so the first list build overflows and their
  // capacity retry runs (a test hook: capacities never change a cell's
  // arithmetic, so the retried results equal an unforced run bit for bit)
  bool shrink_caps = false;

  // serving
  std::thread serve_thread;
  std::mutex serve_mu;
  std::condition_variable serve_cv;
  bool serving = false, serve_stop_flag = false, serve_drain = true;
  mdeos_serve_config serve_cfg{};
  std::deque<ServeQuery> serve_queue;
  std::deque<ServeDone> serve_done;
  std::unordered_map<long long, ServeCell> serve_cells;
  mdeos_serve_stats serve_stats{};
  long long next_ticket = 1;
  double serve_t0 = 0.0;

  ~Ctx();
  mdeos_status init(const mdeos_config* cfg);
  hipStream_t pick(void* stream) const;

  mdeos_status ensure_atoms(int need);
  mdeos_status ensure_cells(int need);
  mdeos_status ensure_scratch(size_t work_n, size_t counters_n, size_t gl_bytes, size_t res_n);
  mdeos_status ensure_stage(size_t bytes);
  void graphs_clear();

  void fill_record(CellRec& r, const mdeos_cell_spec& s, const mdeos_schedule& q, const CellPlan& p, int atom_off);
  mdeos_handle handle_of(int slot) const;
  int slot_of(mdeos_handle h) const;
  mdeos_status alloc_cells(int n, const mdeos_cell_spec* specs, const mdeos_schedule& q, std::vector<int>& out);
  void free_cells(const std::vector<int>& idx);
  mdeos_status upload_records(const std::vector<int>& idx, hipStream_t s);
  mdeos_status upload_state(int slot, const double* xyz, const double* v, hipStream_t s);
  mdeos_status download_atoms(int slot, int which_mask, std::vector<double>& out, hipStream_t s);
  mdeos_status download_record(int slot, CellRec& out, hipStream_t s);

  bool choose_variant(const CellPlan& p, Variant& out) const;
  int rank_variants(const CellPlan& p, std::vector<Variant>& out) const;
  mdeos_status autotune_buckets(std::vector<Bucket>& buckets, hipStream_t s);
  std::string tune_key(const CellPlan& p) const;
  void make_buckets(const std::vector<int>& cells, std::vector<Bucket>& out, int step_budget, bool sticky = false);
  std::map<std::pair<int, int>, CellPlan> sticky_plans;  // serving: bucket capacities only grow
  int timed_launches = 0;
  mdeos_status run_buckets(std::vector<Bucket>& buckets, int step_budget, hipStream_t s, bool use_graph);
  mdeos_status restrict_cells(const std::vector<int>& idx, mdeos_result* out, hipStream_t s);
  AdvanceParams make_params(const Bucket& b, int bi, int step_budget);
  mdeos_status fetch_results(int n, mdeos_result* out, hipStream_t s);
  mdeos_status eval(int n, const mdeos_cell_spec* specs, const mdeos_schedule* sched, mdeos_result* out,
                    hipStream_t s, bool plain);
  mdeos_status eval_noalloc(int n, const mdeos_cell_spec* specs, const mdeos_schedule* sched, mdeos_result* out,
                            hipStream_t s);

  // autotuner
  void load_tune_cache();
  void save_tune_cache();

  // serving
  void serve_loop();
  void serve_shutdown();
};

}  // namespace mdeos
