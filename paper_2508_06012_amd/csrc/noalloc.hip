// mdeos_eval_batch_noalloc: the whole-evaluation entry point (lift, schedule,
// restrict) for callers that cannot allocate memory. Every device buffer the
// kernels use beyond the caller's inputs and outputs (cell records, the atom
// state arena, work lists, counters, device-memory neighbour lists, results)
// lives in one file-scope device array, `scratch`, of kScratchBytes per GPU;
// host staging uses file-scope host arrays. The call allocates nothing: no
// hipMalloc / hipHostMalloc / hipFree, no graphs, no C++ heap.
//
// The array's name is a host-side stand-in, not a device address: its address
// on each device is taken once with hipGetSymbolAddress when a context is
// created on that device (with the device current), and only that pointer is
// handed to kernels and copies.
#include <algorithm>
#include <cstring>
#include <mutex>

#include "mdeos.h"
#include "mdeos_dev.h"
#include "mdeos_host.h"

#define NCHECK(expr)                      \
  do {                                    \
    const hipError_t e_ = (expr);         \
    if (e_ != hipSuccess) {               \
      set_last_error(hipGetErrorString(e_)); \
      return MDEOS_DEVICE_ERROR;          \
    }                                     \
  } while (0)

namespace mdeos {

namespace {

constexpr size_t kScratchBytes = (size_t)MDEOS_NOALLOC_SCRATCH_MIB << 20;
constexpr int kMaxDevices = 64;
constexpr int kMaxGroups = 16;  // launches: one per (atom count, image mode) group

__device__ __align__(256) unsigned char scratch[kScratchBytes];

unsigned char* g_scratch_ptr[kMaxDevices] = {};
std::mutex g_mu;  // the set-up of the pointers and every call (host staging is shared)

// host staging (file scope: nothing is allocated per call)
CellRec h_rec[MDEOS_NOALLOC_MAX_CELLS];
DevResult h_res[MDEOS_NOALLOC_MAX_CELLS];
int h_work[2 * kMaxGroups + 2 * MDEOS_NOALLOC_MAX_CELLS];

struct Group {
  int N, minimg, count, off;
  CellPlan plan;  // merged: capacities are maxima over the group's cells
  Variant v;
  Caps caps;
  int lds, grid;
  size_t gl_off, gl_bytes;
};
Group g_groups[kMaxGroups];
int g_cell_group[MDEOS_NOALLOC_MAX_CELLS];
CellPlan g_plans[MDEOS_NOALLOC_MAX_CELLS];

size_t align256(size_t v) { return (v + 255) / 256 * 256; }

// The best launch shape for a merged plan by the library's static model (the
// first of rank_variants' order), without building the ranked list.
bool best_variant(const Ctx& c, const CellPlan& p, const Caps& caps, Variant& out) {
  bool found = false;
  long best = 0;
  for (int i = 0; i < variant_count(); ++i) {
    const Variant v = variant_at(i);
    const int lds = lds_layout(v.ext, caps, v.list_lds, frc_slots(v)).total;
    if (v.mi != p.minimg || v.nvt != p.nvt || v.eam != (c.potential == MDEOS_POT_EAM ? 1 : 0) ||
        v.block * v.apt < p.N || v.ext - 1 < p.ext_need || lds > kLdsMax)
      continue;
    const int wg_by_lds = kLdsMax / lds, wg_by_regs = std::max(1, 4 * v.wpe / (v.block / 64));
    const int waves = std::min(wg_by_lds, wg_by_regs) * (v.block / 64);
    const int idle = v.block * v.apt - p.N;
    const long score = -(long)waves * 4096 + (idle * 4 + (v.block == 512 ? 0 : 1)) * 16 + (v.list_lds ? 0 : 8) +
                       (v.ext - p.ext_need) / 1024;
    if (!found || score < best) {
      found = true;
      best = score;
      out = v;
    }
  }
  return found;
}

}  // namespace

// Called from context creation with `device` current.
hipError_t noalloc_init(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_scratch_ptr[device]) return hipSuccess;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_scratch_ptr[device] = (unsigned char*)p;
  return hipSuccess;
}

mdeos_status Ctx::eval_noalloc(int n, const mdeos_cell_spec* specs, const mdeos_schedule* sched, mdeos_result* out,
                               hipStream_t s) {
  if (n > MDEOS_NOALLOC_MAX_CELLS) {
    set_last_error("mdeos_eval_batch_noalloc: more than MDEOS_NOALLOC_MAX_CELLS cells");
    return MDEOS_INVALID_ARG;
  }
  for (int i = 0; i < n; ++i) {
    const mdeos_status st = mdeos_validate(&specs[i], sched);
    if (st != MDEOS_OK) return st;
  }
  std::lock_guard<std::mutex> lk(g_mu);
  unsigned char* const base = (device >= 0 && device < kMaxDevices) ? g_scratch_ptr[device] : nullptr;
  if (!base) {
    set_last_error("mdeos_eval_batch_noalloc: workspace of this device not set up");
    return MDEOS_DEVICE_ERROR;
  }
  // plans and groups
  int ng = 0;
  long long total_atoms = 0;
  for (int i = 0; i < n; ++i) {
    CellPlan& p = g_plans[i];
    if (plan_cell(specs[i], cell_skin(specs[i]), p) != MDEOS_OK) {
      set_last_error("mdeos_eval_batch_noalloc: box too large for an LDS-resident extended box");
      return MDEOS_INVALID_ARG;
    }
    p.nvt = sched->ensemble == MDEOS_NVT_LANGEVIN ? 1 : 0;
    total_atoms += p.N;
    int g = 0;
    while (g < ng && !(g_groups[g].N == p.N && g_groups[g].minimg == p.minimg)) ++g;
    if (g == ng) {
      if (ng == kMaxGroups) {
        set_last_error("mdeos_eval_batch_noalloc: more than 16 (atom count, image mode) groups");
        return MDEOS_INVALID_ARG;
      }
      g_groups[g].N = p.N;
      g_groups[g].minimg = p.minimg;
      g_groups[g].count = 0;
      g_groups[g].plan = p;
      ++ng;
    }
    Group& G = g_groups[g];
    G.plan.ext_need = std::max(G.plan.ext_need, p.ext_need);
    G.plan.list_cap = std::max(G.plan.list_cap, p.list_cap);
    G.plan.ncell = std::max(G.plan.ncell, p.ncell);
    G.plan.rl = std::max(G.plan.rl, p.rl);
    g_cell_group[i] = g;
    G.count += 1;
  }
  // launch shapes and work lists: {count, offset} per group, then the cell
  // indices of each group, then 0..n-1 for the restriction
  int off = 2 * ng;
  for (int g = 0; g < ng; ++g) {
    Group& G = g_groups[g];
    G.caps.n_pad = align_up(G.plan.N, 64);
    G.caps.list_cap = G.plan.list_cap;
    G.caps.ncell_cap = G.plan.ncell;
    G.caps.gmax = G.caps.n_pad / 64;
    G.caps.ring = ring_for(G.caps.gmax);
    if (!best_variant(*this, G.plan, G.caps, G.v)) {
      set_last_error("mdeos_eval_batch_noalloc: no launch shape holds a group's merged capacities");
      return MDEOS_INVALID_ARG;
    }
    G.lds = lds_layout(G.v.ext, G.caps, G.v.list_lds, frc_slots(G.v)).total;
    G.grid = std::max(1, std::min(G.count, std::max(1, occupancy(G.v, G.lds)) * n_cu));
    G.off = off;
    h_work[2 * g] = G.count;
    h_work[2 * g + 1] = off;
    off += G.count;
  }
  {
    int fill[kMaxGroups] = {};
    for (int i = 0; i < n; ++i) {
      const int g = g_cell_group[i];
      h_work[g_groups[g].off + fill[g]++] = i;
    }
  }
  const int idx_off = off;
  for (int i = 0; i < n; ++i) h_work[idx_off + i] = i;
  const int n_work = idx_off + n;
  // workspace layout (256-byte aligned pieces)
  const bool prune = prune_lists();
  size_t o = 0;
  const size_t o_cells = o;
  o = align256(o + sizeof(CellRec) * n);
  const size_t o_res = o;
  o = align256(o + sizeof(DevResult) * n);
  const size_t o_work = o;
  o = align256(o + sizeof(int) * n_work);
  const size_t o_cnt = o;
  o = align256(o + sizeof(int) * kMaxGroups);
  const size_t o_arena = o;
  const size_t per_atom = 6 * sizeof(double) + 6 * sizeof(float);
  o = align256(o + (size_t)per_atom * (size_t)total_atoms + 12 * 256);
  size_t lists = 0;
  for (int g = 0; g < ng; ++g) {
    Group& G = g_groups[g];
    G.gl_bytes = G.v.list_lds ? 0 : (prune ? 2 : 1) * (size_t)G.caps.list_cap * G.caps.n_pad * 2;  // per workgroup
  }
  // fewer workgroups (the persistent kernel takes any grid) until the lists fit
  for (;;) {
    lists = 0;
    for (int g = 0; g < ng; ++g) lists += align256(g_groups[g].gl_bytes * g_groups[g].grid);
    if (o + lists <= kScratchBytes) break;
    int gmax = -1;
    for (int g = 0; g < ng; ++g)
      if (g_groups[g].gl_bytes > 0 && g_groups[g].grid > 1 &&
          (gmax < 0 || g_groups[g].gl_bytes * g_groups[g].grid > g_groups[gmax].gl_bytes * g_groups[gmax].grid))
        gmax = g;
    if (gmax < 0) {
      set_last_error("mdeos_eval_batch_noalloc: batch exceeds the static workspace (MDEOS_NOALLOC_SCRATCH_MIB)");
      return MDEOS_INVALID_ARG;
    }
    g_groups[gmax].grid = (g_groups[gmax].grid + 1) / 2;
  }
  {
    size_t lo = o;
    for (int g = 0; g < ng; ++g) {
      g_groups[g].gl_off = lo;
      lo += align256(g_groups[g].gl_bytes * g_groups[g].grid);
    }
  }
  // cell records (the atom state of cell i follows cell i - 1's)
  AtomArena a;
  {
    const size_t cap = (size_t)total_atoms;
    size_t q = o_arena;
    double** d6[6] = {&a.x, &a.y, &a.z, &a.vx, &a.vy, &a.vz};
    float** f6[6] = {&a.fx, &a.fy, &a.fz, &a.bx, &a.by, &a.bz};
    for (double** d : d6) {
      *d = (double*)(base + q);
      q = align256(q + sizeof(double) * cap);
    }
    for (float** f : f6) {
      *f = (float*)(base + q);
      q = align256(q + sizeof(float) * cap);
    }
  }
  int aoff = 0;
  for (int i = 0; i < n; ++i) {
    fill_record(h_rec[i], specs[i], *sched, g_plans[i], aoff);
    aoff += g_plans[i].N;
  }
  CellRec* d_rec = (CellRec*)(base + o_cells);
  DevResult* d_res = (DevResult*)(base + o_res);
  int* d_wk = (int*)(base + o_work);
  int* d_cnt = (int*)(base + o_cnt);
  NCHECK(hipMemcpyAsync(d_rec, h_rec, sizeof(CellRec) * n, hipMemcpyHostToDevice, s));
  NCHECK(hipMemcpyAsync(d_wk, h_work, sizeof(int) * n_work, hipMemcpyHostToDevice, s));
  // the work counters start at zero: a fill kernel, not a memset
  NCHECK(launch_zero_ints(d_cnt, ng, s));
  NCHECK(hipEventRecord(ev_t0, s));
  for (int g = 0; g < ng; ++g) {
    const Group& G = g_groups[g];
    AdvanceParams p;
    p.cells = d_rec;
    p.work_base = d_wk;
    p.meta = d_wk + 2 * g;
    p.counter = d_cnt + g;
    p.step_budget = 0;
    p.a = a;
    p.gl_list = G.v.list_lds ? nullptr : (uint16_t*)(base + G.gl_off);
    p.gl_ilist = (G.v.list_lds || !prune) ? nullptr : p.gl_list + (size_t)G.grid * G.caps.list_cap * G.caps.n_pad;
    p.prune_skin = prune_skin;
    p.caps = G.caps;
    p.kahan = precision == MDEOS_PREC_KAHAN ? 1 : 0;
    p.eam_c = eam_c;
    NCHECK(launch_advance(G.v, p, G.grid, G.lds, s));
  }
  NCHECK(hipEventRecord(ev_t1, s));
  timed_launches = ng;
  NCHECK(launch_restrict(d_rec, d_wk + idx_off, n, d_res, s));
  NCHECK(hipMemcpyAsync(h_res, d_res, sizeof(DevResult) * n, hipMemcpyDeviceToHost, s));
  NCHECK(hipStreamSynchronize(s));
  static_assert(sizeof(DevResult) == sizeof(mdeos_result), "result layout");
  memcpy(out, h_res, sizeof(DevResult) * n);
  return MDEOS_OK;
}

}  // namespace mdeos
