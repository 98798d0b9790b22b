// libmdeos host side: context, device arena, per-cell planning, size buckets,
// persistent launches under captured HIP graphs, and the C ABI of mdeos.h.
#include "mdeos.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "mdeos_dev.h"
#include "mdeos_host.h"

using namespace mdeos;

static thread_local std::string g_last_error;

static void set_error(const std::string& s) { g_last_error = s; }
namespace mdeos {
void set_last_error(const char* msg) { g_last_error = msg; }
}  // namespace mdeos

const char* mdeos_last_error(void) { return g_last_error.c_str(); }

#define HCHECK(expr)                                                                           \
  do {                                                                                         \
    hipError_t e_ = (expr);                                                                    \
    if (e_ != hipSuccess) {                                                                    \
      set_error(std::string(#expr) + ": " + hipGetErrorString(e_));                            \
      return MDEOS_DEVICE_ERROR;                                                               \
    }                                                                                          \
  } while (0)

// ---------------------------------------------------------------------------
// host-only calls

extern "C" const char* mdeos_strerror(mdeos_status s) {
  switch (s) {
    case MDEOS_OK: return "ok";
    case MDEOS_INVALID_ARG: return "invalid argument";
    case MDEOS_OUT_OF_MEMORY: return "out of memory (device or HBM budget)";
    case MDEOS_DEVICE_ERROR: return "device error";
    case MDEOS_NOT_READY: return "not ready";
    case MDEOS_ADMISSION_FULL: return "admission full";
    case MDEOS_NO_DEVICE: return "no HIP device";
    default: return "unknown status";
  }
}

extern "C" const char* mdeos_version(void) { return "mdeos 0.1 (gfx950)"; }

extern "C" int mdeos_device_count(void) {
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess) return 0;
  return n;
}

namespace mdeos {

double box_length(int n_c, double rho) { return n_c * std::cbrt(4.0 / rho); }

static int pick_ext(int need) {
  for (int e : {2048, 3072, 4096, 8176})
    if (need <= e - 1) return e;
  return 0;
}

// Exact number of periodic images within rl of the faces for the FCC start
// lattice: in half-lattice units the sites are (a, b, c) in [0, 2 n_c)^3 with
// a + b + c even, at coordinate l (a / 2 + 1/4).
static int lattice_ghosts(int n_c, double l, double L, double rl) {
  const int m = 2 * n_c;
  int img[2 * MDEOS_MAX_NC];  // n_c <= MDEOS_MAX_NC (validated); no allocation, the no-alloc path plans too
  for (int a = 0; a < m; ++a) {
    const double x = l * (0.5 * a + 0.25);
    img[a] = 1 + (x < rl ? 1 : 0) + (x >= L - rl ? 1 : 0);
  }
  long g = 0;
  for (int a = 0; a < m; ++a)
    for (int b = 0; b < m; ++b)
      for (int c = 0; c < m; ++c)
        if (((a + b + c) & 1) == 0) g += img[a] * img[b] * img[c] - 1;
  return (int)g;
}

// Neighbours within rl of one site of the infinite FCC lattice (all images).
static int lattice_neighbours(double l, double rl) {
  const int k = (int)std::ceil(2.0 * rl / l) + 1;
  int n = 0;
  for (int i = -k; i <= k; ++i)
    for (int j = -k; j <= k; ++j)
      for (int q = -k; q <= k; ++q) {
        if (((i + j + q) & 1) != 0 || (i == 0 && j == 0 && q == 0)) continue;
        const double r2 = 0.25 * l * l * (double)(i * i + j * j + q * q);
        if (r2 < (double)rl * rl) ++n;
      }
  return n;
}

// Plans one cell: geometry, capacities and the LDS it needs. Capacities cover
// the start lattice exactly and the liquid with a margin; a cell that still
// overflows is re-run with larger capacities by the batch paths.
//
// skin <= 0 selects the measured best LJTS skin of the box size (kernel time
// of the uneven batch's cells of each size at skins 0.3-0.8): 0.3 sigma up to
// 150 atoms, 0.4 up to 600 atoms and for rc above 3.5 sigma, 0.6 above 600
// atoms; a box whose extended box does not fit at 0.6 takes 0.4.
mdeos_status plan_cell(const mdeos_cell_spec& s, float skin, CellPlan& out) {
  if (skin <= 0.f) {
    const long n = 4L * s.n_c * s.n_c * s.n_c;
    const float d = n <= 150 ? 0.3f : ((n <= 600 || s.rc > 3.5) ? 0.4f : 0.6f);
    if (d != 0.4f && plan_cell(s, d, out) == MDEOS_OK) return MDEOS_OK;
    skin = 0.4f;
  }
  const double L = box_length(s.n_c, s.rho);
  const double l = std::cbrt(4.0 / s.rho);
  const int N = 4 * s.n_c * s.n_c * s.n_c;
  double sk = std::min<double>(skin, 0.5 * (L - s.rc));
  if (!(sk > 0.0)) return MDEOS_INVALID_ARG;
  const float rl = (float)(s.rc + sk);
  out.N = N;
  out.Lw = L;
  out.L = (float)L;
  out.rl = rl;
  const double ext_len = L + 2.0 * rl;
  // cells of edge >= rl/2 (5^3 stencil) unless that grid exceeds 1000 cells,
  // then edge >= rl (3^3 stencil): keeps the binning arrays within 8 KB of LDS
  int R = 2, nce = (int)std::floor(ext_len * 2.0 / rl);
  if ((long)nce * nce * nce > 1000) {
    R = 1;
    nce = (int)std::floor(ext_len / rl);
  }
  out.stencil = R;
  out.nce = nce;
  out.ncell = nce * nce * nce;
  const double ghosts = s.rho * (ext_len * ext_len * ext_len - L * L * L);
  const int g_lat = lattice_ghosts(s.n_c, l, L, (double)rl);
  out.ext_need = N + std::max((int)std::ceil(1.15 * ghosts + 96.0), g_lat + 32);
  const double nl = 4.0 / 3.0 * M_PI * (double)rl * rl * rl * s.rho;
  const int n_lat = lattice_neighbours(l, (double)rl);
  out.list_cap = align_up(std::max((int)std::ceil(1.25 * nl + 24.0), n_lat + 8), 8);
  out.multi_image = s.rc > 0.5 * L ? 1 : 0;
  out.minimg = 0;
  if (finish_plan(out) == MDEOS_OK) return MDEOS_OK;
  // the ghost-extended box does not fit: minimum image over the real atoms
  // (needs at least three binning cells of edge >= rl per box edge)
  CellPlan mi = out;
  mi.minimg = 1;
  mi.multi_image = 0;
  int Rm = 2, ncm = (int)std::floor(2.0 * L / rl);
  if ((long)ncm * ncm * ncm > 1000 || ncm < 5) {
    Rm = 1;
    ncm = (int)std::floor(L / rl);
  }
  if (ncm < 3) return MDEOS_INVALID_ARG;
  mi.stencil = Rm;
  mi.nce = ncm;
  mi.ncell = ncm * ncm * ncm;
  mi.ext_need = N + 1;
  out = mi;
  return finish_plan(out);
}

// Chooses the position stride and list location of a plan and its LDS bytes.
mdeos_status finish_plan(CellPlan& out) {
  out.ext = out.minimg ? (out.ext_need <= 4087 ? 4088 : 0) : pick_ext(out.ext_need);
  if (out.ext == 0 || out.ncell > 65535) return MDEOS_INVALID_ARG;
  Caps c;
  c.n_pad = align_up(out.N, 64);
  c.list_cap = out.list_cap;
  c.ncell_cap = out.ncell;
  c.gmax = c.n_pad / 64;
  c.ring = ring_for(c.gmax);
  LdsLayout with = lds_layout(out.ext, c, true), without = lds_layout(out.ext, c, false);
  out.list_in_lds = with.total <= kLdsMax ? 1 : 0;
  out.lds_bytes = out.list_in_lds ? with.total : without.total;
  if (out.lds_bytes > kLdsMax) return MDEOS_INVALID_ARG;
  return MDEOS_OK;
}

int ring_for(int gmax) { return std::max(2, std::min(16, 1536 / (24 * gmax))); }

}  // namespace mdeos

extern "C" mdeos_status mdeos_validate(const mdeos_cell_spec* s, const mdeos_schedule* q) {
  if (!s) return MDEOS_INVALID_ARG;
  if (!(std::isfinite(s->rho) && s->rho > 0.0)) return set_error("rho must be > 0"), MDEOS_INVALID_ARG;
  if (!(std::isfinite(s->e) && s->e > 0.0)) return set_error("e must be > 0"), MDEOS_INVALID_ARG;
  if (s->n_c < 1 || s->n_c > MDEOS_MAX_NC) return set_error("n_c out of range"), MDEOS_INVALID_ARG;
  if (!(std::isfinite(s->rc) && s->rc > 0.f)) return set_error("rc must be > 0"), MDEOS_INVALID_ARG;
  if (!(std::isfinite(s->dt) && s->dt > 0.f)) return set_error("dt must be > 0"), MDEOS_INVALID_ARG;
  const double L = box_length(s->n_c, s->rho);
  if (!((double)s->rc < L)) return set_error("rc must be < L"), MDEOS_INVALID_ARG;
  if (q) {
    if (q->n_steps < 1) return set_error("n_steps must be >= 1"), MDEOS_INVALID_ARG;
    if (q->n_avg < 1 || q->n_avg > q->n_steps) return set_error("n_avg out of range"), MDEOS_INVALID_ARG;
    if (q->n_blocks < 2 || q->n_blocks > MDEOS_MAX_BLOCKS || q->n_avg % q->n_blocks != 0)
      return set_error("n_blocks must be in 2..16 and divide n_avg"), MDEOS_INVALID_ARG;
    if (q->n_rescale < 0 || q->n_rescale > MDEOS_MAX_RESCALE) return set_error("n_rescale out of range"), MDEOS_INVALID_ARG;
    for (int i = 0; i < q->n_rescale; ++i)
      if (q->rescale_steps[i] < 0 || q->rescale_steps[i] > q->n_steps - q->n_avg)
        return set_error("rescale step outside [0, n_steps - n_avg]"), MDEOS_INVALID_ARG;
    if (q->energy_every < 1) return set_error("energy_every must be >= 1"), MDEOS_INVALID_ARG;
    if (!(q->drift_tol > 0.0)) return set_error("drift_tol must be > 0"), MDEOS_INVALID_ARG;
    if (q->ensemble != MDEOS_NVE_REPIN && q->ensemble != MDEOS_NVT_LANGEVIN)
      return set_error("ensemble must be MDEOS_NVE_REPIN or MDEOS_NVT_LANGEVIN"), MDEOS_INVALID_ARG;
    if (!(std::isfinite(q->gamma) && q->gamma >= 0.0)) return set_error("gamma must be finite and >= 0"), MDEOS_INVALID_ARG;
  }
  return MDEOS_OK;
}

extern "C" mdeos_status mdeos_plan(const mdeos_cell_spec* s, float skin, mdeos_plan_info* out) {
  mdeos_status st = mdeos_validate(s, nullptr);
  if (st != MDEOS_OK) return st;
  CellPlan p;
  st = plan_cell(*s, skin, p);
  if (st != MDEOS_OK) {
    set_error("box too large for an LDS-resident extended box");
    return st;
  }
  if (out) {
    out->N = p.N;
    out->L = p.L;
    out->rl = p.rl;
    out->ext_cap = p.ext - 1;
    out->list_cap = p.list_cap;
    out->ncell = p.ncell;
    out->lds_bytes = p.lds_bytes;
    out->list_in_lds = p.list_in_lds;
    out->multi_image = p.multi_image;
  }
  return MDEOS_OK;
}

static constexpr size_t kAtomBytes = 6 * sizeof(double) + 6 * sizeof(float);
static size_t arena_elem(int i) { return i < 6 ? sizeof(double) : sizeof(float); }

extern "C" size_t mdeos_cell_bytes(int n_c) {
  const size_t N = 4ull * n_c * n_c * n_c;
  return N * kAtomBytes + sizeof(CellRec);
}

// ---------------------------------------------------------------------------
// range allocator

int RangeAlloc::alloc(int n) {
  for (auto it = free_.begin(); it != free_.end(); ++it) {
    if (it->second >= n) {
      int off = it->first, sz = it->second;
      free_.erase(it);
      if (sz > n) free_[off + n] = sz - n;
      used_ += n;
      return off;
    }
  }
  return -1;
}

void RangeAlloc::release(int off, int n) {
  auto it = free_.emplace(off, n).first;
  used_ -= n;
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

void RangeAlloc::grow(int old_cap, int new_cap) { release_raw(old_cap, new_cap - old_cap); }

void RangeAlloc::release_raw(int off, int n) {
  used_ += n;  // release() subtracts
  release(off, n);
}

// ---------------------------------------------------------------------------
// context

mdeos_status Ctx::init(const mdeos_config* cfg) {
  device = cfg ? cfg->device : 0;
  potential = cfg ? cfg->potential : MDEOS_POT_LJTS;
  if (potential != MDEOS_POT_LJTS && potential != MDEOS_POT_EAM) {
    set_error("potential must be MDEOS_POT_LJTS or MDEOS_POT_EAM");
    return MDEOS_INVALID_ARG;
  }
  const double c_in = cfg ? cfg->eam_c : 0.0;
  if (!std::isfinite(c_in)) {
    set_error("eam_c must be finite");
    return MDEOS_INVALID_ARG;
  }
  eam_c = c_in > 0.0 ? c_in : 39.432;
  skin = (cfg && cfg->skin > 0.f) ? cfg->skin : 0.f;  // 0: per cell (cell_skin)
  const float ps_in = cfg ? cfg->prune_skin : 0.f;
  if (!std::isfinite(ps_in)) {
    set_error("prune_skin must be finite");
    return MDEOS_INVALID_ARG;
  }
  prune_skin = ps_in > 0.f ? ps_in : (ps_in < 0.f ? 0.f : 0.12f);
  hbm_budget = (cfg && cfg->hbm_budget) ? cfg->hbm_budget : (size_t)64 << 30;
  autotune = cfg ? cfg->autotune : 0;
  if (cfg && cfg->tune_cache) tune_cache = cfg->tune_cache;
  precision = cfg ? cfg->precision : MDEOS_PREC_FP64;
  if (precision != MDEOS_PREC_FP64 && precision != MDEOS_PREC_KAHAN) {
    set_error("precision must be MDEOS_PREC_FP64 or MDEOS_PREC_KAHAN");
    return MDEOS_INVALID_ARG;
  }
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= device || device < 0) {
    set_error("no HIP device");
    return MDEOS_NO_DEVICE;
  }
  HCHECK(hipSetDevice(device));
  hipDeviceProp_t prop;
  HCHECK(hipGetDeviceProperties(&prop, device));
  n_cu = prop.multiProcessorCount;
  arch = prop.gcnArchName;
  arch = arch.substr(0, arch.find(':'));
  HCHECK(hipStreamCreateWithFlags(&own_stream, hipStreamNonBlocking));
  for (int i = 0; i < kAux; ++i) {
    HCHECK(hipStreamCreateWithFlags(&aux[i], hipStreamNonBlocking));
    HCHECK(hipEventCreateWithFlags(&ev_join[i], hipEventDisableTiming));
  }
  HCHECK(hipEventCreateWithFlags(&ev_fork, hipEventDisableTiming));
  HCHECK(hipEventCreate(&ev_t0));
  HCHECK(hipEventCreate(&ev_t1));
  if (init_kernel_attributes() != hipSuccess) {
    set_error("hipFuncSetAttribute failed");
    return MDEOS_DEVICE_ERROR;
  }
  if (noalloc_init(device) != hipSuccess) {
    set_error("hipGetSymbolAddress of the no-alloc workspace failed");
    return MDEOS_DEVICE_ERROR;
  }
  load_tune_cache();
  if (const char* sc = getenv("MDEOS_SHRINK_CAPS")) shrink_caps = atoi(sc) != 0;
  if (const char* tl = getenv("MDEOS_TUNE_LOG")) tune_log = atoi(tl) != 0;
  if (const char* fv = getenv("MDEOS_FORCE_VARIANT")) {
    Variant v{};
    const int nf = sscanf(fv, "%d,%d,%d,%d,%d,%d,%d,%d", &v.block, &v.apt, &v.ext, &v.list_lds, &v.wpe, &v.mi,
                          &v.nvt, &v.eam);
    if (nf >= 6 && variant_available(v))
      forced_variant = v;
  }
  return MDEOS_OK;
}

Ctx::~Ctx() {
  hipSetDevice(device);
  hipDeviceSynchronize();
  for (auto& kv : graphs) hipGraphExecDestroy(kv.second.exec);
  for (void* p : arena_ptrs) hipFree(p);
  hipFree(d_cells);
  hipFree(d_counters);
  hipFree(d_work);
  hipFree(d_gl);
  hipFree(d_results);
  hipFree(d_idx);
  hipHostFree(h_stage);
  hipHostFree(h_results);
  if (own_stream) hipStreamDestroy(own_stream);
  for (int i = 0; i < kAux; ++i) {
    if (aux[i]) hipStreamDestroy(aux[i]);
    if (ev_join[i]) hipEventDestroy(ev_join[i]);
  }
  if (ev_fork) hipEventDestroy(ev_fork);
  if (ev_t0) hipEventDestroy(ev_t0);
  if (ev_t1) hipEventDestroy(ev_t1);
}

mdeos_status Ctx::ensure_atoms(int need) {
  if (atoms.used() + need <= atom_cap && atoms.has_room(need)) return MDEOS_OK;
  int new_cap = std::max(atom_cap * 2, atom_cap + need + (1 << 20));
  if ((size_t)new_cap * kAtomBytes > hbm_budget + (kAtomBytes << 20))
    new_cap = (int)std::min<size_t>((size_t)new_cap, hbm_budget / kAtomBytes + need);
  if (atoms.used() + need > new_cap) {
    set_error("HBM budget exhausted");
    return MDEOS_OUT_OF_MEMORY;
  }
  HCHECK(hipStreamSynchronize(own_stream));
  HCHECK(hipDeviceSynchronize());
  std::vector<void*> np(12, nullptr);
  for (int i = 0; i < 12; ++i) {
    if (hipMalloc(&np[i], arena_elem(i) * (size_t)new_cap) != hipSuccess) {
      for (void* q : np) hipFree(q);
      set_error("hipMalloc of the atom arena failed");
      return MDEOS_OUT_OF_MEMORY;
    }
    if (atom_cap > 0)
      HCHECK(hipMemcpy(np[i], arena_ptrs[i], arena_elem(i) * (size_t)atom_cap, hipMemcpyDeviceToDevice));
  }
  for (void* q : arena_ptrs) hipFree(q);
  arena_ptrs = np;
  atoms.grow(atom_cap, new_cap);
  atom_cap = new_cap;
  arena = AtomArena{(double*)np[0], (double*)np[1], (double*)np[2], (double*)np[3], (double*)np[4], (double*)np[5],
                    (float*)np[6],  (float*)np[7],  (float*)np[8],  (float*)np[9],  (float*)np[10], (float*)np[11]};
  graphs_clear();
  return MDEOS_OK;
}

mdeos_status Ctx::ensure_cells(int need) {
  if (slots.has_room(need)) return MDEOS_OK;
  int new_cap = std::max(cell_cap * 2, cell_cap + need + 1024);
  HCHECK(hipDeviceSynchronize());
  CellRec* nc = nullptr;
  if (hipMalloc(&nc, sizeof(CellRec) * (size_t)new_cap) != hipSuccess) {
    set_error("hipMalloc of the cell table failed");
    return MDEOS_OUT_OF_MEMORY;
  }
  if (cell_cap > 0) HCHECK(hipMemcpy(nc, d_cells, sizeof(CellRec) * (size_t)cell_cap, hipMemcpyDeviceToDevice));
  hipFree(d_cells);
  d_cells = nc;
  h_cells.resize(new_cap);
  gen.resize(new_cap, 0);
  live.resize(new_cap, 0);
  slots.grow(cell_cap, new_cap);
  cell_cap = new_cap;
  graphs_clear();
  return MDEOS_OK;
}

template <class T>
static mdeos_status grow_dev(T*& p, size_t& cap, size_t need) {
  if (need <= cap) return MDEOS_OK;
  size_t nc = std::max(need, cap * 2);
  T* q = nullptr;
  if (hipMalloc(&q, sizeof(T) * nc) != hipSuccess) {
    set_error("hipMalloc failed");
    return MDEOS_OUT_OF_MEMORY;
  }
  hipFree(p);
  p = q;
  cap = nc;
  return MDEOS_OK;
}

mdeos_status Ctx::ensure_scratch(size_t work_n, size_t counters_n, size_t gl_bytes, size_t res_n) {
  bool changed = false;
  if (work_n > work_cap || counters_n > counters_cap || gl_bytes > gl_cap || res_n > res_cap) {
    HCHECK(hipDeviceSynchronize());
    changed = true;
  }
  mdeos_status st;
  if ((st = grow_dev(d_work, work_cap, work_n)) != MDEOS_OK) return st;
  if ((st = grow_dev(d_counters, counters_cap, counters_n)) != MDEOS_OK) return st;
  size_t gl_elems = (gl_bytes + 1) / 2;
  if ((st = grow_dev(d_gl, gl_cap_elems, gl_elems)) != MDEOS_OK) return st;
  gl_cap = gl_cap_elems * 2;
  if ((st = grow_dev(d_results, res_cap, res_n)) != MDEOS_OK) return st;
  if ((st = grow_dev(d_idx, idx_cap, res_n)) != MDEOS_OK) return st;
  if (res_n > h_results_cap) {
    hipHostFree(h_results);
    h_results = nullptr;
    if (hipHostMalloc((void**)&h_results, sizeof(DevResult) * res_n, hipHostMallocDefault) != hipSuccess) {
      set_error("hipHostMalloc failed");
      return MDEOS_OUT_OF_MEMORY;
    }
    h_results_cap = res_n;
  }
  if (changed) graphs_clear();
  return MDEOS_OK;
}

mdeos_status Ctx::ensure_stage(size_t bytes) {
  if (bytes <= stage_cap) return MDEOS_OK;
  HCHECK(hipDeviceSynchronize());
  hipHostFree(h_stage);
  h_stage = nullptr;
  size_t nb = std::max(bytes, stage_cap * 2);
  if (hipHostMalloc((void**)&h_stage, nb, hipHostMallocDefault) != hipSuccess) {
    set_error("hipHostMalloc failed");
    return MDEOS_OUT_OF_MEMORY;
  }
  stage_cap = nb;
  return MDEOS_OK;
}

void Ctx::graphs_clear() {
  for (auto& kv : graphs) hipGraphExecDestroy(kv.second.exec);
  graphs.clear();
}

// Fills the host part of a cell record.
void Ctx::fill_record(CellRec& r, const mdeos_cell_spec& s, const mdeos_schedule& q, const CellPlan& p,
                      int atom_off) {
  memset(&r, 0, sizeof(r));
  r.rho = s.rho;
  r.e = s.e;
  r.Lw = p.Lw;
  r.V = p.Lw * p.Lw * p.Lw;
  r.drift_tol = q.drift_tol;
  r.warm_scale = 1.0;
  r.seed = s.seed;
  r.cell_id = s.cell_id;
  r.L = p.L;
  r.rc = s.rc;
  r.dt = s.dt;
  r.rl = p.rl;
  r.n_c = s.n_c;
  r.N = p.N;
  r.n_steps = q.n_steps;
  r.n_avg = q.n_avg;
  r.n_blocks = q.n_blocks;
  r.n_rescale = q.n_rescale;
  for (int i = 0; i < q.n_rescale; ++i) r.rescale_steps[i] = q.rescale_steps[i];
  r.energy_every = q.energy_every;
  r.ensemble = q.ensemble;
  r.gamma = q.gamma;
  r.T_th = 2.0 * p.N * s.e / (3.0 * p.N - 3.0);  // first guess: all energy kinetic
  r.atom_off = atom_off;
  r.nce = p.nce;
  r.stencil = p.stencil;
  r.phase = PH_COLD;
  r.step = 0;
}

mdeos_handle Ctx::handle_of(int slot) const { return ((long long)gen[slot] << 32) | (unsigned)slot; }

int Ctx::slot_of(mdeos_handle h) const {
  long long s = h & 0xffffffffLL;
  if (h < 0 || s >= cell_cap || !live[s] || (long long)gen[s] != (h >> 32)) return -1;
  return (int)s;
}

// Allocates n cells (contiguous slots and atoms when possible).
mdeos_status Ctx::alloc_cells(int n, const mdeos_cell_spec* specs, const mdeos_schedule& q, std::vector<int>& out) {
  std::vector<CellPlan> plans(n);
  long long total_atoms = 0;
  for (int i = 0; i < n; ++i) {
    mdeos_status st = mdeos_validate(&specs[i], &q);
    if (st != MDEOS_OK) return st;
    st = plan_cell(specs[i], cell_skin(specs[i]), plans[i]);
    plans[i].nvt = q.ensemble == MDEOS_NVT_LANGEVIN ? 1 : 0;
    if (st != MDEOS_OK) {
      set_error("cell " + std::to_string(i) + ": box too large for an LDS-resident extended box");
      return st;
    }
    total_atoms += plans[i].N;
  }
  if ((size_t)(atoms.used() + total_atoms) * kAtomBytes + (size_t)(slots.used() + n) * sizeof(CellRec) > hbm_budget) {
    set_error("HBM budget exhausted");
    return MDEOS_OUT_OF_MEMORY;
  }
  mdeos_status st = ensure_cells(n);
  if (st != MDEOS_OK) return st;
  st = ensure_atoms((int)total_atoms);
  if (st != MDEOS_OK) return st;
  out.resize(n);
  int s0 = slots.alloc(n);
  int a0 = atoms.alloc((int)total_atoms);
  int aoff = a0;
  for (int i = 0; i < n; ++i) {
    int slot = s0 >= 0 ? s0 + i : slots.alloc(1);
    int off = a0 >= 0 ? aoff : atoms.alloc(plans[i].N);
    if (slot < 0 || off < 0) {
      set_error("arena fragmentation");
      return MDEOS_OUT_OF_MEMORY;
    }
    aoff += plans[i].N;
    out[i] = slot;
    live[slot] = 1;
    gen[slot] += 1;
    fill_record(h_cells[slot], specs[i], q, plans[i], off);
    cell_plan[slot] = plans[i];
  }
  return MDEOS_OK;
}

void Ctx::free_cells(const std::vector<int>& idx) {
  for (int s : idx) {
    if (s < 0 || !live[s]) continue;
    live[s] = 0;
    slots.release(s, 1);
    atoms.release(h_cells[s].atom_off, h_cells[s].N);
    cell_plan.erase(s);
  }
}

// Uploads the host records of the given slots (contiguous runs in one copy each).
mdeos_status Ctx::upload_records(const std::vector<int>& idx, hipStream_t s) {
  if (idx.empty()) return MDEOS_OK;
  std::vector<int> sorted = idx;
  std::sort(sorted.begin(), sorted.end());
  mdeos_status st = ensure_stage(sizeof(CellRec) * sorted.size());
  if (st != MDEOS_OK) return st;
  // wait for earlier uses of the staging buffer
  HCHECK(hipStreamSynchronize(s));
  CellRec* stage = (CellRec*)h_stage;
  size_t i = 0;
  size_t k = 0;
  while (i < sorted.size()) {
    size_t j = i;
    while (j + 1 < sorted.size() && sorted[j + 1] == sorted[j] + 1) ++j;
    for (size_t q = i; q <= j; ++q) stage[k + (q - i)] = h_cells[sorted[q]];
    HCHECK(hipMemcpyAsync(d_cells + sorted[i], stage + k, sizeof(CellRec) * (j - i + 1), hipMemcpyHostToDevice, s));
    k += j - i + 1;
    i = j + 1;
  }
  return MDEOS_OK;
}

// ---------------------------------------------------------------------------
// buckets and launches

static int variant_score(const Variant& v, int N) {
  // fewest idle threads first, then 512-thread blocks
  int idle = v.block * v.apt - N;
  return idle * 4 + (v.block == 512 ? 0 : 1);
}

static Caps caps_of(const CellPlan& p) {
  Caps c;
  c.n_pad = align_up(p.N, 64);
  c.list_cap = p.list_cap;
  c.ncell_cap = p.ncell;
  c.gmax = c.n_pad / 64;
  c.ring = ring_for(c.gmax);
  return c;
}

// Every launch shape that fits a (merged) plan, best first by a static model:
// most resident waves per CU (registers allow wpe waves per SIMD, LDS allows
// whole boxes), then the fewest idle threads, the neighbour list in LDS, the
// smallest position stride.
int Ctx::rank_variants(const CellPlan& p, std::vector<Variant>& out) const {
  const Caps c = caps_of(p);
  std::vector<std::pair<int, int>> scored;
  for (int i = 0; i < variant_count(); ++i) {
    const Variant v = variant_at(i);
    const int lds = lds_layout(v.ext, c, v.list_lds, frc_slots(v)).total;
    if (v.mi != p.minimg || v.nvt != p.nvt || v.eam != (potential == MDEOS_POT_EAM ? 1 : 0) ||
        v.block * v.apt < p.N || v.ext - 1 < p.ext_need || lds > kLdsMax)
      continue;
    const int wg_by_lds = kLdsMax / lds, wg_by_regs = std::max(1, 4 * v.wpe / (v.block / 64));
    const int waves = std::min(wg_by_lds, wg_by_regs) * (v.block / 64);
    scored.push_back({-waves * 4096 + variant_score(v, p.N) * 16 + (v.list_lds ? 0 : 8) + (v.ext - p.ext_need) / 1024, i});
  }
  std::stable_sort(scored.begin(), scored.end());
  out.clear();
  for (auto& sc : scored) out.push_back(variant_at(sc.second));
  return (int)out.size();
}

// Picks the launch shape for a (merged) plan: a forced shape, else a tuned
// one if the tune cache has one that fits, else the best by the static model.
bool Ctx::choose_variant(const CellPlan& p, Variant& out) const {
  std::vector<Variant> ranked;
  if (rank_variants(p, ranked) == 0) return false;
  auto fits = [&](const Variant& v) {
    for (const Variant& r : ranked)
      if (same_variant(r, v)) return true;
    return false;
  };
  if (forced_variant.block > 0 && fits(forced_variant)) {
    out = forced_variant;
    return true;
  }
  auto tv = tuned.find(tune_key(p));
  if (tv != tuned.end() && fits(tv->second)) {
    out = tv->second;
    return true;
  }
  out = ranked[0];
  return true;
}

// Online autotuning of launch shapes. A cell's results do not depend on the
// launch shape or on chunk boundaries (bit for bit), so candidate shapes are
// timed on successive chunks of the batch's own work and nothing is
// recomputed: one untimed chunk (lift and the first steps), then kTuneRounds
// rounds of one kTuneSteps chunk per candidate, the bucket alone on the
// device. The fastest (mean over rounds) is kept under the bucket's tune key
// and written to the tune cache.
static constexpr int kTuneSteps = 40, kTuneRounds = 2, kTuneMaxCand = 6, kTuneMinCells = 64;

mdeos_status Ctx::autotune_buckets(std::vector<Bucket>& buckets, hipStream_t s) {
  bool changed = false;
  for (Bucket& b : buckets) {
    if (forced_variant.block > 0 || (int)b.cells.size() < kTuneMinCells) continue;
    const std::string key = tune_key(b.plan);
    if (tuned.count(key)) continue;
    std::vector<Variant> cand;
    rank_variants(b.plan, cand);
    if ((int)cand.size() > kTuneMaxCand) cand.resize(kTuneMaxCand);
    if (cand.size() < 2) {
      if (!cand.empty()) tuned[key] = cand[0], changed = true;
      continue;
    }
    int left = 1 << 30;
    for (int c : b.cells) left = std::min(left, h_cells[c].n_steps - h_cells[c].step);
    if (left < (1 + kTuneRounds * (int)cand.size()) * kTuneSteps + 1) continue;
    std::vector<Bucket> one{b};
    auto use = [&](const Variant& v) {
      one[0].v = v;
      one[0].lds = lds_layout(v.ext, one[0].caps, v.list_lds, frc_slots(v)).total;
      one[0].grid = std::max(1, std::min<int>((int)b.cells.size(), std::max(1, occupancy(v, one[0].lds)) * n_cu));
    };
    use(b.v);
    mdeos_status st = run_buckets(one, kTuneSteps, s, false);
    if (st != MDEOS_OK) return st;
    // A candidate is judged by the time of its steps: a chunk of kTuneSteps
    // steps minus a chunk of none, which costs what every chunk pays once
    // (loading the state, rebuilding the lists, storing) and which a whole
    // run pays only once. The cells keep evolving while they are timed (a
    // lattice melting, the rebuild rate settling), so a chunk costs more or
    // less depending on when it runs: rounds alternate the candidate order
    // (forward, then backward) and each candidate takes its mean over the
    // rounds, so a cost that drifts linearly adds the same to every candidate.
    auto timed = [&](int budget, float& ms) {
      mdeos_status e2 = run_buckets(one, budget, s, false);
      if (e2 != MDEOS_OK) return e2;
      if (hipEventSynchronize(ev_t1) != hipSuccess || hipEventElapsedTime(&ms, ev_t0, ev_t1) != hipSuccess)
        return set_error("tuning timer failed"), MDEOS_DEVICE_ERROR;
      return MDEOS_OK;
    };
    std::vector<double> mean(cand.size(), 0.0);
    for (int r = 0; r < kTuneRounds; ++r) {
      for (size_t j = 0; j < cand.size(); ++j) {
        const size_t i = (r & 1) ? cand.size() - 1 - j : j;
        use(cand[i]);
        float t_none = 0.f, t_steps = 0.f;
        if ((st = timed(-1, t_none)) != MDEOS_OK || (st = timed(kTuneSteps, t_steps)) != MDEOS_OK) return st;
        mean[i] += (double)(t_steps - t_none) / kTuneRounds;
        if (tune_log)
          fprintf(stderr, "[mdeos tune] %s round %d: %d,%d,%d,%d,%d,%d,%d,%d no steps %.3f ms, %d steps %.3f ms\n",
                  key.c_str(), r, cand[i].block, cand[i].apt, cand[i].ext, cand[i].list_lds, cand[i].wpe,
                  cand[i].mi, cand[i].nvt, cand[i].eam, t_none, kTuneSteps, t_steps);
      }
    }
    const size_t w = std::min_element(mean.begin(), mean.end()) - mean.begin();
    tuned[key] = cand[w];
    changed = true;
    b.v = cand[w];
    b.lds = lds_layout(b.v.ext, b.caps, b.v.list_lds, frc_slots(b.v)).total;
    b.grid = std::max(1, std::min<int>((int)b.cells.size(), std::max(1, occupancy(b.v, b.lds)) * n_cu));
    ++tune_runs;
  }
  if (changed) save_tune_cache();
  return MDEOS_OK;
}

std::string Ctx::tune_key(const CellPlan& p) const {
  char buf[128];
  snprintf(buf, sizeof(buf), "%s/N%d/rl%.2f/ext%d/list%d/cells%d/mi%d/prec%d", arch.c_str(), p.N, p.rl,
           align_up(p.ext_need, 512), align_up(p.list_cap, 16), align_up(p.ncell, 256), p.minimg, precision);
  std::string key = buf;
  if (p.nvt) key += "/nvt";
  if (potential == MDEOS_POT_EAM) key += "/eam";
  if (prune_lists()) {
    snprintf(buf, sizeof(buf), "/prune%.3f", prune_skin);
    key += buf;
  }
  return key;
}

// Merged plan of a set of cells with one atom count: capacities are maxima.
static CellPlan merge_plans(const std::vector<const CellPlan*>& ps) {
  CellPlan m = *ps[0];  // all plans of a bucket share N and the image method
  for (const CellPlan* p : ps) {
    m.ext_need = std::max(m.ext_need, p->ext_need);
    m.list_cap = std::max(m.list_cap, p->list_cap);
    m.ncell = std::max(m.ncell, p->ncell);
    m.rl = std::max(m.rl, p->rl);
  }
  return m;
}

// Groups cells into launches: one bucket per (atom count, cutoff) with
// capacities that cover every cell in it; a bucket whose merged capacities do
// not fit any launch shape is split by extended-box size. In sticky mode
// (serving) the capacities of a bucket only grow and every bucket seen before
// stays in the launch set (possibly without cells), so the launch set, and with
// it the captured graph, stays fixed while the batch composition changes.
void Ctx::make_buckets(const std::vector<int>& cells, std::vector<Bucket>& out, int step_budget, bool sticky) {
  (void)step_budget;
  std::map<std::pair<int, int>, std::vector<int>> groups;
  for (int s : cells) {
    const CellPlan& p = cell_plan[s];
    groups[{p.N * 4 + p.minimg * 2 + p.nvt, (int)std::lround(h_cells[s].rc * 1000.0)}].push_back(s);
  }
  if (sticky)
    for (auto& kv : sticky_plans) groups[kv.first];  // keep every bucket seen before
  out.clear();
  std::function<void(std::pair<int, int>, std::vector<int>&)> place = [&](std::pair<int, int> key,
                                                                           std::vector<int>& cs) {
    std::vector<const CellPlan*> ps;
    for (int s : cs) ps.push_back(&cell_plan[s]);
    CellPlan merged;
    if (!ps.empty()) merged = merge_plans(ps);
    if (sticky) {
      auto it = sticky_plans.find(key);
      if (it != sticky_plans.end()) {
        if (ps.empty()) merged = it->second;
        else merged = merge_plans({&merged, &it->second});
      }
    }
    if (ps.empty() && !sticky) return;
    Variant v;
    if (!choose_variant(merged, v)) {
      if (cs.size() <= 1) return;  // cannot happen: every single plan fits
      std::sort(cs.begin(), cs.end(), [&](int a, int b) { return cell_plan[a].ext_need < cell_plan[b].ext_need; });
      std::vector<int> lo(cs.begin(), cs.begin() + cs.size() / 2), hi(cs.begin() + cs.size() / 2, cs.end());
      place(key, lo);
      place(key, hi);
      return;
    }
    if (sticky) sticky_plans[key] = merged;
    Bucket b;
    b.v = v;
    b.plan = merged;
    b.caps = caps_of(merged);
    b.lds = lds_layout(v.ext, b.caps, v.list_lds, frc_slots(v)).total;
    b.cells = cs;
    // longest first
    std::stable_sort(b.cells.begin(), b.cells.end(), [&](int a, int c) {
      const CellPlan &pa = cell_plan[a], &pc = cell_plan[c];
      double ca = (double)pa.N * pa.list_cap * (h_cells[a].n_steps - h_cells[a].step);
      double cc = (double)pc.N * pc.list_cap * (h_cells[c].n_steps - h_cells[c].step);
      return ca > cc;
    });
    out.push_back(std::move(b));
  };
  for (auto& kv : groups) place(kv.first, kv.second);
  for (Bucket& b : out) {
    int occ = std::max(1, occupancy(b.v, b.lds));
    b.grid = sticky ? occ * n_cu : std::max(1, std::min<int>((int)b.cells.size(), occ * n_cu));
  }
}

// Launches every bucket (concurrently on the auxiliary streams). The work
// lists and their counts live in device memory, so the captured graph of a
// given set of bucket shapes is replayed for any batch composition.
mdeos_status Ctx::run_buckets(std::vector<Bucket>& buckets, int step_budget, hipStream_t s, bool use_graph) {
  if (buckets.empty()) return MDEOS_OK;
  if (buckets.size() > (size_t)kMaxBuckets) return set_error("too many size buckets"), MDEOS_INVALID_ARG;
  size_t work_n = 2 * kMaxBuckets, gl_bytes = 0;
  for (Bucket& b : buckets) {
    b.work_off = (int)work_n;
    work_n += b.cells.size();
    if (!b.v.list_lds) {
      // the lists of every workgroup, then (with pruning) their inner lists
      b.gl_off = gl_bytes;
      const size_t one = (size_t)b.grid * b.caps.list_cap * b.caps.n_pad * 2;
      gl_bytes += ((prune_lists() ? 2 : 1) * one + 255) / 256 * 256;
    }
  }
  mdeos_status st = ensure_scratch(work_n, kMaxBuckets, gl_bytes, 1);
  if (st != MDEOS_OK) return st;
  std::vector<int> host_work(work_n, 0);
  for (size_t i = 0; i < buckets.size(); ++i) {
    host_work[2 * i] = (int)buckets[i].cells.size();
    host_work[2 * i + 1] = buckets[i].work_off;
    std::copy(buckets[i].cells.begin(), buckets[i].cells.end(), host_work.begin() + buckets[i].work_off);
  }
  char hdr[96];
  snprintf(hdr, sizeof(hdr), "%d|%p|", step_budget, (void*)s);
  std::string key = hdr;
  for (Bucket& b : buckets) {
    char bb[128];
    snprintf(bb, sizeof(bb), "%d,%d,%d,%d,%d,%d,%d,%d,%d,%d,%d,%d,%d,%zu;", b.v.mi, b.v.nvt, b.v.eam, b.v.block, b.v.apt,
             b.v.ext, b.v.list_lds, b.v.wpe, b.caps.list_cap, b.caps.ncell_cap, b.caps.n_pad, b.grid, b.lds, b.gl_off);
    key += bb;
  }
  HCHECK(hipMemcpyAsync(d_work, host_work.data(), sizeof(int) * host_work.size(), hipMemcpyHostToDevice, s));

  auto launch_all = [&](hipStream_t ms) -> hipError_t {
    hipError_t e = launch_zero_ints(d_counters, (int)buckets.size(), ms);
    if (e != hipSuccess) return e;
    if (buckets.size() == 1) {
      Bucket& b = buckets[0];
      return launch_advance(b.v, make_params(b, 0, step_budget), b.grid, b.lds, ms);
    }
    e = hipEventRecord(ev_fork, ms);
    if (e != hipSuccess) return e;
    const int na = std::min<int>(kAux, (int)buckets.size());
    for (int i = 0; i < na; ++i)
      if ((e = hipStreamWaitEvent(aux[i], ev_fork, 0)) != hipSuccess) return e;
    // Longest processing time first: buckets in decreasing estimated
    // duration, each on the stream with the least duration so far, so the
    // longest start at once and the short ones fill in around them. A
    // bucket lasts at least as long as its longest cell (one workgroup
    // advances a cell), and about its total cost over its workgroups when
    // it has many cells; a few large cells must therefore start early.
    std::vector<double> cost(buckets.size(), 0.0), load(na, 0.0);
    std::vector<int> order(buckets.size());
    for (size_t i = 0; i < buckets.size(); ++i) {
      order[i] = (int)i;
      double total = 0.0, longest = 0.0;
      // a minimum-image pair costs about 1.3 times a ghost-image one (the
      // fixed-point image difference adds a conversion and a multiply per axis)
      for (int c : buckets[i].cells) {
        const double one = (double)cell_plan[c].N * cell_plan[c].list_cap *
                           std::max(1, h_cells[c].n_steps - h_cells[c].step) * (cell_plan[c].minimg ? 1.3 : 1.0);
        total += one;
        longest = std::max(longest, one);
      }
      cost[i] = std::max(total / std::max(1, buckets[i].grid), longest);
    }
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
    for (int i : order) {
      const int q = (int)(std::min_element(load.begin(), load.end()) - load.begin());
      load[q] += cost[i];
      Bucket& b = buckets[i];
      if ((e = launch_advance(b.v, make_params(b, i, step_budget), b.grid, b.lds, aux[q])) != hipSuccess) return e;
    }
    for (int i = 0; i < na; ++i) {
      if ((e = hipEventRecord(ev_join[i], aux[i])) != hipSuccess) return e;
      if ((e = hipStreamWaitEvent(ms, ev_join[i], 0)) != hipSuccess) return e;
    }
    return hipSuccess;
  };

  HCHECK(hipEventRecord(ev_t0, s));
  if (!use_graph) {
    HCHECK(launch_all(s));
    HCHECK(hipEventRecord(ev_t1, s));
    timed_launches = (int)buckets.size();
    return MDEOS_OK;
  }
  auto it = graphs.find(key);
  if (it == graphs.end()) {
    if (graphs.size() > 256) graphs_clear();
    hipGraph_t g;
    HCHECK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    hipError_t le = launch_all(s);
    hipError_t ce = hipStreamEndCapture(s, &g);
    if (le != hipSuccess || ce != hipSuccess) {
      if (ce == hipSuccess) hipGraphDestroy(g);
      set_error(std::string("graph capture failed: ") + hipGetErrorString(le != hipSuccess ? le : ce));
      return MDEOS_DEVICE_ERROR;
    }
    GraphEntry ge;
    HCHECK(hipGraphInstantiate(&ge.exec, g, nullptr, nullptr, 0));
    hipGraphDestroy(g);
    it = graphs.emplace(key, ge).first;
  }
  HCHECK(hipGraphLaunch(it->second.exec, s));
  HCHECK(hipEventRecord(ev_t1, s));
  timed_launches = (int)buckets.size();
  return MDEOS_OK;
}

// Restricting operator over the given slots; results to the host.
mdeos_status Ctx::restrict_cells(const std::vector<int>& idx, mdeos_result* out, hipStream_t s) {
  const int n = (int)idx.size();
  if (n == 0) return MDEOS_OK;
  mdeos_status st = ensure_scratch(2 * kMaxBuckets, kMaxBuckets, 0, n);
  if (st != MDEOS_OK) return st;
  HCHECK(hipMemcpyAsync(d_idx, idx.data(), sizeof(int) * n, hipMemcpyHostToDevice, s));
  HCHECK(launch_restrict(d_cells, d_idx, n, d_results, s));
  return fetch_results(n, out, s);
}

AdvanceParams Ctx::make_params(const Bucket& b, int bi, int step_budget) {
  AdvanceParams p;
  p.cells = d_cells;
  p.work_base = d_work;
  p.meta = d_work + 2 * bi;
  p.counter = d_counters + bi;
  p.step_budget = step_budget;
  p.a = arena;
  p.gl_list = b.v.list_lds ? nullptr : d_gl + b.gl_off / 2;
  p.gl_ilist = (b.v.list_lds || !prune_lists()) ? nullptr
                                                 : p.gl_list + (size_t)b.grid * b.caps.list_cap * b.caps.n_pad;
  p.prune_skin = prune_skin;
  p.caps = b.caps;
  p.kahan = precision == MDEOS_PREC_KAHAN ? 1 : 0;
  p.eam_c = eam_c;
  return p;
}

mdeos_status Ctx::fetch_results(int n, mdeos_result* out, hipStream_t s) {
  HCHECK(hipMemcpyAsync(h_results, d_results, sizeof(DevResult) * n, hipMemcpyDeviceToHost, s));
  HCHECK(hipStreamSynchronize(s));
  static_assert(sizeof(DevResult) == sizeof(mdeos_result), "result layout");
  memcpy(out, h_results, sizeof(DevResult) * n);
  return MDEOS_OK;
}

hipStream_t Ctx::pick(void* stream) const { return stream ? (hipStream_t)stream : own_stream; }

// ---------------------------------------------------------------------------
// C ABI

#define CTX_GUARD(ctx)                                  \
  if (!(ctx)) return MDEOS_INVALID_ARG;                 \
  if (hipSetDevice((ctx)->device) != hipSuccess) return MDEOS_DEVICE_ERROR;

extern "C" mdeos_status mdeos_create(const mdeos_config* cfg, mdeos_ctx** out) {
  if (!out) return MDEOS_INVALID_ARG;
  *out = nullptr;
  Ctx* c = new Ctx();
  mdeos_status st = c->init(cfg);
  if (st != MDEOS_OK) {
    delete c;
    return st;
  }
  *out = reinterpret_cast<mdeos_ctx*>(c);
  return MDEOS_OK;
}

extern "C" mdeos_status mdeos_destroy(mdeos_ctx* ctx) {
  if (!ctx) return MDEOS_INVALID_ARG;
  Ctx* c = reinterpret_cast<Ctx*>(ctx);
  c->serve_shutdown();
  delete c;
  return MDEOS_OK;
}

static Ctx* C_(mdeos_ctx* c) { return reinterpret_cast<Ctx*>(c); }

extern "C" mdeos_status mdeos_lift(mdeos_ctx* ctx, int n, const mdeos_cell_spec* specs, const mdeos_schedule* sched,
                                   mdeos_handle* out, void* stream) {
  CTX_GUARD(C_(ctx));
  Ctx* c = C_(ctx);
  if (n < 0 || (n > 0 && (!specs || !sched || !out))) return MDEOS_INVALID_ARG;
  if (n == 0) return MDEOS_OK;
  std::lock_guard<std::recursive_mutex> lk(c->mu);
  hipStream_t s = c->pick(stream);
  std::vector<int> idx;
  mdeos_status st = c->alloc_cells(n, specs, *sched, idx);
  if (st != MDEOS_OK) return st;
  st = c->upload_records(idx, s);
  if (st == MDEOS_OK) {
    std::vector<Bucket> b;
    c->make_buckets(idx, b, -1);
    st = c->run_buckets(b, -1, s, false);
  }
  if (st != MDEOS_OK) {
    c->free_cells(idx);
    return st;
  }
  for (int i = 0; i < n; ++i) out[i] = c->handle_of(idx[i]);
  return MDEOS_OK;
}

extern "C" mdeos_status mdeos_lift_from_state(mdeos_ctx* ctx, const mdeos_cell_spec* spec, const mdeos_schedule* sched,
                                              const double* xyz, const double* v, mdeos_handle* out, void* stream) {
  CTX_GUARD(C_(ctx));
  Ctx* c = C_(ctx);
  if (!spec || !sched || !xyz || !v || !out) return MDEOS_INVALID_ARG;
  std::lock_guard<std::recursive_mutex> lk(c->mu);
  hipStream_t s = c->pick(stream);
  std::vector<int> idx;
  mdeos_status st = c->alloc_cells(1, spec, *sched, idx);
  if (st != MDEOS_OK) return st;
  const int slot = idx[0];
  CellRec& r = c->h_cells[slot];
  r.phase = PH_STATE;
  st = c->upload_state(slot, xyz, v, s);
  if (st == MDEOS_OK) st = c->upload_records(idx, s);
  if (st == MDEOS_OK) {
    std::vector<Bucket> b;
    c->make_buckets(idx, b, -1);
    st = c->run_buckets(b, -1, s, false);
  }
  if (st == MDEOS_OK && hipStreamSynchronize(s) != hipSuccess) st = MDEOS_DEVICE_ERROR;
  if (st != MDEOS_OK) {
    c->free_cells(idx);
    return st;
  }
  *out = c->handle_of(slot);
  return MDEOS_OK;
}

mdeos_status Ctx::upload_state(int slot, const double* xyz, const double* v, hipStream_t s) {
  const CellRec& r = h_cells[slot];
  const int N = r.N;
  mdeos_status st = ensure_stage(sizeof(double) * 6 * N);
  if (st != MDEOS_OK) return st;
  HCHECK(hipStreamSynchronize(s));
  double* f = (double*)h_stage;
  const double L = r.Lw;
  for (int a = 0; a < N; ++a) {
    for (int k = 0; k < 3; ++k) {
      double q = xyz[3 * a + k];
      q = q - L * std::floor(q / L);
      if (q >= L || q < 0.0) q = 0.0;
      f[k * N + a] = q;
      f[(3 + k) * N + a] = v[3 * a + k];
    }
  }
  double* dst[6] = {arena.x, arena.y, arena.z, arena.vx, arena.vy, arena.vz};
  for (int k = 0; k < 6; ++k)
    HCHECK(hipMemcpyAsync(dst[k] + r.atom_off, f + k * N, sizeof(double) * N, hipMemcpyHostToDevice, s));
  HCHECK(hipStreamSynchronize(s));
  return MDEOS_OK;
}

extern "C" mdeos_status mdeos_warm_start(mdeos_ctx* ctx, int n, const mdeos_handle* h, const double* rho,
                                         const double* e, const mdeos_schedule* sched, void* stream) {
  CTX_GUARD(C_(ctx));
  Ctx* c = C_(ctx);
  if (n < 0 || (n > 0 && (!h || !rho || !e || !sched))) return MDEOS_INVALID_ARG;
  std::lock_guard<std::recursive_mutex> lk(c->mu);
  hipStream_t s = c->pick(stream);
  bool has0 = false;
  for (int i = 0; i < sched->n_rescale; ++i) has0 |= sched->rescale_steps[i] == 0;
  if (!has0) return set_error("a warm schedule must re-pin at step 0"), MDEOS_INVALID_ARG;
  std::vector<int> idx(n);
  for (int i = 0; i < n; ++i) {
    idx[i] = c->slot_of(h[i]);
    if (idx[i] < 0) return set_error("stale handle"), MDEOS_INVALID_ARG;
    mdeos_cell_spec sp;
    const CellRec& r = c->h_cells[idx[i]];
    sp.rho = rho[i];
    sp.e = e[i];
    sp.n_c = r.n_c;
    sp.rc = r.rc;
    sp.dt = r.dt;
    sp.seed = r.seed;
    sp.cell_id = r.cell_id;
    mdeos_status st = mdeos_validate(&sp, sched);
    if (st != MDEOS_OK) return st;
  }
  for (int i = 0; i < n; ++i) {
    const int slot = idx[i];
    CellRec& r = c->h_cells[slot];
    mdeos_cell_spec sp;
    sp.rho = rho[i];
    sp.e = e[i];
    sp.n_c = r.n_c;
    sp.rc = r.rc;
    sp.dt = r.dt;
    sp.seed = r.seed;
    sp.cell_id = r.cell_id;
    CellPlan p;
    mdeos_status st = plan_cell(sp, c->cell_skin(sp), p);
    if (st != MDEOS_OK) return set_error("warm target too large"), st;
    p.nvt = sched->ensemble == MDEOS_NVT_LANGEVIN ? 1 : 0;
    const double Lold = r.Lw;
    const int off = r.atom_off, query = r.query;
    c->fill_record(r, sp, *sched, p, off);
    r.warm_scale = p.Lw / Lold;
    r.query = query + 1;
    r.phase = PH_WARM;
    c->cell_plan[slot] = p;
  }
  return c->upload_records(idx, s);
}

extern "C" mdeos_status mdeos_advance(mdeos_ctx* ctx, int n, const mdeos_handle* h, int n_steps, void* stream) {
  CTX_GUARD(C_(ctx));
  Ctx* c = C_(ctx);
  if (n < 0 || n_steps < 0 || (n > 0 && !h)) return MDEOS_INVALID_ARG;
  if (n == 0) return MDEOS_OK;
  std::lock_guard<std::recursive_mutex> lk(c->mu);
  hipStream_t s = c->pick(stream);
  std::vector<int> idx(n);
  for (int i = 0; i < n; ++i) {
    idx[i] = c->slot_of(h[i]);
    if (idx[i] < 0) return set_error("stale handle"), MDEOS_INVALID_ARG;
  }
  std::vector<Bucket> b;
  c->make_buckets(idx, b, n_steps);
  return c->run_buckets(b, n_steps == 0 ? -1 : n_steps, s, true);
}

extern "C" mdeos_status mdeos_restrict(mdeos_ctx* ctx, int n, const mdeos_handle* h, mdeos_result* out, void* stream) {
  CTX_GUARD(C_(ctx));
  Ctx* c = C_(ctx);
  if (n < 0 || (n > 0 && (!h || !out))) return MDEOS_INVALID_ARG;
  if (n == 0) return MDEOS_OK;
  std::lock_guard<std::recursive_mutex> lk(c->mu);
  hipStream_t s = c->pick(stream);
  std::vector<int> idx(n);
  for (int i = 0; i < n; ++i) {
    idx[i] = c->slot_of(h[i]);
    if (idx[i] < 0) return set_error("stale handle"), MDEOS_INVALID_ARG;
  }
  mdeos_status st = c->restrict_cells(idx, out, s);
  if (st != MDEOS_OK) return st;
  for (int i = 0; i < n; ++i) {
    const bool failed = (out[i].status & (MDEOS_CELL_NONFINITE | MDEOS_CELL_OVERFLOW)) != 0;
    if (!failed && out[i].n_samples < c->h_cells[idx[i]].n_avg) return MDEOS_NOT_READY;
  }
  return MDEOS_OK;
}

// Runs lift + schedule + restrict for n cells (batched, or one launch per cell
// for the plain path). Cells that overflowed a capacity are re-run from the
// lift with larger capacities; capacities do not change a cell's arithmetic.
mdeos_status Ctx::eval(int n, const mdeos_cell_spec* specs, const mdeos_schedule* sched, mdeos_result* out,
                       hipStream_t s, bool plain) {
  std::vector<int> idx;
  mdeos_status st = alloc_cells(n, specs, *sched, idx);
  if (st != MDEOS_OK) return st;
  if (shrink_caps) {
    for (int slot : idx) {
      CellPlan p = cell_plan[slot];
      p.list_cap = 8;
      if (finish_plan(p) != MDEOS_OK) continue;
      const CellRec old = h_cells[slot];
      mdeos_cell_spec sp{old.rho, old.e, old.n_c, old.rc, old.dt, old.seed, old.cell_id};
      fill_record(h_cells[slot], sp, *sched, p, old.atom_off);
      cell_plan[slot] = p;
    }
  }
  std::vector<int> pos(n);
  for (int i = 0; i < n; ++i) pos[i] = i;
  std::vector<int> todo = idx;
  for (int attempt = 0; attempt < 3 && st == MDEOS_OK && !todo.empty(); ++attempt) {
    st = upload_records(todo, s);
    if (st != MDEOS_OK) break;
    std::vector<mdeos_result> res(todo.size());
    if (!plain) {
      std::vector<Bucket> b;
      make_buckets(todo, b, 0);
      if (autotune) st = autotune_buckets(b, s);
      if (st == MDEOS_OK) st = run_buckets(b, 0, s, true);
      if (st == MDEOS_OK) st = restrict_cells(todo, res.data(), s);
    } else {
      for (size_t i = 0; i < todo.size() && st == MDEOS_OK; ++i) {
        std::vector<int> one{todo[i]};
        std::vector<Bucket> b;
        make_buckets(one, b, 0);
        for (Bucket& q : b) q.grid = 1;
        st = run_buckets(b, 0, s, false);
        if (st == MDEOS_OK) st = restrict_cells(one, res.data() + i, s);
      }
    }
    if (st != MDEOS_OK) break;
    std::vector<int> again, again_pos;
    for (size_t i = 0; i < todo.size(); ++i) {
      out[pos[i]] = res[i];
      if (!(res[i].status & MDEOS_CELL_OVERFLOW) || attempt == 2) continue;
      const int slot = todo[i];
      CellPlan p = cell_plan[slot];
      const CellRec old = h_cells[slot];
      mdeos_cell_spec sp{old.rho, old.e, old.n_c, old.rc, old.dt, old.seed, old.cell_id};
      // grow by half, to the sizes the overflow measured plus a margin, and
      // never below what a fresh plan of the cell gives
      CellPlan fresh;
      const bool have_fresh = plan_cell(sp, cell_skin(sp), fresh) == MDEOS_OK && fresh.minimg == p.minimg;
      p.ext_need = std::max(p.ext_need + p.ext_need / 2, res[i].max_ext + 64);
      p.list_cap = align_up(std::max(p.list_cap + p.list_cap / 2, res[i].max_list + 16), 8);
      if (have_fresh) {
        p.ext_need = std::max(p.ext_need, fresh.ext_need);
        p.list_cap = std::max(p.list_cap, fresh.list_cap);
      }
      if (finish_plan(p) != MDEOS_OK) continue;  // no larger launch shape: report the overflow
      fill_record(h_cells[slot], sp, *sched, p, old.atom_off);
      cell_plan[slot] = p;
      again.push_back(slot);
      again_pos.push_back(pos[i]);
    }
    todo = again;
    pos = again_pos;
  }
  free_cells(idx);
  return st;
}

extern "C" mdeos_status mdeos_eval_batch(mdeos_ctx* ctx, int n, const mdeos_cell_spec* specs,
                                         const mdeos_schedule* sched, mdeos_result* out, void* stream) {
  CTX_GUARD(C_(ctx));
  Ctx* c = C_(ctx);
  if (n < 0 || (n > 0 && (!specs || !sched || !out))) return MDEOS_INVALID_ARG;
  if (n == 0) return MDEOS_OK;
  std::lock_guard<std::recursive_mutex> lk(c->mu);
  return c->eval(n, specs, sched, out, c->pick(stream), false);
}

extern "C" mdeos_status mdeos_eval_batch_noalloc(mdeos_ctx* ctx, int n, const mdeos_cell_spec* specs,
                                                 const mdeos_schedule* sched, mdeos_result* out, void* stream) {
  CTX_GUARD(C_(ctx));
  Ctx* c = C_(ctx);
  if (n < 0 || (n > 0 && (!specs || !sched || !out))) return MDEOS_INVALID_ARG;
  if (n == 0) return MDEOS_OK;
  std::lock_guard<std::recursive_mutex> lk(c->mu);
  return c->eval_noalloc(n, specs, sched, out, c->pick(stream));
}

extern "C" mdeos_status mdeos_eval_plain(mdeos_ctx* ctx, int n, const mdeos_cell_spec* specs,
                                         const mdeos_schedule* sched, mdeos_result* out, void* stream) {
  CTX_GUARD(C_(ctx));
  Ctx* c = C_(ctx);
  if (n < 0 || (n > 0 && (!specs || !sched || !out))) return MDEOS_INVALID_ARG;
  if (n == 0) return MDEOS_OK;
  std::lock_guard<std::recursive_mutex> lk(c->mu);
  return c->eval(n, specs, sched, out, c->pick(stream), true);
}

extern "C" mdeos_status mdeos_release(mdeos_ctx* ctx, int n, const mdeos_handle* h) {
  CTX_GUARD(C_(ctx));
  Ctx* c = C_(ctx);
  if (n < 0 || (n > 0 && !h)) return MDEOS_INVALID_ARG;
  std::lock_guard<std::recursive_mutex> lk(c->mu);
  HCHECK(hipDeviceSynchronize());
  std::vector<int> idx;
  for (int i = 0; i < n; ++i) {
    int s = c->slot_of(h[i]);
    if (s < 0) return set_error("stale handle"), MDEOS_INVALID_ARG;
    idx.push_back(s);
  }
  c->free_cells(idx);
  return MDEOS_OK;
}

// Copies the selected arena arrays (bit k of which_mask = array k: x, y, z,
// vx, vy, vz, fx, fy, fz, bx, by, bz) of one cell to out[k * N + i] as doubles.
extern "C" mdeos_status mdeos_last_advance_time(mdeos_ctx* ctx, double* ms, int* n_launches) {
  CTX_GUARD(C_(ctx));
  Ctx* c = C_(ctx);
  std::lock_guard<std::recursive_mutex> lk(c->mu);
  if (c->timed_launches == 0) return set_error("no advance launch yet"), MDEOS_NOT_READY;
  HCHECK(hipEventSynchronize(c->ev_t1));
  float f = 0.f;
  HCHECK(hipEventElapsedTime(&f, c->ev_t0, c->ev_t1));
  if (ms) *ms = f;
  if (n_launches) *n_launches = c->timed_launches;
  return MDEOS_OK;
}

mdeos_status Ctx::download_atoms(int slot, int which_mask, std::vector<double>& out, hipStream_t s) {
  const CellRec& r = h_cells[slot];
  const int N = r.N;
  out.assign((size_t)12 * N, 0.0);
  std::vector<float> tmpf((size_t)6 * N);
  for (int k = 0; k < 12; ++k) {
    if (!(which_mask & (1 << k))) continue;
    if (k < 6) {
      const double* src = (const double*)arena_ptrs[k] + r.atom_off;
      HCHECK(hipMemcpyAsync(out.data() + (size_t)k * N, src, sizeof(double) * N, hipMemcpyDeviceToHost, s));
    } else {
      const float* src = (const float*)arena_ptrs[k] + r.atom_off;
      HCHECK(hipMemcpyAsync(tmpf.data() + (size_t)(k - 6) * N, src, sizeof(float) * N, hipMemcpyDeviceToHost, s));
    }
  }
  HCHECK(hipStreamSynchronize(s));
  for (int k = 6; k < 12; ++k)
    if (which_mask & (1 << k))
      for (int i = 0; i < N; ++i) out[(size_t)k * N + i] = tmpf[(size_t)(k - 6) * N + i];
  return MDEOS_OK;
}

mdeos_status Ctx::download_record(int slot, CellRec& out, hipStream_t s) {
  HCHECK(hipMemcpyAsync(&out, d_cells + slot, sizeof(CellRec), hipMemcpyDeviceToHost, s));
  HCHECK(hipStreamSynchronize(s));
  return MDEOS_OK;
}

extern "C" mdeos_status mdeos_state_export(mdeos_ctx* ctx, mdeos_handle h, double* xyz, double* v, int* step) {
  CTX_GUARD(C_(ctx));
  Ctx* c = C_(ctx);
  std::lock_guard<std::recursive_mutex> lk(c->mu);
  int slot = c->slot_of(h);
  if (slot < 0) return set_error("stale handle"), MDEOS_INVALID_ARG;
  hipStream_t s = c->own_stream;
  HCHECK(hipDeviceSynchronize());
  std::vector<double> a;
  mdeos_status st = c->download_atoms(slot, 0x3f, a, s);
  if (st != MDEOS_OK) return st;
  CellRec r;
  st = c->download_record(slot, r, s);
  if (st != MDEOS_OK) return st;
  const int N = r.N;
  const double L = r.Lw;
  for (int i = 0; i < N; ++i)
    for (int k = 0; k < 3; ++k) {
      if (xyz) {
        double q = a[(size_t)k * N + i];
        q -= L * std::floor(q / L);
        if (q >= L || q < 0.0) q = 0.0;
        xyz[3 * i + k] = q;
      }
      if (v) v[3 * i + k] = a[(size_t)(3 + k) * N + i];
    }
  if (step) *step = r.step;
  return MDEOS_OK;
}

extern "C" mdeos_status mdeos_debug_forces(mdeos_ctx* ctx, const mdeos_cell_spec* spec, const double* xyz, double* F,
                                           double* U, double* W) {
  CTX_GUARD(C_(ctx));
  Ctx* c = C_(ctx);
  if (!spec || !xyz) return MDEOS_INVALID_ARG;
  std::lock_guard<std::recursive_mutex> lk(c->mu);
  hipStream_t s = c->own_stream;
  mdeos_schedule q{};
  q.n_steps = 2;
  q.n_avg = 2;
  q.n_blocks = 2;
  q.energy_every = 1;
  q.drift_tol = 1.0;
  std::vector<int> idx;
  mdeos_status st = c->alloc_cells(1, spec, q, idx);
  if (st != MDEOS_OK) return st;
  const int slot = idx[0];
  const int N = c->h_cells[slot].N;
  c->h_cells[slot].phase = PH_FORCES;
  std::vector<double> zero((size_t)3 * N, 0.0);
  st = c->upload_state(slot, xyz, zero.data(), s);
  if (st == MDEOS_OK) st = c->upload_records(idx, s);
  if (st == MDEOS_OK) {
    std::vector<Bucket> b;
    c->make_buckets(idx, b, -1);
    st = c->run_buckets(b, -1, s, false);
  }
  CellRec r;
  std::vector<double> a;
  if (st == MDEOS_OK) st = c->download_record(slot, r, s);
  if (st == MDEOS_OK && F) st = c->download_atoms(slot, 0x1c0, a, s);
  if (st == MDEOS_OK) {
    if (r.status & ST_OVERFLOW) {
      set_error("neighbour capacity overflow");
      st = MDEOS_DEVICE_ERROR;
    } else {
      if (U) *U = r.U;
      if (W) *W = r.W;
      if (F)
        for (int i = 0; i < N; ++i)
          for (int k = 0; k < 3; ++k) F[3 * i + k] = a[(size_t)(6 + k) * N + i];
    }
  }
  c->free_cells(idx);
  return st;
}

extern "C" mdeos_status mdeos_debug_trajectory(mdeos_ctx* ctx, mdeos_handle h, int n_steps, double* F, double* K,
                                               double* U, double* W) {
  CTX_GUARD(C_(ctx));
  Ctx* c = C_(ctx);
  if (n_steps < 0) return MDEOS_INVALID_ARG;
  std::lock_guard<std::recursive_mutex> lk(c->mu);
  int slot = c->slot_of(h);
  if (slot < 0) return set_error("stale handle"), MDEOS_INVALID_ARG;
  hipStream_t s = c->own_stream;
  HCHECK(hipDeviceSynchronize());
  const int one = 1;
  HCHECK(hipMemcpy(&c->d_cells[slot].debug_energy, &one, sizeof(int), hipMemcpyHostToDevice));
  c->h_cells[slot].debug_energy = 1;
  std::vector<int> idx{slot};
  auto record = [&](int k) -> mdeos_status {
    CellRec r;
    mdeos_status st = c->download_record(slot, r, s);
    if (st != MDEOS_OK) return st;
    const int N = r.N;
    if (K) K[k] = r.K;
    if (U) U[k] = r.U;
    if (W) W[k] = r.W;
    if (F) {
      std::vector<double> a;
      st = c->download_atoms(slot, 0x1c0, a, s);
      if (st != MDEOS_OK) return st;
      for (int i = 0; i < N; ++i)
        for (int q = 0; q < 3; ++q) F[((size_t)k * N + i) * 3 + q] = a[(size_t)(6 + q) * N + i];
    }
    return MDEOS_OK;
  };
  // a cell whose lift or warm start is still pending (a warm start only marks
  // the cell) runs that phase first, so that step 0 is the re-targeted state
  CellRec r0;
  mdeos_status st = c->download_record(slot, r0, s);
  if (st == MDEOS_OK && (r0.phase == PH_COLD || r0.phase == PH_STATE || r0.phase == PH_WARM)) {
    std::vector<Bucket> b;
    c->make_buckets(idx, b, -1);
    st = c->run_buckets(b, -1, s, false);
  }
  if (st == MDEOS_OK) st = record(0);
  for (int k = 1; k <= n_steps && st == MDEOS_OK; ++k) {
    std::vector<Bucket> b;
    c->make_buckets(idx, b, 1);
    st = c->run_buckets(b, 1, s, false);
    if (st == MDEOS_OK) st = record(k);
  }
  const int zero = 0;
  hipMemcpy(&c->d_cells[slot].debug_energy, &zero, sizeof(int), hipMemcpyHostToDevice);
  c->h_cells[slot].debug_energy = 0;
  return st;
}
