// Internal layout shared by the host library and the gfx950 kernels of
// libmdeos: the device-resident cell record, the launch parameters of the
// persistent advance kernel and the LDS layout of one box.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mdeos {

constexpr int kMaxRescale = 8;
constexpr int kMaxBlocks = 16;
constexpr float kSentinelPos = 1.0e15f;  // position of the padding neighbour

// Phase of a resident cell: what the next advance launch does first.
enum Phase : int {
  PH_COLD = 0,    // lattice, E_cold, velocity draw and pin (lifting operator)
  PH_STATE = 1,   // E_cold from the lattice, then the uploaded state
  PH_WARM = 2,    // dilate the resident state to the new density, re-pin
  PH_RUN = 3,     // continue from the stored state
  PH_FORCES = 4,  // debug: forces, E_pot and W of the uploaded positions
  PH_DONE = 5,    // schedule finished
};

enum CellStatus : int {
  ST_NONFINITE = 1,
  ST_BELOW_COLD = 2,
  ST_DRIFT = 4,
  ST_OVERFLOW = 8,
  ST_COLD_RELIFT = 16,
};

// One resident cell. Host writes the query part; kernels own the rest.
struct alignas(16) CellRec {
  // query
  double rho, e;       // density, energy per atom above E_cold
  double Lw, V;        // box edge and volume in FP64
  double drift_tol;
  double warm_scale;   // L_new / L_old of a pending warm start
  unsigned long long seed;
  long long cell_id;
  double dt;            // time step (FP64 integration)
  float L, rc, rl;      // FP32 geometry; rl = rc + skin
  int n_c, N;
  int n_steps, n_avg, n_blocks, n_rescale;
  int rescale_steps[kMaxRescale];
  int energy_every;
  int atom_off;        // offset of this cell's atoms in the SoA arena
  int nce;             // binning cells per edge of the extended box
  int stencil;         // binning stencil half-width (cells of edge >= rl / stencil)
  int phase;
  int step;            // steps completed
  int status;
  int debug_energy;    // 1: compute E_pot every step
  int n_builds;        // neighbour-list builds so far
  int max_list;        // largest neighbour count seen
  int max_ext;         // largest real + ghost count seen
  // accumulators (FP64)
  double Ecold;        // total cold energy
  double sumP[kMaxBlocks], sumT[kMaxBlocks];
  double P_ref, sumdP2, sumU;
  int nU, pad0;
  double E_w0, E_n;
  double K, U, W;      // values of the last completed step
  double pair_sum;     // ordered in-range pairs summed over sampled (energy) steps
  int pair_steps;      // number of sampled steps
  int ensemble;        // MDEOS_NVE_REPIN or MDEOS_NVT_LANGEVIN
  double gamma;        // Langevin friction
  double T_th;         // thermostat temperature (Langevin)
  double segU;         // E_pot summed over the current temperature-update window
  int segN, seg_prev;  // its sample count; the previous update step
  int query;           // queries of this cell before this one (warm starts); thermostat noise stream
  int nS;              // sampled steps in the stress sums
  double sigK[6], sigV[6];  // kinetic (sum v_a v_b) and virial (sum d_a f_b) tensors summed over them
};

// Result in the layout of mdeos_result.
struct DevResult {
  double P, P_se, P_rms, T, T_se, Epot_mean, Ecold, drift;
  double pairs;
  int n_samples, status, n_builds, max_list, max_ext, pad;
  double stress[6];
};

// Structure-of-arrays atom state in device memory; each array has `cap` entries.
struct AtomArena {
  double *x, *y, *z;     // positions (unwrapped since the last list build)
  double *vx, *vy, *vz;  // velocities
  float *fx, *fy, *fz;  // forces of the last step
  float *bx, *by, *bz;  // positions at the last list build (wrapped)
};

// Launch-wide capacities of one bucket (all cells of a launch share them).
struct Caps {
  int n_pad;      // max atoms per cell rounded up to 64
  int list_cap;   // neighbours per atom (multiple of 8)
  int ncell_cap;  // binning cells
  int ring;       // steps buffered before the FP64 bookkeeping runs
  int gmax;       // groups of 64 atoms per cell (n_pad / 64)
};

struct AdvanceParams {
  CellRec* cells;
  const int* work_base;  // cell indices of every bucket, longest first
  const int* meta;       // this bucket's {number of cells, offset into work_base}
  int* counter;          // work counter (zeroed before the launch)
  int step_budget;      // steps per cell in this launch: 0 = to the end, < 0 = none (lift only)
  AtomArena a;
  uint16_t* gl_list;    // device-memory neighbour lists (per workgroup), or null
  uint16_t* gl_ilist;   // device-memory inner (pruned) lists, same shape as gl_list, or null: no pruning
  float prune_skin;     // the inner lists hold the entries within rc + prune_skin
  Caps caps;
  int kahan;            // 1: Kahan-compensated FP32 per-atom energy/virial sums, 0: FP64
  double eam_c;         // embedding strength of the embedded-atom variants
};

// LDS layout of one box. EXT is the stride of each position array (compile
// time), so the three coordinates of neighbour j sit at byte offsets
// 4 j, 4 (j + EXT) and 4 (j + 2 EXT) and one VGPR address serves all three
// loads.
struct LdsLayout {
  int pos;        // float[3][EXT] (uint32[3][EXT] fixed point for minimum image)
  int list;       // uint16[list_cap/8][n_pad][8] (when the list lives in LDS)
  int tmp;        // uint16[EXT]   (the ghost-count scan uses tmp..sorted as int[N]; outside the
                  //                list build the embedded-atom forces keep F'(rhobar) there as float[EXT])
  int sorted;     // uint16[EXT]
  int cstart;     // int[ncell_cap + 1]
  int cfill;      // int[ncell_cap]
  int ring;       // double[ring][gmax][3]
  int red;        // double[gmax][6] (per-group sums of up to six values)
  int ctl;        // control block (int/float/double scalars)
  int frc;        // float[3][frc_slots]: forces of the shapes that keep them in LDS
  int total;
};

__host__ __device__ inline int align_up(int v, int a) { return (v + a - 1) / a * a; }

__host__ __device__ inline LdsLayout lds_layout(int ext, const Caps& c, bool list_in_lds, int frc_slots = 0) {
  LdsLayout l;
  int o = 0;
  l.pos = o; o += 12 * ext;
  l.list = o; o += list_in_lds ? 2 * c.list_cap * c.n_pad : 0;
  o = align_up(o, 16);
  l.tmp = o; o += 2 * ext;
  l.sorted = o; o += 2 * ext;
  o = align_up(o, 16);
  l.cstart = o; o += 4 * (c.ncell_cap + 1);
  l.cfill = o; o += 4 * c.ncell_cap;
  o = align_up(o, 16);
  l.ring = o; o += 8 * 3 * c.gmax * c.ring;
  l.red = o; o += 8 * 6 * c.gmax;
  l.ctl = o; o += 1024;
  l.frc = o; o += 12 * frc_slots;
  l.total = align_up(o, 256);
  return l;
}

// Kernel variants the library is built with (template arguments of the
// advance kernel): threads per box, atoms per thread, position stride, where
// the neighbour list lives, the waves per SIMD the registers must allow, and
// minimum image (no ghosts) for large boxes, Langevin integration, and the
// embedded-atom potential instead of LJTS.
struct Variant {
  int block, apt, ext, list_lds, wpe, mi, nvt, eam;
};
// Whether a launch shape keeps its forces in LDS (the minimum-image shapes
// with four or more atoms per thread, whose per-atom state outgrows the
// registers), and the force slots it then needs.
__host__ __device__ constexpr bool forces_in_lds(bool mi, int apt) { return mi && apt >= 4; }
inline int frc_slots(const Variant& v) { return forces_in_lds(v.mi != 0, v.apt) ? v.block * v.apt : 0; }
inline bool same_variant(const Variant& a, const Variant& b) {
  return a.block == b.block && a.apt == b.apt && a.ext == b.ext && a.list_lds == b.list_lds && a.wpe == b.wpe &&
         a.mi == b.mi && a.nvt == b.nvt && a.eam == b.eam;
}

// Host entry points implemented in kernels.hip.
hipError_t launch_advance(const Variant& v, const AdvanceParams& p, int grid, int lds_bytes, hipStream_t s);
hipError_t launch_restrict(const CellRec* cells, const int* idx, int n, DevResult* out, hipStream_t s);
hipError_t launch_zero_ints(int* p, int n, hipStream_t s);
bool variant_available(const Variant& v);
int variant_count();
Variant variant_at(int i);

}  // namespace mdeos
