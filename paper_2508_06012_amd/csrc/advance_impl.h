// The persistent advance kernel of libmdeos (included by the per-variant
// translation units; each instantiates a few launch shapes).
//
// One workgroup owns one periodic box at a time ("cell" = one continuum
// quadrature point's EOS query, Sec. III) and keeps it resident in LDS for a
// whole chunk of steps:
//   - lifting operator (Sec. III, Eqs. numdens/numAtoms): FCC lattice at rho,
//     cold energy of the static lattice, Gaussian velocities (Philox4x64-10 +
//     Box-Muller) at T0 = 2 N e / N_DOF, zero net momentum, scaled so the
//     energy above the cold lattice is N e;
//   - microscopic model (Sec. II.B): velocity Verlet with a Verlet neighbour
//     list over an LDS-resident extended box (real atoms + periodic ghost
//     images), LJTS pair forces in FP32 with per-atom FP32 partials promoted to
//     FP64 for the energy and virial reductions; or the embedded-atom form of
//     Eq. Etot, a density walk then a force walk over the same lists;
//   - temperature update (Eq. Tcontribution) as an instantaneous energy re-pin
//     at scheduled steps, in FP64;
//   - restricting operator (Eq. stress): P = (2K + W) / (3V), T = 2K / N_DOF,
//     block-averaged in FP64.
// Every reduction runs in a fixed order over groups of 64 consecutive atoms,
// and neighbour lists are built in a deterministic order, so a cell's bits do
// not depend on the launch shape, the batch it runs in, or chunk boundaries.
// Sums of products are written as explicit fma chains: left to the compiler,
// a + b * c + d * e can be fused in more than one way, and the choice may
// differ between the launch shapes' instantiations.
#pragma once
#include <type_traits>

#include "mdeos_dev.h"
#include "mdeos_host.h"

#define DEVI __device__ __attribute__((always_inline)) inline

namespace mdeos {

namespace {

struct Ctl {
  int item;
  int need_rebuild;
  int stop;
  int overflow;
  int n_ext;
  int wsum[17];
  float wmax[16];
  float pmax[16];
  int do_rescale;
  int pad1;
  double lam;
  double scal[4];
  // accumulators of the cell being advanced (wave 0 owns them)
  double sumP[kMaxBlocks], sumT[kMaxBlocks];
  double P_ref, sumdP2, sumU;
  double E_w0, E_n;
  double K, U, W;
  int nU;
  int status;
  // Langevin thermostat: temperature, and the E_pot window of the next
  // temperature update (wave 0 owns them)
  double T_th, segU;
  int segN, seg_prev;
  // stress tensor sums over the sampled window steps (thread 0 owns them)
  double sigK[6], sigV[6];
  int nS;
};

DEVI uint64_t mulhi64(uint64_t a, uint64_t b) { return __umul64hi(a, b); }

// Philox4x64-10 (Salmon et al., SC11): ten rounds, Weyl key schedule.
DEVI void philox4x64_10(uint64_t k0, uint64_t k1, uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                        uint64_t& o0, uint64_t& o1, uint64_t& o2, uint64_t& o3) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
  const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    uint64_t lo0 = M0 * c0, hi0 = mulhi64(M0, c0);
    uint64_t lo1 = M1 * c2, hi1 = mulhi64(M1, c2);
    uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
    k0 += W0; k1 += W1;
  }
  o0 = c0; o1 = c1; o2 = c2; o3 = c3;
}

// Standard normal of (atom a, component c): Box-Muller on Philox words 0, 1
// with key (seed, cell_id) and counter (3a + c, 0, 0, 0).
DEVI double gauss(uint64_t seed, int64_t cell_id, int a, int c) {
  uint64_t w0, w1, w2, w3;
  philox4x64_10(seed, (uint64_t)cell_id, (uint64_t)(3 * a + c), 0, 0, 0, w0, w1, w2, w3);
  const double two_m53 = 1.0 / 9007199254740992.0;
  double u1 = 1.0 - (double)(w0 >> 11) * two_m53;
  double u2 = (double)(w1 >> 11) * two_m53;
  return sqrt(-2.0 * log(u1)) * cos(2.0 * M_PI * u2);
}

// Thermostat noise of atom a at step k of query q: one Philox block with key
// (seed, cell_id) at counter (a, k, 1, q); Box-Muller (cos, sin) on words 0-1
// and cos on words 2-3. The uniforms are those of the definition; the
// transform runs in FP32 on the hardware log2 / sin / cos (angles in
// revolutions), which keeps this off the register budget of the step loop
// (the numbers differ from an FP64 transform by about 1e-7 relative).
DEVI void noise3(uint64_t seed, int64_t cell_id, int a, int k, int q, double& z0, double& z1, double& z2) {
  uint64_t w0, w1, w2, w3;
  philox4x64_10(seed, (uint64_t)cell_id, (uint64_t)a, (uint64_t)k, 1, (uint64_t)q, w0, w1, w2, w3);
  const double two_m53 = 1.0 / 9007199254740992.0;
  const float u1 = (float)(1.0 - (double)(w0 >> 11) * two_m53), u2 = (float)((double)(w1 >> 11) * two_m53);
  const float u3 = (float)(1.0 - (double)(w2 >> 11) * two_m53), u4 = (float)((double)(w3 >> 11) * two_m53);
  const float m2ln2 = -1.3862943611198906f;  // -2 ln 2: -2 ln u = -2 ln 2 log2 u
  const float r1 = __builtin_sqrtf(m2ln2 * __builtin_amdgcn_logf(u1));
  const float r2 = __builtin_sqrtf(m2ln2 * __builtin_amdgcn_logf(u3));
  z0 = (double)(r1 * __builtin_amdgcn_cosf(u2));
  z1 = (double)(r1 * __builtin_amdgcn_sinf(u2));
  z2 = (double)(r2 * __builtin_amdgcn_cosf(u4));
}

// Cross-lane moves on the DPP network (no LDS traffic). CTRL codes:
// 0xB1 quad_perm [1,0,3,2] (lane ^ 1), 0x4E quad_perm [2,3,0,1] (lane ^ 2),
// 0x141 row_half_mirror, 0x140 row_mirror.
template <int CTRL>
DEVI int dpp_i(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, false);
}
template <int CTRL>
DEVI double dpp_d(double v) {
  const int lo = dpp_i<CTRL>(__double2loint(v)), hi = dpp_i<CTRL>(__double2hiint(v));
  return __hiloint2double(hi, lo);
}
DEVI double readlane_d(double v, int lane) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
  return __hiloint2double(hi, lo);
}

// Sum of a double over the 64 lanes in a fixed tree (pairs, quads, eighths,
// rows of 16, then the four rows); every lane gets the same value.
DEVI double wave_sum(double v) {
  v += dpp_d<0xB1>(v);
  v += dpp_d<0x4E>(v);
  v += dpp_d<0x141>(v);
  v += dpp_d<0x140>(v);
  return (readlane_d(v, 0) + readlane_d(v, 16)) + (readlane_d(v, 32) + readlane_d(v, 48));
}
DEVI float wave_max(float v) {
  v = fmaxf(v, __int_as_float(dpp_i<0xB1>(__float_as_int(v))));
  v = fmaxf(v, __int_as_float(dpp_i<0x4E>(__float_as_int(v))));
  v = fmaxf(v, __int_as_float(dpp_i<0x141>(__float_as_int(v))));
  v = fmaxf(v, __int_as_float(dpp_i<0x140>(__float_as_int(v))));
  const float a = fmaxf(__int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 0)),
                        __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 16)));
  const float b = fmaxf(__int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 32)),
                        __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 48)));
  return fmaxf(a, b);
}
DEVI int wave_max_i(int v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
  return v;
}

DEVI double wrap1(double x, double L) {
  // positions move less than L between list builds: one correction suffices
  if (x >= L) x -= L;
  else if (x < 0.0) x += L;
  if (x >= L || x < 0.0) x = 0.0;
  return x;
}

// MI (minimum image): only the real atoms are held in LDS, binning cells
// tile [0, L) periodically and every pair takes its nearest periodic image
// (boxes with L >= 3 rl whose ghost-extended box would not fit in LDS).
// Their LDS positions are 32-bit fixed-point fractions of the box edge
// (unit L / 2^32, about 3e-9 sigma for the largest boxes): the wrapped
// integer difference of two coordinates, read as signed, is the nearest-image
// difference, so a pair costs an integer subtract and a conversion per axis
// instead of an FP64 image correction, and a slot takes 12 bytes.
// What the pair loop sums per atom besides the force.
enum { ACC_F = 0, ACC_FW = 1, ACC_FWU = 2, ACC_FWUS = 3 };

template <int BLOCK, int APT, int EXT, bool LLDS, bool MI, bool NVT, bool EAM>
struct Box {
  static constexpr int NW = BLOCK / 64;
  static constexpr int SENT = EXT - 1;  // padding neighbour index
  using PT = typename std::conditional<MI, uint32_t, float>::type;  // LDS position type
  static constexpr int PB = sizeof(PT);
  // inner lists (device-memory lists of the embedded-atom shapes only: its two
  // walks per step are where they pay; the LJTS shapes carry none of their registers)
  static constexpr bool PRUNE = !LLDS && EAM;
  // Cell-sorted position slots (ghost-image LJTS shapes): a list build places
  // every atom and image at its slot in cell order (cells in index order,
  // each cell's members by extended index), keeps the extended-index -> slot
  // map in `sorted`, and lists name slots. A row of the binning stencil is
  // then a run of consecutive slots, read without an index load. The walk
  // visits the same neighbours in the same order as with positions by
  // extended index, so the bits do not change. (The embedded-atom shapes keep
  // F'(rhobar) where the map would live; minimum-image boxes hold no images.)
  static constexpr bool SORTED = !MI && !EAM;
  // Forces of the minimum-image shapes with four or more atoms per thread
  // live in LDS (float[3][BLOCK * APT]), not in registers: those boxes leave
  // LDS to spare, and their per-atom state otherwise outgrows the registers.
  static constexpr bool FLDS = forces_in_lds(MI, APT);

  const AdvanceParams& p;
  LdsLayout lay;
  unsigned char* lds;
  PT* px;  // py = px + EXT, pz = px + 2 EXT
  uint16_t* list;  // [list_cap/8][n_pad][8]
  // Inner lists (device memory, same shape): the entries of `list` within
  // rc + prune_skin of the positions at the last prune, in list order. The
  // force walks use them while `inner` is set; entries between rc and the
  // list radius only ever add exact zeros, so the walk over either list
  // gives the same bits.
  uint16_t* ilist;
  bool inner;
  uint16_t *tmp, *sorted;
  float* frc;  // forces in LDS (FLDS)
  float* fpv;  // F'(rhobar) per position slot (embedded-atom forces; shares tmp/sorted, live outside list builds)
  int *cstart, *cfill, *scanbuf;
  double *ring, *red;
  Ctl* ctl;
  int t, lane, wv;

  // cell constants
  CellRec* c;
  int N, G, n_pad, list_cap, ncell, nce, R;
  float L, rl, rl2, rc2, inv_ce;
  float sL;  // fixed-point unit of the minimum-image positions, L / 2^32
  float rlc2;  // (rl in cell edges)^2, widened by a relative 1e-4 so clipping stays conservative
  float rin2, pthr;  // inner-list radius^2 (rc + prune_skin)^2; prune trigger (displacement^2)
  bool prune_cell;   // this cell keeps inner lists
  double invLw;
  double Lw, dt, hdt;
  double V, Ndof, u_shift;
  // embedded-atom form in shifted-force truncation: f_s(r) = r^-6 + e_c6 r - e_k6,
  // V_s(r) = r^-9 + e_c9 r - e_k9 (e_c6 = 6 rc^-7, e_k6 = 7 rc^-6, e_c9 = 9 rc^-10,
  // e_k9 = 10 rc^-9), F(rhobar) = -eam_c sqrt(rhobar)
  float e_c6, e_k6, e_c9, e_k9;
  double eam_c;
  double Ecold;  // total cold energy (uniform across the workgroup)
  // the schedule, read once per cell (the step loop writes other fields of
  // the cell record, which would otherwise force these to be re-read)
  int n_steps, n_avg, n_blocks, energy_every, debug_energy, n_rescale;
  int rescale_at[MDEOS_MAX_RESCALE];
  // Langevin (GJF) in half-step form: c = gamma dt / 2, b = 1 / (1 + c),
  // a = (1 - c) / (1 + c); u = sqrt(b) (v + dt f / 2 + beta / 2),
  // x += sqrt(b) dt u, v = (a / sqrt(b)) u + dt f' / 2 + beta / 2, which is
  // the two-line GJF step since (a + 1) / 2 = b
  static constexpr bool nvt = NVT;  // Langevin (GJF) integration; else velocity Verlet
  double gjf_sb, gjf_a_sb, gamma_dt2;
  int query;
  uint64_t seed;
  int64_t cell_id;
  bool kahan;    // per-atom energy/virial sums in compensated FP32 (uniform)

  // owned atoms: a = t + k BLOCK
  // state in FP64 (positions unwrapped since the last list build), forces and
  // build positions in FP32
  double x[APT], y[APT], z[APT], vx[APT], vy[APT], vz[APT];
  float fx[APT], fy[APT], fz[APT], bx[APT], by[APT], bz[APT];
  int gofs[APT], gmask[APT], nblk[APT];
  int sslot[APT];  // slot of each owned atom (SORTED)
  int fnb[APT];                      // blocks of the list the force walks use (wave-uniform)
  float prx[APT], pry[APT], prz[APT];  // positions at the last prune
  double pairs_t;  // ordered in-range pairs of this thread's atoms over sampled steps
  int esteps;      // sampled (energy) steps in this launch

  DEVI Box(const AdvanceParams& pp, unsigned char* l) : p(pp), lds(l) {
    lay = lds_layout(EXT, p.caps, LLDS, FLDS ? BLOCK * APT : 0);
    px = (PT*)(lds + lay.pos);
    list = LLDS ? (uint16_t*)(lds + lay.list)
                : p.gl_list + (size_t)blockIdx.x * (size_t)p.caps.list_cap * (size_t)p.caps.n_pad;
    ilist = (!PRUNE || p.gl_ilist == nullptr || p.kahan != 0)
                ? nullptr
                : p.gl_ilist + (size_t)blockIdx.x * (size_t)p.caps.list_cap * (size_t)p.caps.n_pad;
    inner = false;
    tmp = (uint16_t*)(lds + lay.tmp);
    sorted = (uint16_t*)(lds + lay.sorted);
    cstart = (int*)(lds + lay.cstart);
    cfill = (int*)(lds + lay.cfill);
    scanbuf = (int*)(lds + lay.tmp);
    fpv = (float*)(lds + lay.tmp);
    frc = (float*)(lds + lay.frc);
    ring = (double*)(lds + lay.ring);
    red = (double*)(lds + lay.red);
    ctl = (Ctl*)(lds + lay.ctl);
    t = threadIdx.x;
    lane = t & 63;
    wv = t >> 6;
    n_pad = p.caps.n_pad;
    list_cap = p.caps.list_cap;
    kahan = p.kahan != 0;
  }

  // force components of owned atom k
  DEVI float& FX(int k) {
    if constexpr (FLDS) return frc[t + k * BLOCK];
    else return fx[k];
  }
  DEVI float& FY(int k) {
    if constexpr (FLDS) return frc[BLOCK * APT + t + k * BLOCK];
    else return fy[k];
  }
  DEVI float& FZ(int k) {
    if constexpr (FLDS) return frc[2 * BLOCK * APT + t + k * BLOCK];
    else return fz[k];
  }
  DEVI PT& PX(int j) { return px[j]; }
  DEVI PT& PY(int j) { return px[EXT + j]; }
  DEVI PT& PZ(int j) { return px[2 * EXT + j]; }
  // LDS form of a coordinate: FP32, or (MI) the fixed-point fraction of L of
  // the wrapped coordinate, floor(2^32 frac(v / L)) (clamped below 2^32)
  DEVI PT to_pt(double v) const {
    if constexpr (MI) {
      const double u = v * invLw;
      return (uint32_t)fmin((u - floor(u)) * 4294967296.0, 4294967295.0);
    } else {
      return (float)v;
    }
  }
  // a_i - a_j of two LDS coordinates as FP32 (MI: the nearest image)
  DEVI float pdiff(PT a, PT b) const {
    if constexpr (MI)
      return (float)(int32_t)(a - b) * sL;
    else
      return a - b;
  }
  // FP32 coordinate of an LDS position (MI: in [0, L))
  DEVI float pcoord(PT v) const {
    if constexpr (MI)
      return (float)v * sL;
    else
      return v;
  }

  DEVI void load_cell(int cidx) {
    c = p.cells + cidx;
    N = c->N;
    G = (N + 63) / 64;
    L = c->L;
    rl = c->rl;
    rl2 = rl * rl;
    rc2 = c->rc * c->rc;
    dt = c->dt;
    hdt = 0.5 * dt;
    Lw = c->Lw;
    nce = c->nce;
    R = c->stencil;
    ncell = nce * nce * nce;
    inv_ce = MI ? (float)nce / L : (float)nce / (L + 2.0f * rl);
    {
      const float rlc = rl * inv_ce * 1.0001f;
      rlc2 = rlc * rlc;
    }
    {
      // Inner lists pay off only inside the skin. A pair dropped at a prune
      // (r >= rc + ps) reaches rc only after the two atoms moved ps apart, so
      // a prune follows as soon as any atom has moved ps / 2; the trigger sits
      // 1 % below that, far above the FP32 rounding of the distances.
      const float rcf = c->rc, ps = p.prune_skin;
      prune_cell = ilist != nullptr && ps > 0.f && rl - rcf > ps;
      rin2 = (rcf + ps) * (rcf + ps);
      pthr = 0.98f * 0.25f * ps * ps;
    }
    invLw = 1.0 / c->Lw;
    sL = (float)(c->Lw * 0x1p-32);
    V = c->V;
    Ndof = 3.0 * N - 3.0;
    double irc2 = 1.0 / ((double)c->rc * (double)c->rc);
    double irc6 = irc2 * irc2 * irc2;
    u_shift = 4.0 * fma(irc6, irc6, -irc6);
    if (EAM) {
      const double rcd = c->rc, irc = 1.0 / rcd;
      e_c6 = (float)(6.0 * irc6 * irc);
      e_k6 = (float)(7.0 * irc6);
      e_c9 = (float)(9.0 * irc6 * irc2 * irc2);
      e_k9 = (float)(10.0 * irc6 * irc2 * irc);
      eam_c = p.eam_c;
    }
    Ecold = c->Ecold;
    n_steps = c->n_steps;
    n_avg = c->n_avg;
    n_blocks = c->n_blocks;
    energy_every = c->energy_every;
    debug_energy = c->debug_energy;
    n_rescale = c->n_rescale;
#pragma unroll
    for (int r = 0; r < MDEOS_MAX_RESCALE; ++r) rescale_at[r] = r < n_rescale ? c->rescale_steps[r] : -1;
    seed = c->seed;
    cell_id = c->cell_id;
    {
      const double hg = 0.5 * c->gamma;
      const double b = 1.0 / fma(hg, dt, 1.0), a = fma(-hg, dt, 1.0) / fma(hg, dt, 1.0);
      gjf_sb = sqrt(b);
      gjf_a_sb = a / gjf_sb;
      gamma_dt2 = 2.0 * c->gamma * dt;
    }
    query = c->query;
  }
  // first scheduled step >= k, or -1
  DEVI int next_update(int k) const {
    int best = -1;
#pragma unroll
    for (int r = 0; r < MDEOS_MAX_RESCALE; ++r)
      if (rescale_at[r] >= k && (best < 0 || rescale_at[r] < best)) best = rescale_at[r];
    return best;
  }

  // --- block helpers --------------------------------------------------------

  // In-place exclusive scan of arr[0..n) (LDS); returns the total.
  DEVI int block_scan(int* arr, int n) {
    const int per = (n + BLOCK - 1) / BLOCK;
    const int lo = min(t * per, n), hi = min(lo + per, n);
    int s = 0;
    for (int i = lo; i < hi; ++i) s += arr[i];
    int inc = s;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      int v = __shfl_up(inc, o, 64);
      if (lane >= o) inc += v;
    }
    if (lane == 63) ctl->wsum[wv] = inc;
    __syncthreads();
    if (t == 0) {
      int acc = 0;
      for (int w = 0; w < NW; ++w) {
        int v = ctl->wsum[w];
        ctl->wsum[w] = acc;
        acc += v;
      }
      ctl->wsum[NW] = acc;
    }
    __syncthreads();
    int run = ctl->wsum[wv] + inc - s;
    for (int i = lo; i < hi; ++i) {
      int v = arr[i];
      arr[i] = run;
      run += v;
    }
    int total = ctl->wsum[NW];
    __syncthreads();
    return total;
  }

  // Per-group (64 consecutive atoms) FP64 sums of three per-atom values into
  // dst[g][0..2]; each wave writes its own groups.
  DEVI void group_sums(const double (&a)[APT], const double (&b)[APT], const double (&cc)[APT], double* dst) {
#pragma unroll
    for (int k = 0; k < APT; ++k) {
      double sa = wave_sum(a[k]), sb = wave_sum(b[k]), sc = wave_sum(cc[k]);
      int g = k * NW + wv;
      if (lane == 0 && g < p.caps.gmax) {
        dst[3 * g + 0] = sa;
        dst[3 * g + 1] = sb;
        dst[3 * g + 2] = sc;
      }
    }
  }

  // Per-group FP64 sums of one per-atom value into dst[3 g] (the K slot of a
  // ring entry); each wave writes its own groups.
  DEVI void group_sums1(const double (&a)[APT], double* dst) {
#pragma unroll
    for (int k = 0; k < APT; ++k) {
      const double sa = wave_sum(a[k]);
      const int g = k * NW + wv;
      if (lane == 0 && g < p.caps.gmax) dst[3 * g] = sa;
    }
  }

  // Block-wide FP64 sums of three per-atom values, summed over groups in
  // index order; the result is visible to every thread.
  DEVI void reduce_now(const double (&a)[APT], const double (&b)[APT], const double (&cc)[APT], double& A,
                             double& B, double& C) {
    group_sums(a, b, cc, red);
    __syncthreads();
    if (t == 0) {
      double s0 = 0.0, s1 = 0.0, s2 = 0.0;
      for (int g = 0; g < G; ++g) {
        s0 += red[3 * g + 0];
        s1 += red[3 * g + 1];
        s2 += red[3 * g + 2];
      }
      ctl->scal[0] = s0;
      ctl->scal[1] = s1;
      ctl->scal[2] = s2;
    }
    __syncthreads();
    A = ctl->scal[0];
    B = ctl->scal[1];
    C = ctl->scal[2];
    __syncthreads();
  }

  // Adds the block sums of six per-atom values (groups summed in index order,
  // FP64) to acc6 (thread 0).
  DEVI void tensor_add(const double (&a)[6][APT], double* acc6) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      group_sums(a[3 * h], a[3 * h + 1], a[3 * h + 2], red);
      __syncthreads();
      if (t == 0) {
        double s0 = 0.0, s1 = 0.0, s2 = 0.0;
        for (int g = 0; g < G; ++g) {
          s0 += red[3 * g + 0];
          s1 += red[3 * g + 1];
          s2 += red[3 * g + 2];
        }
        acc6[3 * h + 0] += s0;
        acc6[3 * h + 1] += s1;
        acc6[3 * h + 2] += s2;
      }
      __syncthreads();
    }
  }

  DEVI bool valid(int k) const { return t + k * BLOCK < N; }

  // --- neighbour structures -------------------------------------------------

  DEVI int ghost_mask(float xx, float yy, float zz) const {
    int m = 0;
    m |= (xx < rl) ? 1 : 0;
    m |= (xx >= L - rl) ? 2 : 0;
    m |= (yy < rl) ? 4 : 0;
    m |= (yy >= L - rl) ? 8 : 0;
    m |= (zz < rl) ? 16 : 0;
    m |= (zz >= L - rl) ? 32 : 0;
    return m;
  }
  DEVI static int n_images(int m) {
    int nx = 1 + (m & 1) + ((m >> 1) & 1);
    int ny = 1 + ((m >> 2) & 1) + ((m >> 3) & 1);
    int nz = 1 + ((m >> 4) & 1) + ((m >> 5) & 1);
    return nx * ny * nz - 1;
  }

  // Writes the periodic images of one atom at (xx, yy, zz) starting at ghost
  // slot g, in the fixed order sx, sy, sz in {-1, 0, 1} (lexicographic). An
  // image with shift +1 exists when the coordinate is below rl, -1 when it is
  // at least L - rl: exactly the images that fall in [-rl, L + rl).
  DEVI void write_images(double xx, double yy, double zz, int m, int g) {
    // allowed shifts of each axis in ascending order: -1 (if any), 0, +1 (if any)
    const int nfx = (m >> 1) & 1, nfy = (m >> 3) & 1, nfz = (m >> 5) & 1;
    const int nx = 1 + (m & 1) + nfx, ny = 1 + ((m >> 2) & 1) + nfy, nz = 1 + ((m >> 4) & 1) + nfz;
#pragma unroll 1
    for (int ix = 0; ix < nx; ++ix) {
      const int sx = ix - nfx;
      const float X = (float)(xx + sx * Lw);
#pragma unroll 1
      for (int iy = 0; iy < ny; ++iy) {
        const int sy = iy - nfy;
        const float Y = (float)(yy + sy * Lw);
#pragma unroll 1
        for (int iz = 0; iz < nz; ++iz) {
          const int sz = iz - nfz;
          if ((sx | sy | sz) == 0) continue;
          PX(g) = X;
          PY(g) = Y;
          PZ(g) = (float)(zz + sz * Lw);
          ++g;
        }
      }
    }
  }

  // Calls fn(X, Y, Z, i) for the periodic images of one atom in the order
  // write_images stores them (i = 0, 1, ...), with the same FP32 coordinates.
  template <class FN>
  DEVI void for_images(double xx, double yy, double zz, int m, FN&& fn) const {
    const int nfx = (m >> 1) & 1, nfy = (m >> 3) & 1, nfz = (m >> 5) & 1;
    const int nx = 1 + (m & 1) + nfx, ny = 1 + ((m >> 2) & 1) + nfy, nz = 1 + ((m >> 4) & 1) + nfz;
    int i = 0;
#pragma unroll 1
    for (int ix = 0; ix < nx; ++ix) {
      const int sx = ix - nfx;
      const float X = (float)(xx + sx * Lw);
#pragma unroll 1
      for (int iy = 0; iy < ny; ++iy) {
        const int sy = iy - nfy;
        const float Y = (float)(yy + sy * Lw);
#pragma unroll 1
        for (int iz = 0; iz < nz; ++iz) {
          const int sz = iz - nfz;
          if ((sx | sy | sz) == 0) continue;
          fn(X, Y, (float)(zz + sz * Lw), i);
          ++i;
        }
      }
    }
  }
  // Current images of one atom into their sorted slots (SORTED).
  DEVI void write_images_sorted(double xx, double yy, double zz, int m, int g) {
    for_images(xx, yy, zz, m, [&](float X, float Y, float Z, int i) __attribute__((always_inline)) {
      const int sl = sorted[g + i];
      PX(sl) = X;
      PY(sl) = Y;
      PZ(sl) = Z;
    });
  }

  // F'(rhobar) of one atom into its ghost slots g .. g + n_images(m) - 1
  // (the slots write_images fills for the same mask).
  DEVI void write_image_vals(float v, int m, int g) {
    const int n = n_images(m);
#pragma unroll 1
    for (int i = 0; i < n; ++i) fpv[g + i] = v;
  }

  // Binning cell of a coordinate, clamped to the grid. Written so that no
  // value, NaN and infinities included, reaches a float-to-int conversion
  // out of its range: NaN and negative values land in cell 0.
  DEVI int cell_coord(float v) const {
    const float u = (MI ? v : v + rl) * inv_ce;
    return u >= 1.0f ? min((int)fminf(u, (float)nce), nce - 1) : 0;
  }
  DEVI int wrapc(int q) const { return q < 0 ? q + nce : (q >= nce ? q - nce : q); }
  DEVI int cell_xyz(float X, float Y, float Z) const {
    return (cell_coord(Z) * nce + cell_coord(Y)) * nce + cell_coord(X);
  }
  DEVI int cell_of(int e) { return cell_xyz(pcoord(PX(e)), pcoord(PY(e)), pcoord(PZ(e))); }

  // Builds ghosts, the binning and every atom's neighbour list from the
  // build positions (bx, by, bz). Returns false on a capacity overflow.
  DEVI bool build_lists() {
    // real atoms at their build positions; ghost counts
#pragma unroll
    for (int k = 0; k < APT; ++k) {
      int a = t + k * BLOCK;
      gmask[k] = 0;
      if (a < N) {
        if (!SORTED) {
          PX(a) = to_pt(bx[k]);
          PY(a) = to_pt(by[k]);
          PZ(a) = to_pt(bz[k]);
        }
        if (!MI) {
          gmask[k] = ghost_mask(bx[k], by[k], bz[k]);
          scanbuf[a] = n_images(gmask[k]);
        }
      }
    }
    __syncthreads();
    int n_ghost = MI ? 0 : block_scan(scanbuf, N);
    int n_ext = N + n_ghost;
    if (n_ext > SENT || ncell > p.caps.ncell_cap) {
      if (t == 0) atomicMax(&c->max_ext, n_ext);
      return false;
    }
    if constexpr (SORTED) {
      // Every atom and its images, enumerated by their owner: cell counts,
      // placement, then the rank inside the cell by extended index, which
      // gives the slot; the position goes there and the slot into `sorted`.
      // (scanbuf, read here, shares tmp..sorted: both are written only after
      // the barriers below.)
#pragma unroll
      for (int k = 0; k < APT; ++k) {
        const int a = t + k * BLOCK;
        sslot[k] = SENT;
        if (a < N) gofs[k] = N + scanbuf[a];
      }
      for (int q = t; q < ncell; q += BLOCK) {
        cstart[q] = 0;
        cfill[q] = 0;
      }
      if (t == 0) cstart[ncell] = 0;
      __syncthreads();
#pragma unroll
      for (int k = 0; k < APT; ++k) {
        if (!valid(k)) continue;
        atomicAdd(&cstart[cell_xyz(bx[k], by[k], bz[k])], 1);
        if (gmask[k])
          for_images((double)bx[k], (double)by[k], (double)bz[k], gmask[k],
                     [&](float X, float Y, float Z, int) __attribute__((always_inline)) {
                       atomicAdd(&cstart[cell_xyz(X, Y, Z)], 1);
                     });
      }
      __syncthreads();
      block_scan(cstart, ncell + 1);
#pragma unroll
      for (int k = 0; k < APT; ++k) {
        if (!valid(k)) continue;
        const int a = t + k * BLOCK;
        auto place = [&](float X, float Y, float Z, int e) __attribute__((always_inline)) {
          const int cq = cell_xyz(X, Y, Z);
          tmp[cstart[cq] + atomicAdd(&cfill[cq], 1)] = (uint16_t)e;
        };
        place(bx[k], by[k], bz[k], a);
        if (gmask[k])
          for_images((double)bx[k], (double)by[k], (double)bz[k], gmask[k],
                     [&](float X, float Y, float Z, int i) __attribute__((always_inline)) {
                       place(X, Y, Z, gofs[k] + i);
                     });
      }
      __syncthreads();
#pragma unroll
      for (int k = 0; k < APT; ++k) {
        if (!valid(k)) continue;
        const int a = t + k * BLOCK;
        auto settle = [&](float X, float Y, float Z, int e) __attribute__((always_inline)) {
          const int cq = cell_xyz(X, Y, Z);
          const int lo = cstart[cq], hi = cstart[cq + 1];
          int r = 0;
          for (int q = lo; q < hi; ++q) r += (tmp[q] < e) ? 1 : 0;
          PX(lo + r) = X;
          PY(lo + r) = Y;
          PZ(lo + r) = Z;
          sorted[e] = (uint16_t)(lo + r);
          return lo + r;
        };
        sslot[k] = settle(bx[k], by[k], bz[k], a);
        if (gmask[k])
          for_images((double)bx[k], (double)by[k], (double)bz[k], gmask[k],
                     [&](float X, float Y, float Z, int i) __attribute__((always_inline)) {
                       settle(X, Y, Z, gofs[k] + i);
                     });
      }
      __syncthreads();
    } else {
#pragma unroll
      for (int k = 0; k < APT; ++k) {
        int a = t + k * BLOCK;
        if (a < N && !MI) {
          gofs[k] = N + scanbuf[a];
          write_images((double)bx[k], (double)by[k], (double)bz[k], gmask[k], gofs[k]);
        }
      }
      for (int q = t; q < ncell; q += BLOCK) {
        cstart[q] = 0;
        cfill[q] = 0;
      }
      if (t == 0) cstart[ncell] = 0;
      __syncthreads();
      // bin every extended atom
      for (int e = t; e < n_ext; e += BLOCK) atomicAdd(&cstart[cell_of(e)], 1);
      __syncthreads();
      block_scan(cstart, ncell + 1);
      for (int e = t; e < n_ext; e += BLOCK) {
        int cq = cell_of(e);
        int s = atomicAdd(&cfill[cq], 1);
        tmp[cstart[cq] + s] = (uint16_t)e;
      }
      __syncthreads();
      // stable order inside each cell: rank by extended index
      for (int e = t; e < n_ext; e += BLOCK) {
        int cq = cell_of(e);
        int lo = cstart[cq], hi = cstart[cq + 1];
        int r = 0;
        for (int q = lo; q < hi; ++q) r += (tmp[q] < e) ? 1 : 0;
        sorted[lo + r] = (uint16_t)e;
      }
      __syncthreads();
    }
    // neighbour lists: rows of the (2R+1)^3 stencil in fixed order
    int over = 0;
#pragma unroll
    for (int k = 0; k < APT; ++k) {
      int a = t + k * BLOCK;
      int cnt = 0;
      auto push = [&](uint32_t v) __attribute__((always_inline)) {
        if (cnt < list_cap) list[(((cnt >> 3) * n_pad + a) << 3) + (cnt & 7)] = (uint16_t)v;
        ++cnt;
      };
      // Appends the atoms in cell order lo..hi within rl of the build
      // position of atom a, in order. Four candidates per round: their
      // positions (and, without sorted slots, their indices first) are all
      // loaded before the first is tested, so the LDS latency is paid once
      // per four. Entries past hi point at the atom itself, which the
      // self test drops. Pushed values are position offsets: slots when
      // SORTED, extended indices otherwise.
      const float bxi = bx[k], byi = by[k], bzi = bz[k];
      const PT bpx = to_pt(bxi), bpy = to_pt(byi), bpz = to_pt(bzi);
      const int self = SORTED ? sslot[k] : a;
      auto scan = [&](int lo, int hi) __attribute__((always_inline)) {
        for (int q = lo; q < hi; q += 4) {
          int e4[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            if (SORTED) {
              e4[u] = q + u < hi ? q + u : self;
            } else {
              const int e = sorted[min(q + u, hi - 1)];
              e4[u] = q + u < hi ? e : a;
            }
          }
          float d2[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const float ddx = pdiff(bpx, PX(e4[u])), ddy = pdiff(bpy, PY(e4[u])), ddz = pdiff(bpz, PZ(e4[u]));
            d2[u] = fmaf(ddx, ddx, fmaf(ddy, ddy, ddz * ddz));
          }
#pragma unroll
          for (int u = 0; u < 4; ++u)
            if (d2[u] < rl2 && e4[u] != self) push((uint32_t)(PB * e4[u]));
        }
      };
      // an atom whose position is not finite (a blown-up cell, which the
      // step's observables flag) gets an empty list: the stencil bounds below
      // convert coordinates to integers
      const bool fin = isfinite(bx[k]) && isfinite(by[k]) && isfinite(bz[k]);
      if (a < N && MI && fin) {
        // periodic stencil, one cell at a time (the grid has at least 2R+1
        // cells per edge); rows and cells the rl-sphere cannot reach are
        // skipped (see the ghost branch)
        const float xi = bx[k], yi = by[k], zi = bz[k];
        const int cx = cell_coord(xi), cy = cell_coord(yi), cz = cell_coord(zi);
        const float ux = xi * inv_ce, uy = yi * inv_ce, uz = zi * inv_ce;
        for (int dz = -R; dz <= R; ++dz) {
          const float gz = fmaxf(0.f, fmaxf((float)(cz + dz) - uz, uz - (float)(cz + dz + 1)));
          const float rz = rlc2 - gz * gz;
          if (rz <= 0.f) continue;
          const int zz = wrapc(cz + dz);
          for (int dy = -R; dy <= R; ++dy) {
            const float gy = fmaxf(0.f, fmaxf((float)(cy + dy) - uy, uy - (float)(cy + dy + 1)));
            const float rr = rz - gy * gy;
            if (rr <= 0.f) continue;
            const float wx = sqrtf(rr);
            const int yy = wrapc(cy + dy);
            const int x0 = max(cx - R, (int)floorf(ux - wx)), x1 = min(cx + R, (int)floorf(ux + wx));
            for (int dx = x0 - cx; dx <= x1 - cx; ++dx) {
              const int cq = (zz * nce + yy) * nce + wrapc(cx + dx);
              scan(cstart[cq], cstart[cq + 1]);
            }
          }
        }
      } else if (a < N && fin) {
        // Rows (dy, dz) of the stencil in fixed order. In cell units (u = the
        // atom's fractional cell coordinate) a row is skipped when its y and z
        // cell intervals are at least rl away, and its x range is cut to the
        // cells that the chord of the rl-sphere touches: only cells holding no
        // point within rl are dropped, so the list and its order are those of
        // the full stencil.
        const float xi = bx[k], yi = by[k], zi = bz[k];
        const int cx = cell_coord(xi), cy = cell_coord(yi), cz = cell_coord(zi);
        const float ux = (xi + rl) * inv_ce, uy = (yi + rl) * inv_ce, uz = (zi + rl) * inv_ce;
        for (int dz = -R; dz <= R; ++dz) {
          const int zz = cz + dz;
          if (zz < 0 || zz >= nce) continue;
          const float gz = fmaxf(0.f, fmaxf((float)zz - uz, uz - (float)(zz + 1)));
          const float rz = rlc2 - gz * gz;
          if (rz <= 0.f) continue;
          for (int dy = -R; dy <= R; ++dy) {
            const int yy = cy + dy;
            if (yy < 0 || yy >= nce) continue;
            const float gy = fmaxf(0.f, fmaxf((float)yy - uy, uy - (float)(yy + 1)));
            const float rr = rz - gy * gy;
            if (rr <= 0.f) continue;
            const float wx = sqrtf(rr);
            const int x0 = max(max(cx - R, 0), (int)floorf(ux - wx));
            const int x1 = min(min(cx + R, nce - 1), (int)floorf(ux + wx));
            if (x0 > x1) continue;
            const int row = (zz * nce + yy) * nce;
            scan(cstart[row + x0], cstart[row + x1 + 1]);
          }
        }
      }
      over |= (cnt > list_cap) ? 1 : 0;
      int cm = wave_max_i(cnt);
      if (lane == 0 && cm > 0) atomicMax(&c->max_list, cm);
      cm = min(cm, list_cap);
      int nb = __builtin_amdgcn_readfirstlane((cm + 7) >> 3);
      nblk[k] = nb;
      if (PRUNE) fnb[k] = nb;
      // pad every lane of the wave (also atoms past N) to nb blocks: with the
      // far-away sentinel, or (minimum image, where no point is far from all
      // atoms) with the atom itself, which the r^2 > 0 test drops
      if (a < n_pad) {
        int from = (a < N) ? min(cnt, list_cap) : 0;
        const uint16_t pad = (uint16_t)(PB * (MI ? (a < N ? a : SENT) : SENT));
        // the open row entry by entry, then whole 16-byte padding rows
        int q = from;
        for (; (q & 7) && q < 8 * nb; ++q) list[(((q >> 3) * n_pad + a) << 3) + (q & 7)] = pad;
        const uint32_t pp = (uint32_t)pad * 0x00010001u;
        for (int b = q >> 3; b < nb; ++b) reinterpret_cast<uint4*>(list)[b * n_pad + a] = make_uint4(pp, pp, pp, pp);
      }
    }
    if (over) ctl->overflow = 1;
    inner = false;
    __syncthreads();
    bool ok = ctl->overflow == 0;
    if (t == 0) atomicMax(&c->max_ext, n_ext);
    ctl->n_ext = n_ext;
    return ok;
  }

  // Current positions of real atoms and their ghost images into LDS.
  DEVI void refresh_positions() {
#pragma unroll
    for (int k = 0; k < APT; ++k) {
      int a = t + k * BLOCK;
      if (a < N) {
        const int sl = SORTED ? sslot[k] : a;
        PX(sl) = to_pt(x[k]);
        PY(sl) = to_pt(y[k]);
        PZ(sl) = to_pt(z[k]);
        if (gmask[k]) {
          if (SORTED)
            write_images_sorted(x[k], y[k], z[k], gmask[k], gofs[k]);
          else
            write_images(x[k], y[k], z[k], gmask[k], gofs[k]);
        }
      }
    }
  }

  // Wrap the current positions into [0, L) and rebuild the lists from them.
  DEVI bool rebuild() {
#pragma unroll
    for (int k = 0; k < APT; ++k) {
      if (valid(k)) {
        x[k] = wrap1(x[k], Lw);
        y[k] = wrap1(y[k], Lw);
        z[k] = wrap1(z[k], Lw);
      }
      bx[k] = (float)x[k];
      by[k] = (float)y[k];
      bz[k] = (float)z[k];
    }
    if (t == 0) c->n_builds += 1;  // chunk-start reconstructions are not counted
    return build_lists();
  }

  // Per-group sums of one atom's walk, formed right after it so that no
  // per-atom sum outlives the walk in registers: for owned atom k, the wave
  // owning its group g adds the halved virial w and energy u (full lists see
  // every pair twice) and the halved pair virial tensor s6 over its 64 lanes,
  // and lane 0 writes them (0 where ACC does not ask for a value; atoms past
  // N add 0). The in-range pair count goes to pairs_t on energy steps.
  template <int ACC>
  DEVI void walk_sums(int k, double w, double u, int cin, const float (&s6)[6], double* gdst, double* tdst) {
    const bool v = valid(k);
    const int g = k * NW + wv;
    const double W = ACC >= ACC_FW ? wave_sum(v ? 0.5 * w : 0.0) : 0.0;
    const double U = ACC >= ACC_FWU ? wave_sum(v ? 0.5 * u : 0.0) : 0.0;
    if (ACC >= ACC_FWU) pairs_t += (double)(v ? cin : 0);
    if (lane == 0 && g < p.caps.gmax) {
      gdst[3 * g + 1] = W;
      gdst[3 * g + 2] = U;
    }
    if (ACC == ACC_FWUS) {
#pragma unroll
      for (int c6 = 0; c6 < 6; ++c6) {
        const double sc = wave_sum(v ? 0.5 * (double)s6[c6] : 0.0);
        if (lane == 0 && g < p.caps.gmax) tdst[6 * g + c6] = sc;
      }
    }
  }

  // --- pair forces (LJTS, FP32) -------------------------------------------------
  // For every listed neighbour j of i with r^2 < rc^2:
  //   f_ij = 24 r^-2 r^-6 (2 r^-6 - 1) d, pair virial r.f = 24 r^-6 (2 r^-6 - 1),
  //   energy 4 r^-6 (r^-6 - 1) - 4 (rc^-12 - rc^-6).
  // Neighbours between rc and rl and the padding entries add exact zeros.
  // ACC selects what else is summed per atom besides the FP32 force:
  // ACC_F nothing, ACC_FW the virial, ACC_FWU virial, energy and the in-range
  // pair count. KAHAN sums virial and energy in FP32 with Kahan compensation,
  // otherwise each term is promoted and summed in FP64.
  // Hands the list blocks of owned atom a (nb blocks of 8 entries, two 16-bit
  // byte offsets per word) to fn in order.
  // The list the force walks use: the inner lists after a prune, otherwise
  // the lists of the last build.
  DEVI const uint16_t* force_list() const { return (PRUNE && inner) ? ilist : list; }
  DEVI int force_blocks(int k) const { return PRUNE ? fnb[k] : nblk[k]; }

  template <class FN>
  DEVI void walk_list(const uint16_t* base, int a, int nb, FN&& fn) {
    if (a < n_pad && nb > 0) {
      // Blocks are loaded one ahead into two alternating registers, so a
      // block's load latency (device memory when the list does not fit in
      // LDS) overlaps the arithmetic of the block before it.
      // The loads are unconditional (the index is clamped to the last
      // block, nb - 1 < list_cap / 8), so the wait before a block only
      // covers the load issued before it.
      // The scheduling barriers keep each load where it is issued (the
      // scheduler would otherwise sink it next to its use).
      const uint4* row = reinterpret_cast<const uint4*>(base) + a;
      uint4 e0 = row[0];
      for (int b = 0; b < nb; b += 2) {
        const uint4 e1 = row[min(b + 1, nb - 1) * n_pad];
        __builtin_amdgcn_sched_barrier(0);
        fn(e0);
        if (b + 1 >= nb) break;
        e0 = row[min(b + 2, nb - 1) * n_pad];
        __builtin_amdgcn_sched_barrier(0);
        fn(e1);
      }
    }
  }

  // Inner lists from the current positions: the entries of each atom's list
  // with r^2 < (rc + prune_skin)^2, in list order, each wave padded to its
  // longest like the lists of a build. Every thread writes and later reads
  // only the rows of its own atoms.
  DEVI void prune() {
    const char* pb = reinterpret_cast<const char*>(px);
#pragma unroll
    for (int k = 0; k < APT; ++k) {
      const int a = t + k * BLOCK;
      const PT xi = to_pt(x[k]), yi = to_pt(y[k]), zi = to_pt(z[k]);
      int cnt = 0;
      auto block = [&](const uint4 ent) __attribute__((always_inline)) {
        const uint32_t wd4[4] = {ent.x, ent.y, ent.z, ent.w};
#pragma unroll
        for (int m = 0; m < 8; ++m) {
          const uint32_t off = (m & 1) ? (wd4[m >> 1] >> 16) : (wd4[m >> 1] & 0xffffu);
          const PT* q = reinterpret_cast<const PT*>(pb + off);
          const float dx = pdiff(xi, q[0]), dy = pdiff(yi, q[EXT]), dz = pdiff(zi, q[2 * EXT]);
          const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
          if (MI ? (r2 < rin2 && r2 > 0.0f) : r2 < rin2) {
            // cnt never exceeds the entries of the outer row (< list_cap)
            ilist[(((cnt >> 3) * n_pad + a) << 3) + (cnt & 7)] = (uint16_t)off;
            ++cnt;
          }
        }
      };
      walk_list(list, a, a < N ? nblk[k] : 0, block);
      const int nb = __builtin_amdgcn_readfirstlane((wave_max_i(cnt) + 7) >> 3);
      fnb[k] = nb;
      if (a < n_pad) {
        const uint16_t pad = (uint16_t)(PB * (MI ? (a < N ? a : SENT) : SENT));
        int q = cnt;
        for (; (q & 7) && q < 8 * nb; ++q) ilist[(((q >> 3) * n_pad + a) << 3) + (q & 7)] = pad;
        const uint32_t pp = (uint32_t)pad * 0x00010001u;
        for (int b = q >> 3; b < nb; ++b) reinterpret_cast<uint4*>(ilist)[b * n_pad + a] = make_uint4(pp, pp, pp, pp);
      }
      prx[k] = (float)x[k];
      pry[k] = (float)y[k];
      prz[k] = (float)z[k];
    }
    inner = true;
    __syncthreads();
  }

  template <int ACC, bool KAHAN>
  DEVI void forces_impl(double* gdst, double* tdst) {
    const char* pb = reinterpret_cast<const char*>(px);
#pragma unroll
    for (int k = 0; k < APT; ++k) {
      const int a = t + k * BLOCK;
      const PT xi = to_pt(x[k]), yi = to_pt(y[k]), zi = to_pt(z[k]);
      float ax = 0.f, ay = 0.f, az = 0.f;
      double wd = 0.0, ud = 0.0;                  // FP64 sums
      float ws = 0.f, wc = 0.f, us = 0.f, uc = 0.f;  // Kahan sums and compensations
      float sxx = 0.f, syy = 0.f, szz = 0.f, sxy = 0.f, sxz = 0.f, syz = 0.f;  // virial tensor
      int cin = 0;
      const int nb = force_blocks(k);
      // one block of 8 list entries (two 16-bit byte offsets per word)
      auto block = [&](const uint4 ent) __attribute__((always_inline)) {
        const uint32_t wd4[4] = {ent.x, ent.y, ent.z, ent.w};
#pragma unroll
        for (int m = 0; m < 8; ++m) {
          const uint32_t off = (m & 1) ? (wd4[m >> 1] >> 16) : (wd4[m >> 1] & 0xffffu);
          const PT* q = reinterpret_cast<const PT*>(pb + off);
          const float dx = pdiff(xi, q[0]), dy = pdiff(yi, q[EXT]), dz = pdiff(zi, q[2 * EXT]);
          const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
          const bool in = MI ? (r2 < rc2 && r2 > 0.0f) : r2 < rc2;
          const float ir2 = in ? __builtin_amdgcn_rcpf(r2) : 0.0f;
          const float ir6 = ir2 * ir2 * ir2;
          const float vir = fmaf(48.0f, ir6, -24.0f) * ir6;
          const float ff = vir * ir2;
          if (ACC == ACC_FWUS) {
            // pair virial tensor d_a f_b with f = ff d (six components)
            const float fdx = ff * dx, fdy = ff * dy, fdz = ff * dz;
            ax = fmaf(ff, dx, ax);
            ay = fmaf(ff, dy, ay);
            az = fmaf(ff, dz, az);
            sxx = fmaf(fdx, dx, sxx);
            syy = fmaf(fdy, dy, syy);
            szz = fmaf(fdz, dz, szz);
            sxy = fmaf(fdx, dy, sxy);
            sxz = fmaf(fdx, dz, sxz);
            syz = fmaf(fdy, dz, syz);
          } else {
            ax = fmaf(ff, dx, ax);
            ay = fmaf(ff, dy, ay);
            az = fmaf(ff, dz, az);
          }
          if (ACC >= ACC_FW) {
            if (KAHAN) {
              const float y1 = vir - wc, t1 = ws + y1;
              wc = (t1 - ws) - y1;
              ws = t1;
            } else {
              wd += (double)vir;
            }
          }
          if (ACC >= ACC_FWU) {
            const float e = fmaf(ir6, ir6, -ir6);
            if (KAHAN) {
              const float y2 = e - uc, t2 = us + y2;
              uc = (t2 - us) - y2;
              us = t2;
            } else {
              ud += (double)e;
            }
            cin += in ? 1 : 0;
          }
        }
      };
      walk_list(force_list(), a, nb, block);
      FX(k) = ax;
      FY(k) = ay;
      FZ(k) = az;
      if (KAHAN) {
        wd = (double)ws - (double)wc;
        ud = (double)us - (double)uc;
      }
      walk_sums<ACC>(k, wd, fma(-(double)cin, u_shift, 4.0 * ud), cin, {sxx, syy, szz, sxy, sxz, syz}, gdst, tdst);
    }
  }

  // --- embedded-atom forces (Eq. Etot, FP32 pair math) --------------------------
  // First walk: rhobar_i = sum_j f_s(r_ij) over the listed neighbours in range.
  // Each owner then keeps F'(rhobar_i) = -c / (2 sqrt(rhobar_i)) (0 for an
  // atom with no neighbour in range, which no pair uses) and 2 F(rhobar_i) in
  // FP64, and writes F' as float into LDS for the atom and its ghost images.
  // After a barrier, the second walk forms, with d = x_i - x_j,
  //   f_ij = -[V_s'(r) + (F'_i + F'_j) f_s'(r)] d / r
  //        = r^-1 [9 r^-10 - e_c9 + (F'_i + F'_j)(6 r^-7 - e_c6)] d,
  // the pair virial r.f_ij and, on energy steps, V_s(r). Out-of-range
  // neighbours and padding take 1/r = 0, so they add exact zeros.
  DEVI void eam_density(float (&fpi)[APT], double (&emb)[APT]) {
    const char* pb = reinterpret_cast<const char*>(px);
    if (t == 0) fpv[SENT] = 0.0f;  // the padding slot's F' must be finite
#pragma unroll
    for (int k = 0; k < APT; ++k) {
      const int a = t + k * BLOCK;
      const PT xi = to_pt(x[k]), yi = to_pt(y[k]), zi = to_pt(z[k]);
      float rs = 0.f;
      auto block = [&](const uint4 ent) __attribute__((always_inline)) {
        const uint32_t wd4[4] = {ent.x, ent.y, ent.z, ent.w};
#pragma unroll
        for (int m = 0; m < 8; ++m) {
          const uint32_t off = (m & 1) ? (wd4[m >> 1] >> 16) : (wd4[m >> 1] & 0xffffu);
          const PT* q = reinterpret_cast<const PT*>(pb + off);
          const float dx = pdiff(xi, q[0]), dy = pdiff(yi, q[EXT]), dz = pdiff(zi, q[2 * EXT]);
          const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
          const bool in = MI ? (r2 < rc2 && r2 > 0.0f) : r2 < rc2;
          const float ir = in ? __builtin_amdgcn_rsqf(r2) : 0.0f;
          const float ir2 = ir * ir;
          const float ir4 = ir2 * ir2;
          const float fr = fmaf(e_c6, r2 * ir, fmaf(ir4, ir2, -e_k6));
          rs += in ? fr : 0.0f;
        }
      };
      walk_list(force_list(), a, force_blocks(k), block);
      const double rb = (double)rs;
      const double sq = rb > 0.0 ? sqrt(rb) : 0.0;
      fpi[k] = rb > 0.0 ? (float)(-eam_c / (2.0 * sq)) : 0.0f;
      emb[k] = -2.0 * eam_c * sq;
      if (a < N) {
        fpv[a] = fpi[k];
        if (!MI && gmask[k]) write_image_vals(fpi[k], gmask[k], gofs[k]);
      }
    }
  }

  template <int ACC, bool KAHAN>
  DEVI void eam_forces_impl(double* gdst, double* tdst) {
    float fpi[APT];
    double emb[APT];
    eam_density(fpi, emb);
    __syncthreads();  // every F' of this step is in LDS
    const char* pb = reinterpret_cast<const char*>(px);
    const char* fb = reinterpret_cast<const char*>(fpv);
#pragma unroll
    for (int k = 0; k < APT; ++k) {
      const int a = t + k * BLOCK;
      const PT xi = to_pt(x[k]), yi = to_pt(y[k]), zi = to_pt(z[k]);
      const float fpk = fpi[k];
      float ax = 0.f, ay = 0.f, az = 0.f;
      double wd = 0.0, ud = 0.0;
      float ws = 0.f, wc = 0.f, us = 0.f, uc = 0.f;
      float sxx = 0.f, syy = 0.f, szz = 0.f, sxy = 0.f, sxz = 0.f, syz = 0.f;
      int cin = 0;
      auto block = [&](const uint4 ent) __attribute__((always_inline)) {
        const uint32_t wd4[4] = {ent.x, ent.y, ent.z, ent.w};
#pragma unroll
        for (int m = 0; m < 8; ++m) {
          const uint32_t off = (m & 1) ? (wd4[m >> 1] >> 16) : (wd4[m >> 1] & 0xffffu);
          const PT* q = reinterpret_cast<const PT*>(pb + off);
          // F' of neighbour j: float slot j (the offset is 4 j)
          const float fpj = *reinterpret_cast<const float*>(fb + off);
          const float dx = pdiff(xi, q[0]), dy = pdiff(yi, q[EXT]), dz = pdiff(zi, q[2 * EXT]);
          const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
          const bool in = MI ? (r2 < rc2 && r2 > 0.0f) : r2 < rc2;
          const float ir = in ? __builtin_amdgcn_rsqf(r2) : 0.0f;
          const float ir2 = ir * ir;
          const float ir6 = ir2 * ir2 * ir2;
          const float ir7 = ir6 * ir;
          const float ir10 = ir6 * ir2 * ir2;
          const float dv = fmaf(9.0f, ir10, -e_c9);
          const float df = fmaf(6.0f, ir7, -e_c6);
          const float ff = ir * fmaf(fpk + fpj, df, dv);
          const float vir = ff * r2;
          if (ACC == ACC_FWUS) {
            const float fdx = ff * dx, fdy = ff * dy, fdz = ff * dz;
            ax = fmaf(ff, dx, ax);
            ay = fmaf(ff, dy, ay);
            az = fmaf(ff, dz, az);
            sxx = fmaf(fdx, dx, sxx);
            syy = fmaf(fdy, dy, syy);
            szz = fmaf(fdz, dz, szz);
            sxy = fmaf(fdx, dy, sxy);
            sxz = fmaf(fdx, dz, sxz);
            syz = fmaf(fdy, dz, syz);
          } else {
            ax = fmaf(ff, dx, ax);
            ay = fmaf(ff, dy, ay);
            az = fmaf(ff, dz, az);
          }
          if (ACC >= ACC_FW) {
            if (KAHAN) {
              const float y1 = vir - wc, t1 = ws + y1;
              wc = (t1 - ws) - y1;
              ws = t1;
            } else {
              wd += (double)vir;
            }
          }
          if (ACC >= ACC_FWU) {
            const float e = in ? fmaf(e_c9, r2 * ir, fmaf(ir6 * ir2, ir, -e_k9)) : 0.0f;
            if (KAHAN) {
              const float y2 = e - uc, t2 = us + y2;
              uc = (t2 - us) - y2;
              us = t2;
            } else {
              ud += (double)e;
            }
            cin += in ? 1 : 0;
          }
        }
      };
      walk_list(force_list(), a, force_blocks(k), block);
      FX(k) = ax;
      FY(k) = ay;
      FZ(k) = az;
      if (KAHAN) {
        wd = (double)ws - (double)wc;
        ud = (double)us - (double)uc;
      }
      // sum_j V_s + 2 F(rhobar_i), halved with the pair terms below
      walk_sums<ACC>(k, wd, ud + emb[k], cin, {sxx, syy, szz, sxy, sxz, syz}, gdst, tdst);
    }
  }

  // Forces of every owned atom into (fx, fy, fz), and per 64-atom group the
  // halved sums ACC asks for: W / 2 and E_pot / 2 into gdst[3 g + 1] and
  // gdst[3 g + 2], the pair virial tensor / 2 into tdst[6 g + c].
  template <int ACC>
  DEVI void forces(double* gdst, double* tdst = nullptr) {
    if (EAM) {
      if (kahan)
        eam_forces_impl<ACC, true>(gdst, tdst);
      else
        eam_forces_impl<ACC, false>(gdst, tdst);
    } else {
      if (kahan)
        forces_impl<ACC, true>(gdst, tdst);
      else
        forces_impl<ACC, false>(gdst, tdst);
    }
  }

  // --- per-step bookkeeping (FP64) --------------------------------------------------

  DEVI bool is_rescale(int k) const {
    bool hit = false;
#pragma unroll
    for (int r = 0; r < MDEOS_MAX_RESCALE; ++r) hit = hit || rescale_at[r] == k;
    return hit;
    return false;
  }
  DEVI bool is_energy_step(int k) const {
    const int n = n_steps, w0 = n - n_avg;
    return debug_energy || (k % energy_every == 0) || k == n || k == w0 || is_rescale(k);
  }

  // Observables of step k from the block sums (wave 0 only; all lanes compute
  // the same values, lane 0 writes). Eq. stress: P = (2K + W) / (3V).
  DEVI double pressure(double K, double W) const { return (2.0 * K + W) / (3.0 * V); }
  DEVI double temperature(double K) const { return 2.0 * K / Ndof; }
  DEVI void observe(int k, double K, double W, double U, bool energy) {
    record(k, K, W, U, pressure(K, W), temperature(K), energy);
  }
  // Folds step k (P and T already formed) into the accumulators, in step order.
  DEVI void record(int k, double K, double W, double U, double P, double T, bool energy) {
    const int n = n_steps, w0 = n - n_avg;
    bool bad = !isfinite(K) || !isfinite(W) || (energy && !isfinite(U));
    if (lane == 0) {
      if (bad) {
        ctl->status |= ST_NONFINITE;
        ctl->stop = 1;
      }
      ctl->K = K;
      ctl->W = W;
      if (energy) ctl->U = U;
      if (k > w0) {
        const int idx = k - w0 - 1;
        const int bl = n_avg / n_blocks;
        const int b = idx / bl;
        ctl->sumP[b] += P;
        ctl->sumT[b] += T;
        if (idx == 0) ctl->P_ref = P;
        const double dp = P - ctl->P_ref;
        ctl->sumdP2 = fma(dp, dp, ctl->sumdP2);
        if (energy && (k % energy_every == 0 || k == n)) {
          ctl->sumU += U;
          ctl->nU += 1;
        }
      }
      if (k == w0) ctl->E_w0 = K + U;
      if (k == n) ctl->E_n = K + U;
      if (nvt) {
        // E_pot window of the next temperature update: second half of the
        // segment since the previous one
        const int s = next_update(k), prev = ctl->seg_prev;
        if (s >= 0 && k > prev + (s - prev) / 2 && (k % energy_every == 0 || k == s)) {
          ctl->segU += U;
          ctl->segN += 1;
        }
      }
    }
  }

  // Steps k_first..k_last have their group sums in ring slots (k % ring).
  // Lane s forms step k_first + s (box sums, P, T); the accumulation then
  // runs in step order.
  DEVI void flush(int k_first, int k_last) {
    if (wv != 0 || k_last < k_first) return;
    const int R = p.caps.ring;
    const int cnt = k_last - k_first + 1;
    double Ks = 0.0, Ws = 0.0, Us = 0.0, Ps = 0.0, Ts = 0.0;
    if (lane < cnt) {
      const double* r = ring + (size_t)((k_first + lane) % R) * 3 * p.caps.gmax;
      for (int g = 0; g < G; ++g) {
        Ks += r[3 * g + 0];
        Ws += r[3 * g + 1];
        Us += r[3 * g + 2];
      }
      Ps = pressure(Ks, Ws);
      Ts = temperature(Ks);
    }
    for (int s = 0; s < cnt; ++s) {
      const double K = readlane_d(Ks, s), W = readlane_d(Ws, s), U = readlane_d(Us, s);
      const double P = readlane_d(Ps, s), T = readlane_d(Ts, s);
      const int k = k_first + s;
      record(k, K, W, U, P, T, is_energy_step(k));
    }
  }

  // --- load / store ------------------------------------------------------------------

  DEVI void load_state() {
    const int off = c->atom_off;
#pragma unroll
    for (int k = 0; k < APT; ++k) {
      int a = t + k * BLOCK;
      if (a < N) {
        x[k] = p.a.x[off + a]; y[k] = p.a.y[off + a]; z[k] = p.a.z[off + a];
        vx[k] = p.a.vx[off + a]; vy[k] = p.a.vy[off + a]; vz[k] = p.a.vz[off + a];
        FX(k) = p.a.fx[off + a]; FY(k) = p.a.fy[off + a]; FZ(k) = p.a.fz[off + a];
        bx[k] = p.a.bx[off + a]; by[k] = p.a.by[off + a]; bz[k] = p.a.bz[off + a];
      } else {
        x[k] = y[k] = z[k] = vx[k] = vy[k] = vz[k] = 0.0;
        FX(k) = FY(k) = FZ(k) = bx[k] = by[k] = bz[k] = 0.f;
      }
    }
  }
  DEVI void store_state() {
    const int off = c->atom_off;
#pragma unroll
    for (int k = 0; k < APT; ++k) {
      int a = t + k * BLOCK;
      if (a < N) {
        p.a.x[off + a] = x[k]; p.a.y[off + a] = y[k]; p.a.z[off + a] = z[k];
        p.a.vx[off + a] = vx[k]; p.a.vy[off + a] = vy[k]; p.a.vz[off + a] = vz[k];
        p.a.fx[off + a] = FX(k); p.a.fy[off + a] = FY(k); p.a.fz[off + a] = FZ(k);
        p.a.bx[off + a] = bx[k]; p.a.by[off + a] = by[k]; p.a.bz[off + a] = bz[k];
      }
    }
  }
  DEVI void load_acc() {
    if (t == 0) {
      for (int b = 0; b < kMaxBlocks; ++b) {
        ctl->sumP[b] = c->sumP[b];
        ctl->sumT[b] = c->sumT[b];
      }
      ctl->P_ref = c->P_ref; ctl->sumdP2 = c->sumdP2; ctl->sumU = c->sumU; ctl->nU = c->nU;
      ctl->E_w0 = c->E_w0; ctl->E_n = c->E_n; ctl->K = c->K; ctl->U = c->U; ctl->W = c->W;
      ctl->status = c->status;
      ctl->stop = 0;
      ctl->overflow = 0;
      ctl->T_th = c->T_th; ctl->segU = c->segU; ctl->segN = c->segN; ctl->seg_prev = c->seg_prev;
      for (int q = 0; q < 6; ++q) {
        ctl->sigK[q] = c->sigK[q];
        ctl->sigV[q] = c->sigV[q];
      }
      ctl->nS = c->nS;
    }
  }
  DEVI void clear_acc() {
    if (t == 0) {
      for (int b = 0; b < kMaxBlocks; ++b) ctl->sumP[b] = ctl->sumT[b] = 0.0;
      ctl->P_ref = ctl->sumdP2 = ctl->sumU = 0.0;
      ctl->nU = 0;
      ctl->E_w0 = ctl->E_n = ctl->K = ctl->U = ctl->W = 0.0;
      ctl->status = 0;
      ctl->stop = 0;
      ctl->overflow = 0;
      ctl->T_th = c->T_th;  // the host's first guess, 2 N e / N_DOF
      ctl->segU = 0.0;
      ctl->segN = 0;
      ctl->seg_prev = 0;
      for (int q = 0; q < 6; ++q) ctl->sigK[q] = ctl->sigV[q] = 0.0;
      ctl->nS = 0;
    }
  }
  DEVI void store_acc(int step, int phase) {
    if (t == 0) {
      for (int b = 0; b < kMaxBlocks; ++b) {
        c->sumP[b] = ctl->sumP[b];
        c->sumT[b] = ctl->sumT[b];
      }
      c->P_ref = ctl->P_ref; c->sumdP2 = ctl->sumdP2; c->sumU = ctl->sumU; c->nU = ctl->nU;
      c->E_w0 = ctl->E_w0; c->E_n = ctl->E_n; c->K = ctl->K; c->U = ctl->U; c->W = ctl->W;
      c->status = ctl->status;
      c->step = step;
      c->phase = phase;
      c->T_th = ctl->T_th; c->segU = ctl->segU; c->segN = ctl->segN; c->seg_prev = ctl->seg_prev;
      for (int q = 0; q < 6; ++q) {
        c->sigK[q] = ctl->sigK[q];
        c->sigV[q] = ctl->sigV[q];
      }
      c->nS = ctl->nS;
    }
  }

  // --- lift pieces ----------------------------------------------------------------------

  // FCC lattice at the cell's density, l = (4 / rho)^(1/3) (Eq. numdens with
  // alpha = 4): atom a = 4((ix n_c + iy) n_c + iz) + b at l((ix,iy,iz) + basis_b + 1/4).
  DEVI void lattice_positions(double rho) {
    const int nc = c->n_c;
    const double l = cbrt(4.0 / rho);
#pragma unroll
    for (int k = 0; k < APT; ++k) {
      int a = t + k * BLOCK;
      if (a < N) {
        int b = a & 3, cell = a >> 2;
        int iz = cell % nc, iy = (cell / nc) % nc, ix = cell / (nc * nc);
        double ox = (b == 2 || b == 3) ? 0.5 : 0.0;
        double oy = (b == 1 || b == 3) ? 0.5 : 0.0;
        double oz = (b == 1 || b == 2) ? 0.5 : 0.0;
        // rounded to float like the stored lattice of the oracle
        x[k] = (double)(float)(l * (ix + ox + 0.25));
        y[k] = (double)(float)(l * (iy + oy + 0.25));
        z[k] = (double)(float)(l * (iz + oz + 0.25));
      } else {
        x[k] = y[k] = z[k] = 0.0;
      }
    }
  }

  // Forces, E_pot and W at the current positions with fresh lists.
  // Returns false on overflow.
  DEVI bool full_force_pass(double& U, double& W) {
    if (!rebuild()) return false;
    refresh_positions();
    __syncthreads();
    forces<ACC_FWU>(red);
    __syncthreads();
    if (t == 0) {
      double s1 = 0.0, s2 = 0.0;
      for (int g = 0; g < G; ++g) {
        s1 += red[3 * g + 1];
        s2 += red[3 * g + 2];
      }
      ctl->scal[1] = s1;
      ctl->scal[2] = s2;
    }
    __syncthreads();
    W = ctl->scal[1];
    U = ctl->scal[2];
    __syncthreads();
    return true;
  }

  DEVI double kinetic_now() {
    double ka[APT], za[APT];
#pragma unroll
    for (int k = 0; k < APT; ++k) {
      ka[k] = valid(k) ? 0.5 * fma(vx[k], vx[k], fma(vy[k], vy[k], vz[k] * vz[k])) : 0.0;
      za[k] = 0.0;
    }
    double K, z1, z2;
    reduce_now(ka, za, za, K, z1, z2);
    return K;
  }

  // Cold energy: E_pot of the static lattice at the cell's density.
  DEVI bool cold_energy(double& Ec) {
    lattice_positions(c->rho);
    double W;
    return full_force_pass(Ec, W);
  }

  // Gaussian velocities at T0 = 2 N e / N_DOF, centre of mass removed, scaled
  // so K = N e exactly (FP64), then rounded to float.
  DEVI void draw_velocities() {
    const double T0 = 2.0 * N * c->e / Ndof;
    const double sT = sqrt(T0);
    double v0[APT], v1[APT], v2[APT];
#pragma unroll
    for (int k = 0; k < APT; ++k) {
      int a = t + k * BLOCK;
      if (a < N) {
        v0[k] = gauss(c->seed, c->cell_id, a, 0) * sT;
        v1[k] = gauss(c->seed, c->cell_id, a, 1) * sT;
        v2[k] = gauss(c->seed, c->cell_id, a, 2) * sT;
      } else {
        v0[k] = v1[k] = v2[k] = 0.0;
      }
    }
    double m0, m1, m2;
    reduce_now(v0, v1, v2, m0, m1, m2);
    m0 /= N; m1 /= N; m2 /= N;
    double ke[APT], za[APT];
#pragma unroll
    for (int k = 0; k < APT; ++k) {
      if (valid(k)) {
        v0[k] -= m0; v1[k] -= m1; v2[k] -= m2;
        ke[k] = 0.5 * fma(v0[k], v0[k], fma(v1[k], v1[k], v2[k] * v2[k]));
      } else {
        ke[k] = 0.0;
      }
      za[k] = 0.0;
    }
    double K, z1, z2;
    reduce_now(ke, za, za, K, z1, z2);
    const double lam = sqrt(N * c->e / K);
#pragma unroll
    for (int k = 0; k < APT; ++k) {
      // rounded to float: the lifted state is float-representable (as in the oracle)
      vx[k] = valid(k) ? (double)(float)(v0[k] * lam) : 0.0;
      vy[k] = valid(k) ? (double)(float)(v1[k] * lam) : 0.0;
      vz[k] = valid(k) ? (double)(float)(v2[k] * lam) : 0.0;
    }
  }

  // Step-0 record after a lift: observables (and the re-pin when 0 is
  // scheduled). U0, W0 are the energy and virial of the current positions.
  DEVI void record_step0(double U0, double W0) {
    double K = kinetic_now();
    if (is_rescale(0)) {
      const double Kt = fma((double)N, c->e, -(U0 - Ecold));
      if (Kt <= 0.0) {
        if (t == 0) ctl->status |= ST_BELOW_COLD;
      } else {
        const double lam = sqrt(Kt / K);
#pragma unroll
        for (int k = 0; k < APT; ++k) {
          vx[k] *= lam; vy[k] *= lam; vz[k] *= lam;
        }
        K = kinetic_now();
        // a step-0 temperature update has no sampled window: with the
        // instantaneous E_pot it is this same re-pin, T = 2 K_t / N_DOF
        if (nvt && t == 0) ctl->T_th = 2.0 * Kt / Ndof;
      }
    }
    if (wv == 0) observe(0, K, W0, U0, true);
    __syncthreads();
  }

  // --- the cell -----------------------------------------------------------------------

  // Advances cell cidx from where it stands: a cell not yet lifted is lifted
  // first (its state and accumulators then stored as at step 0), and the
  // steps always start from the stored state, as after a chunk boundary, so
  // the kernel holds one copy of the step loop and a whole run takes the path
  // of a chunked one.
  DEVI void run(int cidx) {
    load_cell(cidx);
    const int phase = c->phase;
    if (phase == PH_DONE) return;
    if (phase != PH_RUN) {
      if (!lift_cell(phase) || p.step_budget < 0) return;  // (a lift-only launch ends here)
      __syncthreads();
      if (c->phase != PH_RUN) return;
    }
    const int step = c->step;
    load_acc();
    load_state();
    __syncthreads();
    if (!build_lists()) {
      fail_overflow(step);
      return;
    }
    refresh_positions();
    advance_steps(step);
  }

  // Lifting operator and the forces-only pass; false when the cell failed or
  // is done (nothing left to advance in this launch).
  DEVI bool lift_cell(int phase) {
    clear_acc();
    __syncthreads();
    double Ec = 0.0, U0 = 0.0, W0 = 0.0;
    if (phase == PH_FORCES) {
      load_state();
      if (!full_force_pass(U0, W0)) {
        fail_overflow(0);
        return false;
      }
#pragma unroll
      for (int k = 0; k < APT; ++k) vx[k] = vy[k] = vz[k] = 0.0;
      store_state();
      if (t == 0) {
        c->U = U0;
        c->W = W0;
        c->K = 0.0;
        c->phase = PH_DONE;
        c->status = 0;
      }
      return false;
    }
    // lifting operator: E_cold of the static lattice at rho
    lattice_positions(c->rho);
    if (!full_force_pass(Ec, W0)) {
      fail_overflow(0);
      return false;
    }
    if (t == 0) c->Ecold = Ec;
    Ecold = Ec;
    U0 = Ec;
    bool cold = phase == PH_COLD;
    if (!cold) {
      load_state();
      if (phase == PH_WARM) {
        // dilate the resident configuration to the new box: x <- x L'/L
        const double Lold = c->Lw / c->warm_scale;
        const double s = c->warm_scale;
#pragma unroll
        for (int k = 0; k < APT; ++k) {
          if (valid(k)) {
            x[k] = wrap1(wrap1(x[k], Lold) * s, Lw);
            y[k] = wrap1(wrap1(y[k], Lold) * s, Lw);
            z[k] = wrap1(wrap1(z[k], Lold) * s, Lw);
          }
        }
      }
      __syncthreads();
      if (!full_force_pass(U0, W0)) {
        fail_overflow(0);
        return false;
      }
      if (phase == PH_WARM && !(fma((double)N, c->e, -(U0 - Ec)) > 0.0)) {
        // no kinetic energy left above the new cold lattice: lift cold instead
        cold = true;
        if (t == 0) ctl->status |= ST_COLD_RELIFT;
        lattice_positions(c->rho);
        if (!full_force_pass(U0, W0)) {
          fail_overflow(0);
          return false;
        }
      }
    }
    if (cold) draw_velocities();
    record_step0(U0, W0);
    // the state after the lift, as a launch that stops at step 0 leaves it
    store_state();
    const bool done = n_steps <= 0 || ctl->stop != 0;
    store_acc(0, done ? PH_DONE : PH_RUN);
    return !done;
  }

  DEVI void fail_overflow(int step) {
    if (t == 0) {
      c->status |= ST_OVERFLOW;
      c->phase = PH_DONE;
      c->step = step;
    }
  }

  DEVI void advance_steps(int step) {
    const int n = n_steps;
    int target = n;
    if (p.step_budget > 0) target = min(n, step + p.step_budget);
    else if (p.step_budget < 0) target = step;
    const int RING = p.caps.ring;
    const float thr = 0.25f * (rl - sqrtf(rc2)) * (rl - sqrtf(rc2));  // (skin / 2)^2
    int pending = step + 1;  // first step not yet flushed
    pairs_t = 0.0;
    esteps = 0;
    bool fresh = true;  // the first step of a launch prunes (the build before it left outer lists)
    if (PRUNE) {
#pragma unroll
      for (int q = 0; q < APT; ++q) {
        prx[q] = (float)x[q];
        pry[q] = (float)y[q];
        prz[q] = (float)z[q];
      }
    }
    __syncthreads();
    bool stopped = ctl->stop != 0;
    while (step < target && !stopped) {
      const int k = step + 1;
      // kick + drift, own ghosts, displacements since the build and the prune
      float dm = 0.f, dp = 0.f;
      // Langevin noise amplitude of this step: beta has variance 2 gamma T dt
      const double hsig = nvt ? 0.5 * sqrt(gamma_dt2 * ctl->T_th) : 0.0;
#pragma unroll
      for (int q = 0; q < APT; ++q) {
        if (valid(q)) {
          if (nvt) {
            // GJF first half: u = sqrt(b) (v + dt f / 2 + beta / 2); x += sqrt(b) dt u
            double z0, z1, z2;
            noise3(seed, cell_id, t + q * BLOCK, k, query, z0, z1, z2);
            vx[q] = gjf_sb * fma(hdt, (double)FX(q), fma(hsig, z0, vx[q]));
            vy[q] = gjf_sb * fma(hdt, (double)FY(q), fma(hsig, z1, vy[q]));
            vz[q] = gjf_sb * fma(hdt, (double)FZ(q), fma(hsig, z2, vz[q]));
            x[q] = fma(gjf_sb * dt, vx[q], x[q]);
            y[q] = fma(gjf_sb * dt, vy[q], y[q]);
            z[q] = fma(gjf_sb * dt, vz[q], z[q]);
          } else {
            vx[q] = fma(hdt, (double)FX(q), vx[q]);
            vy[q] = fma(hdt, (double)FY(q), vy[q]);
            vz[q] = fma(hdt, (double)FZ(q), vz[q]);
            x[q] = fma(dt, vx[q], x[q]);
            y[q] = fma(dt, vy[q], y[q]);
            z[q] = fma(dt, vz[q], z[q]);
          }
          const float ex = (float)x[q] - bx[q], ey = (float)y[q] - by[q], ez = (float)z[q] - bz[q];
          dm = fmaxf(dm, fmaf(ex, ex, fmaf(ey, ey, ez * ez)));
          if (PRUNE && prune_cell) {
            const float gx = (float)x[q] - prx[q], gy = (float)y[q] - pry[q], gz = (float)z[q] - prz[q];
            dp = fmaxf(dp, fmaf(gx, gx, fmaf(gy, gy, gz * gz)));
          }
        }
      }
      // owners write their atoms and ghost images (the last barrier of the
      // previous step ended every read of the old positions)
      refresh_positions();
      dm = wave_max(dm);
      if (lane == 0) ctl->wmax[wv] = dm;
      if (PRUNE && prune_cell) {
        dp = wave_max(dp);
        if (lane == 0) ctl->pmax[wv] = dp;
      }
      __syncthreads();
      float gm = 0.f, gp = 0.f;
#pragma unroll
      for (int w = 0; w < NW; ++w) gm = fmaxf(gm, ctl->wmax[w]);
      if (PRUNE && prune_cell) {
#pragma unroll
        for (int w = 0; w < NW; ++w) gp = fmaxf(gp, ctl->pmax[w]);
      }
      const bool rebuilt = gm > thr;
      if (rebuilt) {
        if (!rebuild()) {
          flush(pending, step);
          __syncthreads();
          store_acc(step, PH_DONE);
          if (t == 0) c->status |= ST_OVERFLOW;
          return;
        }
        refresh_positions();
        __syncthreads();
      }
      if (PRUNE && prune_cell && (rebuilt || fresh || gp > pthr)) {
        prune();
        fresh = false;
      }
      const bool energy = is_energy_step(k);
      // steps where the stress tensor of Eq. stress is sampled (as <E_pot>)
      const bool sample = energy && k > n_steps - n_avg && (k % energy_every == 0 || k == n_steps);
      // this step's ring slot: the walks write W and E_pot per group, the
      // kinetic sums below K
      double* slot = ring + (size_t)(k % RING) * 3 * p.caps.gmax;
      if (sample) {
        forces<ACC_FWUS>(slot, red);
        ++esteps;
        // pair virial tensor (halved per group by the walks), groups in order
        __syncthreads();
        if (t == 0) {
#pragma unroll
          for (int c6 = 0; c6 < 6; ++c6) {
            double sc = 0.0;
            for (int g = 0; g < G; ++g) sc += red[6 * g + c6];
            ctl->sigV[c6] += sc;
          }
        }
        __syncthreads();
      } else if (energy) {
        forces<ACC_FWU>(slot);
        ++esteps;
      } else if (k > n_steps - n_avg || debug_energy) {
        forces<ACC_FW>(slot);  // the virial enters P only inside the averaging window
      } else {
        forces<ACC_F>(slot);
      }
      double ka[APT];
#pragma unroll
      for (int q = 0; q < APT; ++q) {
        if (nvt) {
          // GJF second half, the same noise redrawn: v = (a / sqrt(b)) u + dt f' / 2 + beta / 2
          if (valid(q)) {
            double z0, z1, z2;
            noise3(seed, cell_id, t + q * BLOCK, k, query, z0, z1, z2);
            vx[q] = fma(gjf_a_sb, vx[q], fma(hdt, (double)FX(q), hsig * z0));
            vy[q] = fma(gjf_a_sb, vy[q], fma(hdt, (double)FY(q), hsig * z1));
            vz[q] = fma(gjf_a_sb, vz[q], fma(hdt, (double)FZ(q), hsig * z2));
          }
        } else {
          vx[q] = fma(hdt, (double)FX(q), vx[q]);
          vy[q] = fma(hdt, (double)FY(q), vy[q]);
          vz[q] = fma(hdt, (double)FZ(q), vz[q]);
        }
        ka[q] = valid(q) ? 0.5 * fma(vx[q], vx[q], fma(vy[q], vy[q], vz[q] * vz[q])) : 0.0;
      }
      group_sums1(ka, slot);
      if (sample) {
        double kt[6][APT];  // kinetic tensor m v_a v_b
#pragma unroll
        for (int q = 0; q < APT; ++q) {
          const bool v = valid(q);
          kt[0][q] = v ? vx[q] * vx[q] : 0.0;
          kt[1][q] = v ? vy[q] * vy[q] : 0.0;
          kt[2][q] = v ? vz[q] * vz[q] : 0.0;
          kt[3][q] = v ? vx[q] * vy[q] : 0.0;
          kt[4][q] = v ? vx[q] * vz[q] : 0.0;
          kt[5][q] = v ? vy[q] * vz[q] : 0.0;
        }
        tensor_add(kt, ctl->sigK);
        if (t == 0) ctl->nS += 1;
      }
      step = k;
      __syncthreads();
      if (is_rescale(k)) {
        // energy re-pin (Eq. Tcontribution): K <- N e - (E_pot - E_cold)
        flush(pending, k - 1);
        if (t == 0) {
          const double* r = ring + (size_t)(k % RING) * 3 * p.caps.gmax;
          double K = 0.0, W = 0.0, U = 0.0;
          for (int g = 0; g < G; ++g) {
            K += r[3 * g + 0];
            W += r[3 * g + 1];
            U += r[3 * g + 2];
          }
          double Kt;
          if (nvt) {
            // temperature update (Eq. Tcontribution) with E_pot averaged over
            // the window; velocities go to that temperature, which becomes
            // the thermostat's
            if (k > ctl->seg_prev) {
              ctl->segU += U;
              ctl->segN += 1;
            }
            const double Ubar = ctl->segN > 0 ? ctl->segU / ctl->segN : U;
            Kt = fma((double)N, c->e, -(Ubar - Ecold));
            if (Kt > 0.0 && isfinite(Kt)) ctl->T_th = 2.0 * Kt / Ndof;
            ctl->segU = 0.0;
            ctl->segN = 0;
            ctl->seg_prev = k;
          } else {
            Kt = fma((double)N, c->e, -(U - Ecold));  // energy re-pin with the instantaneous E_pot
          }
          ctl->do_rescale = (Kt > 0.0 && isfinite(Kt)) ? 1 : 0;
          ctl->lam = (Kt > 0.0) ? sqrt(Kt / K) : 1.0;
          if (!(Kt > 0.0)) ctl->status |= ST_BELOW_COLD;
          ctl->scal[3] = W;
          ctl->scal[2] = U;
        }
        __syncthreads();
        const double W = ctl->scal[3], U = ctl->scal[2];
        double K;
        if (ctl->do_rescale) {
          const double lam = ctl->lam;
#pragma unroll
          for (int q = 0; q < APT; ++q) {
            vx[q] *= lam; vy[q] *= lam; vz[q] *= lam;
          }
        }
        K = kinetic_now();
        if (wv == 0) observe(k, K, W, U, true);
        pending = k + 1;
        __syncthreads();
      } else if (k - pending + 1 >= RING || k == target) {
        flush(pending, k);
        pending = k + 1;
        __syncthreads();
      }
      stopped = ctl->stop != 0;
    }
    if (pending <= step) {
      flush(pending, step);
      __syncthreads();
    }
    {
      double pa[APT], za[APT];
#pragma unroll
      for (int q = 0; q < APT; ++q) {
        pa[q] = q == 0 ? pairs_t : 0.0;
        za[q] = 0.0;
      }
      double P, z1, z2;
      reduce_now(pa, za, za, P, z1, z2);
      if (t == 0) {
        c->pair_sum += P;
        c->pair_steps += esteps;
      }
    }
    store_state();
    const bool done = (step >= n) || stopped;
    store_acc(step, done ? PH_DONE : PH_RUN);
  }
};

template <int BLOCK, int APT, int EXT, bool LLDS, int WPE, bool MI, bool NVT, bool EAM>
__global__ void __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(WPE))) k_advance(AdvanceParams p) {
  extern __shared__ __align__(16) unsigned char lds[];
  Box<BLOCK, APT, EXT, LLDS, MI, NVT, EAM> box(p, lds);
  if (threadIdx.x == 0) {
    // the padding neighbour (minimum-image lists pad with the atom itself;
    // there only threads past the last atom name this slot)
    box.PX(EXT - 1) = MI ? 0 : kSentinelPos;
    box.PY(EXT - 1) = MI ? 0 : kSentinelPos;
    box.PZ(EXT - 1) = MI ? 0 : kSentinelPos;
  }
  const int n_work = p.meta[0];
  const int* work = p.work_base + p.meta[1];
  for (;;) {
    if (threadIdx.x == 0) box.ctl->item = atomicAdd(p.counter, 1);
    __syncthreads();
    const int item = box.ctl->item;
    __syncthreads();
    if (item >= n_work) break;
    box.run(work[item]);
    __syncthreads();
  }
}

}  // namespace

// Host-side wrappers of one launch shape, defined in the variant translation units.
#define MDEOS_DEFINE_VARIANT(B, A, E, L, W, M, T, P)                                                      \
  namespace variants {                                                                                     \
  hipError_t launch_##B##_##A##_##E##_##L##_##W##_##M##_##T##_##P(const AdvanceParams& p, int grid, int lds,  \
                                                                  hipStream_t s) {                         \
    hipLaunchKernelGGL((k_advance<B, A, E, L != 0, W, M != 0, T != 0, P != 0>), dim3(grid), dim3(B), lds, s, \
                       p);                                                                                 \
    return hipGetLastError();                                                                              \
  }                                                                                                        \
  hipError_t attr_##B##_##A##_##E##_##L##_##W##_##M##_##T##_##P() {                                          \
    return hipFuncSetAttribute((const void*)k_advance<B, A, E, L != 0, W, M != 0, T != 0, P != 0>,          \
                               hipFuncAttributeMaxDynamicSharedMemorySize, kLdsMax);                       \
  }                                                                                                        \
  int occ_##B##_##A##_##E##_##L##_##W##_##M##_##T##_##P(int lds) {                                           \
    int n = 0;                                                                                             \
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(                                                      \
            &n, (const void*)k_advance<B, A, E, L != 0, W, M != 0, T != 0, P != 0>, B, lds) != hipSuccess)  \
      n = 1;                                                                                               \
    return n;                                                                                              \
  }                                                                                                        \
  }

}  // namespace mdeos
