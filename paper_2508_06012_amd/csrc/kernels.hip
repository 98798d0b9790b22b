// gfx950 kernels of libmdeos outside the advance kernel (restricting
// operator, counter reset) and the dispatch over the advance launch shapes.
#include "mdeos_dev.h"
#include "mdeos_host.h"
#include "variants.h"

namespace mdeos {

namespace variants {
#define X(B, A, E, L, W, M, T, P)                                                                          \
  hipError_t launch_##B##_##A##_##E##_##L##_##W##_##M##_##T##_##P(const AdvanceParams& p, int grid, int lds,  \
                                                                  hipStream_t s);                            \
  hipError_t attr_##B##_##A##_##E##_##L##_##W##_##M##_##T##_##P();                                           \
  int occ_##B##_##A##_##E##_##L##_##W##_##M##_##T##_##P(int lds);
MDEOS_VARIANTS(X)
#undef X
}  // namespace variants

namespace {

// Restricting operator: time averages and block standard errors (FP64).
// A cell still inside its averaging window gets the averages of the samples
// recorded so far and block errors over its completed blocks only (NaN with
// fewer than two); its drift is NaN until the window's last step.
__global__ void k_restrict(const CellRec* cells, const int* idx, int n, DevResult* out) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const CellRec& c = cells[idx[i]];
  DevResult r;
  const bool fin = c.phase == PH_DONE;
  const int B = c.n_blocks, na = c.n_avg, bl = na / B;
  const int done = fin ? na : min(na, max(0, c.step - (c.n_steps - na)));
  const int Bc = fin ? B : min(B, done / bl);  // completed blocks
  double sP = 0.0, sT = 0.0;
  for (int b = 0; b < B; ++b) {
    sP += c.sumP[b];
    sT += c.sumT[b];
  }
  r.P = done > 0 ? sP / done : NAN;
  r.T = done > 0 ? sT / done : NAN;
  double cP = 0.0, cT = 0.0;
  for (int b = 0; b < Bc; ++b) {
    cP += c.sumP[b];
    cT += c.sumT[b];
  }
  const double mP = cP / ((double)Bc * bl), mT = cT / ((double)Bc * bl);
  double aP = 0.0, aT = 0.0;
  for (int b = 0; b < Bc; ++b) {
    const double mp = c.sumP[b] / bl - mP, mt = c.sumT[b] / bl - mT;
    aP += mp * mp;
    aT += mt * mt;
  }
  r.P_se = Bc >= 2 ? sqrt(aP / (Bc * (Bc - 1.0))) : NAN;
  r.T_se = Bc >= 2 ? sqrt(aT / (Bc * (Bc - 1.0))) : NAN;
  // one pass about the window's first sample: var = <(P - P_ref)^2> - (<P> - P_ref)^2
  const double d = r.P - c.P_ref;
  const double var = c.sumdP2 / done - d * d;
  r.P_rms = done > 0 ? sqrt(var > 0.0 ? var : 0.0) : NAN;
  r.Epot_mean = c.nU > 0 ? c.sumU / c.nU / c.N : NAN;
  r.Ecold = c.Ecold / c.N;
  r.drift = fin ? (c.E_n - c.E_w0) / c.N : NAN;
  // Eq. stress: (kinetic + pair virial) / V averaged over the sampled steps
  for (int q = 0; q < 6; ++q) r.stress[q] = c.nS > 0 ? (c.sigK[q] + c.sigV[q]) / (c.nS * c.V) : NAN;
  int st = c.status;
  if (fin && c.ensemble != MDEOS_NVT_LANGEVIN && fabs(r.drift) > c.drift_tol) st |= ST_DRIFT;  // energy is not conserved under a thermostat
  if (st & (ST_NONFINITE | ST_OVERFLOW)) {
    r.P = r.P_se = r.P_rms = r.T = r.T_se = r.Epot_mean = r.drift = NAN;
    for (int q = 0; q < 6; ++q) r.stress[q] = NAN;
  }
  r.pairs = c.pair_steps > 0 ? c.pair_sum / c.pair_steps : 0.0;
  r.n_samples = done;
  r.status = st;
  r.n_builds = c.n_builds;
  r.max_list = c.max_list;
  r.max_ext = c.max_ext;
  r.pad = 0;
  out[i] = r;
}

__global__ void k_zero_ints(int* p, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

}  // namespace

static const Variant kVariants[] = {
#define X(B, A, E, L, W, M, T, P) {B, A, E, L, W, M, T, P},
    MDEOS_VARIANTS(X)
#undef X
};

int variant_count() { return (int)(sizeof(kVariants) / sizeof(kVariants[0])); }
Variant variant_at(int i) { return kVariants[i]; }

bool variant_available(const Variant& v) {
  for (const Variant& w : kVariants)
    if (same_variant(w, v)) return true;
  return false;
}

hipError_t launch_advance(const Variant& v, const AdvanceParams& p, int grid, int lds_bytes, hipStream_t s) {
#define X(B, A, E, L, W, M, T, P)                                                                  \
  if (v.block == B && v.apt == A && v.ext == E && v.list_lds == L && v.wpe == W && v.mi == M && v.nvt == T && \
      v.eam == P)                                                                                           \
    return variants::launch_##B##_##A##_##E##_##L##_##W##_##M##_##T##_##P(p, grid, lds_bytes, s);
  MDEOS_VARIANTS(X)
#undef X
  return hipErrorInvalidValue;
}

hipError_t init_kernel_attributes() {
  hipError_t e = hipSuccess;
#define X(B, A, E, L, W, M, T, P) \
  if (e == hipSuccess) e = variants::attr_##B##_##A##_##E##_##L##_##W##_##M##_##T##_##P();
  MDEOS_VARIANTS(X)
#undef X
  return e;
}

int occupancy(const Variant& v, int lds_bytes) {
#define X(B, A, E, L, W, M, T, P)                                                                  \
  if (v.block == B && v.apt == A && v.ext == E && v.list_lds == L && v.wpe == W && v.mi == M && v.nvt == T && \
      v.eam == P)                                                                                           \
    return variants::occ_##B##_##A##_##E##_##L##_##W##_##M##_##T##_##P(lds_bytes);
  MDEOS_VARIANTS(X)
#undef X
  return 1;
}

hipError_t launch_restrict(const CellRec* cells, const int* idx, int n, DevResult* out, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_restrict, dim3((n + 127) / 128), dim3(128), 0, s, cells, idx, n, out);
  return hipGetLastError();
}

hipError_t launch_zero_ints(int* p, int n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero_ints, dim3((n + 255) / 256), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

}  // namespace mdeos
