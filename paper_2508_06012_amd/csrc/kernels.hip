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
__global__ void k_restrict(const CellRec* cells, const int* idx, int n, DevResult* out) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const CellRec& c = cells[idx[i]];
  DevResult r;
  const int B = c.n_blocks, na = c.n_avg, bl = na / B;
  const int done = (c.phase == PH_DONE) ? c.n_avg : max(0, c.step - (c.n_steps - c.n_avg));
  double sP = 0.0, sT = 0.0;
  for (int b = 0; b < B; ++b) {
    sP += c.sumP[b];
    sT += c.sumT[b];
  }
  r.P = sP / na;
  r.T = sT / na;
  double aP = 0.0, aT = 0.0;
  for (int b = 0; b < B; ++b) {
    const double mp = c.sumP[b] / bl - r.P, mt = c.sumT[b] / bl - r.T;
    aP += mp * mp;
    aT += mt * mt;
  }
  r.P_se = sqrt(aP / (B * (B - 1.0)));
  r.T_se = sqrt(aT / (B * (B - 1.0)));
  const double d = r.P - c.P_ref;
  const double var = c.sumdP2 / na - d * d;
  r.P_rms = sqrt(var > 0.0 ? var : 0.0);
  r.Epot_mean = c.nU > 0 ? c.sumU / c.nU / c.N : NAN;
  r.Ecold = c.Ecold / c.N;
  r.drift = (c.E_n - c.E_w0) / c.N;
  // Eq. stress: (kinetic + pair virial) / V averaged over the sampled steps
  for (int q = 0; q < 6; ++q) r.stress[q] = c.nS > 0 ? (c.sigK[q] + c.sigV[q]) / (c.nS * c.V) : NAN;
  int st = c.status;
  if (c.ensemble != MDEOS_NVT_LANGEVIN && fabs(r.drift) > c.drift_tol) st |= ST_DRIFT;  // energy is not conserved under a thermostat
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
