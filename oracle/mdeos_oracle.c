/*
 * mdeos oracle: a plain, slow, FP64 CPU implementation of the in-line
 * molecular-dynamics equation of state (lift -> advance -> restrict) for a
 * truncated-shifted Lennard-Jones (LJTS) fluid in reduced units, or for a
 * many-body material of the embedded-atom form (Eq. Etot).
 *
 * TEST INFRASTRUCTURE. Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg load this library. The product path (the HIP
 * library and its Python binding) never calls it, and it shares no code,
 * header, table or helper with that path.
 *
 * Every routine follows the paper ("Advancing Material Modeling in Hydrocodes
 * Beyond Equations of State", arXiv 2508.06012) step by step:
 *   - lifting operator (Sec. III): number density -> lattice parameter
 *     (Eq. numdens), atom count (Eq. numAtoms), cold energy from the static
 *     lattice, first-guess temperature, Gaussian velocities, temperature
 *     update of Eq. Tcontribution;
 *   - microscopic model (Sec. II.B): Newton's equations integrated with
 *     velocity Verlet, periodic boundaries; or, for thermostatted lifting and
 *     canonical (NVT) production (Sec. III), the GJF Langevin integrator the
 *     paper cites (Sec. II.B) with the iterated temperature updates of
 *     Eq. Tcontribution;
 *   - restricting operator (Sec. III, Eq. stress): pressure as one third of
 *     the trace of the kinetic + virial stress, time averaged; fluctuation
 *     reported as an RMS (Sec. IV.B).
 * Readings of passages the paper leaves open (reduced units, FCC start,
 * N = 4 n_c^3, N_DOF = 3N - 3, the energy zero at E_cold, NVE production
 * with instantaneous energy re-pinning, block standard errors) are listed
 * with the project's design notes; each is restated next to the code here.
 *
 * Arrays of positions, velocities and forces are row-major [N][3] doubles.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_NONFINITE 1
#define ORC_BELOW_COLD 2
#define ORC_DRIFT 4

typedef struct {
    double rho;      /* reduced number density rho* */
    double e;        /* target specific internal energy per atom, measured from E_cold */
    int n_c;         /* FCC unit cells per box edge; N = 4 n_c^3 */
    double rc;       /* LJTS cutoff radius */
    double dt;       /* time step */
    uint64_t seed;   /* Philox key word 0 */
    int64_t cell_id; /* Philox key word 1 */
    int64_t query;   /* index of this query of the cell (0 for the first); thermostat counter word 3 */
    int potential;   /* 0: LJTS (well depth from the schedule); 1: embedded-atom form (Eq. Etot) */
    double eam_c;    /* embedding strength c of the embedded-atom form */
} orc_cell;

typedef struct {
    int n_steps;          /* velocity-Verlet steps after the lift */
    int n_avg;            /* samples averaged: steps n_steps-n_avg+1 .. n_steps */
    int n_blocks;         /* blocks for the standard error */
    int n_rescale;        /* number of energy re-pin steps */
    int rescale_steps[8]; /* steps at which the energy is re-pinned (0 = right after the lift) */
    int energy_every;     /* potential energy enters <E_pot> on steps divisible by this */
    double drift_tol;     /* |E(n) - E(n - n_avg)| / N above this sets the drift status */
    double eps;           /* LJ well depth (1 in reduced units; 0 switches the potential off) */
    int ensemble;         /* 0: velocity Verlet with energy re-pins; 1: Langevin (GJF) with temperature updates */
    double gamma;         /* Langevin friction (ensemble 1) */
} orc_sched;

typedef struct {
    double P, P_se, P_rms, T, T_se, Epot_mean, Ecold, drift;
    double stress[6]; /* <sigma> (xx, yy, zz, xy, xz, yz) of Eq. stress over the sampled window steps */
    int n_samples, status;
} orc_result;

/* ---------------------------------------------------------------------------
 * Philox4x64-10 counter-based generator, from its published definition
 * (Salmon, Moraes, Dror and Shaw, "Parallel random numbers: as easy as
 * 1, 2, 3", SC11): ten rounds of two 64x64->128 multiplications with the
 * round keys bumped by two Weyl constants between rounds.
 * The paper only says the velocities are drawn from a Gaussian (Sec. III);
 * a counter-based generator makes each atom's draw reproducible on its own.
 * ------------------------------------------------------------------------- */
static void mulhilo64(uint64_t a, uint64_t b, uint64_t *lo, uint64_t *hi)
{
    unsigned __int128 p = (unsigned __int128)a * (unsigned __int128)b;
    *lo = (uint64_t)p;
    *hi = (uint64_t)(p >> 64);
}

void orc_philox4x64_10(const uint64_t key[2], const uint64_t ctr[4], uint64_t out[4])
{
    const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
    const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
    uint64_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t lo0, hi0, lo1, hi1;
        mulhilo64(M0, c0, &lo0, &hi0);
        mulhilo64(M1, c2, &lo1, &hi1);
        uint64_t n0 = hi1 ^ c1 ^ k0;
        uint64_t n1 = lo1;
        uint64_t n2 = hi0 ^ c3 ^ k1;
        uint64_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += W0;
        k1 += W1;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Standard normal for atom a, component c: Box-Muller on the first two words
 * of Philox4x64-10 with key (seed, cell_id) and counter (3a + c, 0, 0, 0).
 * u1 = 1 - (w0 >> 11) 2^-53 lies in (0, 1], u2 = (w1 >> 11) 2^-53 in [0, 1). */
double orc_gauss(uint64_t seed, int64_t cell_id, int64_t a, int c)
{
    uint64_t key[2] = {seed, (uint64_t)cell_id};
    uint64_t ctr[4] = {(uint64_t)(3 * a + c), 0, 0, 0};
    uint64_t w[4];
    orc_philox4x64_10(key, ctr, w);
    const double two_m53 = 1.0 / 9007199254740992.0;
    double u1 = 1.0 - (double)(w[0] >> 11) * two_m53;
    double u2 = (double)(w[1] >> 11) * two_m53;
    return sqrt(-2.0 * log(u1)) * cos(2.0 * M_PI * u2);
}

/* ---------------------------------------------------------------------------
 * Lifting operator, geometry (Sec. III, Eqs. numdens and numAtoms).
 * Reduced units: n = rho*. FCC with alpha = 4 atoms per cubic cell, lattice
 * parameter l = (alpha / rho)^(1/3), box edge L = n_c l, N = alpha n_c^3.
 * Atom a = 4((ix n_c + iy) n_c + iz) + b sits at l((ix,iy,iz) + basis_b + 1/4).
 * ------------------------------------------------------------------------- */
/* Thermostat noise of atom a at step k of query q: three standard normal
 * numbers from one Philox4x64-10 block with key (seed, cell_id) and counter
 * (a, k, 1, q) (the third counter word keeps this stream apart from the
 * lift's draws, the fourth apart from the cell's earlier queries).
 * Box-Muller on words (0, 1) gives z0 = R cos(theta), z1 = R sin(theta); on
 * words (2, 3), z2 = R' cos(theta'), with u = 1 - (w >> 11) 2^-53 for the
 * radius and u = (w >> 11) 2^-53 for the angle. */
void orc_noise3(uint64_t seed, int64_t cell_id, int64_t a, int64_t k, int64_t q, double z[3])
{
    const double two_m53 = 1.0 / 9007199254740992.0;
    const double two_pi = 6.283185307179586476925286766559;
    uint64_t key[2] = {seed, (uint64_t)cell_id};
    uint64_t ctr[4] = {(uint64_t)a, (uint64_t)k, 1u, (uint64_t)q};
    uint64_t w[4];
    orc_philox4x64_10(key, ctr, w);
    double u1 = 1.0 - (double)(w[0] >> 11) * two_m53;
    double u2 = (double)(w[1] >> 11) * two_m53;
    double u3 = 1.0 - (double)(w[2] >> 11) * two_m53;
    double u4 = (double)(w[3] >> 11) * two_m53;
    double r1 = sqrt(-2.0 * log(u1)), r2 = sqrt(-2.0 * log(u3));
    z[0] = r1 * cos(two_pi * u2);
    z[1] = r1 * sin(two_pi * u2);
    z[2] = r2 * cos(two_pi * u4);
}

double orc_lattice_param(double rho) { return cbrt(4.0 / rho); }
double orc_box_length(int n_c, double rho) { return n_c * orc_lattice_param(rho); }

void orc_lattice(int n_c, double rho, double *x)
{
    static const double basis[4][3] = {{0.0, 0.0, 0.0}, {0.0, 0.5, 0.5}, {0.5, 0.0, 0.5}, {0.5, 0.5, 0.0}};
    double l = orc_lattice_param(rho);
    for (int ix = 0; ix < n_c; ++ix)
        for (int iy = 0; iy < n_c; ++iy)
            for (int iz = 0; iz < n_c; ++iz)
                for (int b = 0; b < 4; ++b) {
                    int a = 4 * ((ix * n_c + iy) * n_c + iz) + b;
                    x[3 * a + 0] = l * (ix + basis[b][0] + 0.25);
                    x[3 * a + 1] = l * (iy + basis[b][1] + 0.25);
                    x[3 * a + 2] = l * (iz + basis[b][2] + 0.25);
                }
}

/* ---------------------------------------------------------------------------
 * Pair interaction: LJTS. phi(r) = 4 eps (r^-12 - r^-6) - 4 eps (rc^-12 - rc^-6)
 * for r < rc (strict), 0 otherwise. The force is -dphi/dr of the unshifted
 * part (the shift only moves the energy zero).
 * Pair virial r.f enters W; W/(3V) is the configurational part of the trace
 * of Eq. stress divided by three (Sec. III).
 * ------------------------------------------------------------------------- */
static void pair_term(double dx, double dy, double dz, double rc, double eps,
                      int i, int j, double *F, double *U, double *W, double *S)
{
    double r2 = dx * dx + dy * dy + dz * dz;
    if (!(r2 < rc * rc)) return;
    double ir2 = 1.0 / r2;
    double ir6 = ir2 * ir2 * ir2;
    double irc6 = 1.0 / (rc * rc * rc * rc * rc * rc);
    double phi = 4.0 * eps * (ir6 * ir6 - ir6) - 4.0 * eps * (irc6 * irc6 - irc6);
    /* f_ij = -dphi/dr * d/r = 24 eps r^-2 (2 r^-12 - r^-6) d */
    double ff = 24.0 * eps * ir2 * ir6 * (2.0 * ir6 - 1.0);
    F[3 * i + 0] += ff * dx; F[3 * i + 1] += ff * dy; F[3 * i + 2] += ff * dz;
    F[3 * j + 0] -= ff * dx; F[3 * j + 1] -= ff * dy; F[3 * j + 2] -= ff * dz;
    *U += phi;
    *W += ff * r2;
    if (S) {
        /* virial part of Eq. stress in pair form: sum over pairs of d_a f_b, f = ff d */
        S[0] += ff * dx * dx; S[1] += ff * dy * dy; S[2] += ff * dz * dz;
        S[3] += ff * dx * dy; S[4] += ff * dx * dz; S[5] += ff * dy * dz;
    }
}

/* All pairs i < j. When rc <= L/2 exactly one periodic image can be in range
 * and the minimum image (round half to even) is used; otherwise every image
 * n in {-1,0,1}^3 is tried (rc < L keeps self-images out of range). */
/* Forces, E_pot, the scalar virial W and, if S is not NULL, the virial
 * tensor S[6] = (xx, yy, zz, xy, xz, yz) of the pairs in range. */
void orc_forces_tensor(int N, double L, double rc, double eps, const double *x,
                       double *F, double *U_out, double *W_out, double *S)
{
    double U = 0.0, W = 0.0;
    if (S) memset(S, 0, sizeof(double) * 6);
    memset(F, 0, sizeof(double) * 3 * (size_t)N);
    if (eps != 0.0) {
        int multi = rc > 0.5 * L;
        for (int i = 0; i < N; ++i)
            for (int j = i + 1; j < N; ++j) {
                double d0 = x[3 * i + 0] - x[3 * j + 0];
                double d1 = x[3 * i + 1] - x[3 * j + 1];
                double d2 = x[3 * i + 2] - x[3 * j + 2];
                if (!multi) {
                    d0 -= L * nearbyint(d0 / L);
                    d1 -= L * nearbyint(d1 / L);
                    d2 -= L * nearbyint(d2 / L);
                    pair_term(d0, d1, d2, rc, eps, i, j, F, &U, &W, S);
                } else {
                    for (int n0 = -1; n0 <= 1; ++n0)
                        for (int n1 = -1; n1 <= 1; ++n1)
                            for (int n2 = -1; n2 <= 1; ++n2)
                                pair_term(d0 + n0 * L, d1 + n1 * L, d2 + n2 * L, rc, eps, i, j, F, &U, &W, S);
                }
            }
    }
    *U_out = U;
    *W_out = W;
}

void orc_forces(int N, double L, double rc, double eps, const double *x,
                double *F, double *U_out, double *W_out)
{
    orc_forces_tensor(N, L, rc, eps, x, F, U_out, W_out, NULL);
}

/* An independent route to the same pair set: a linked-cell list with cells of
 * edge >= rc (at least three per side) and the 27-cell stencil with explicit
 * image shifts. Used only to cross-check orc_forces. Returns -1 if the box
 * has fewer than three cells per side (the caller then uses orc_forces). */
int orc_forces_celllist(int N, double L, double rc, double eps, const double *x,
                        double *F, double *U_out, double *W_out)
{
    int nc = (int)floor(L / rc);
    if (nc < 3) return -1;
    double ce = L / nc;
    int ncell = nc * nc * nc;
    int *head = (int *)malloc(sizeof(int) * ncell);
    int *next = (int *)malloc(sizeof(int) * N);
    for (int c = 0; c < ncell; ++c) head[c] = -1;
    for (int i = N - 1; i >= 0; --i) {
        int c3[3];
        for (int k = 0; k < 3; ++k) {
            int ck = (int)floor(x[3 * i + k] / ce);
            if (ck < 0) ck = 0;
            if (ck >= nc) ck = nc - 1;
            c3[k] = ck;
        }
        int c = (c3[0] * nc + c3[1]) * nc + c3[2];
        next[i] = head[c];
        head[c] = i;
    }
    double U = 0.0, W = 0.0;
    memset(F, 0, sizeof(double) * 3 * (size_t)N);
    /* Each atom i visits every neighbour j in the 27 cells and keeps j > i:
     * every unordered pair is seen once from its smaller index. */
    for (int i = 0; i < N && eps != 0.0; ++i) {
        int ci[3];
        for (int k = 0; k < 3; ++k) {
            int ck = (int)floor(x[3 * i + k] / ce);
            if (ck < 0) ck = 0;
            if (ck >= nc) ck = nc - 1;
            ci[k] = ck;
        }
        for (int s0 = -1; s0 <= 1; ++s0)
            for (int s1 = -1; s1 <= 1; ++s1)
                for (int s2 = -1; s2 <= 1; ++s2) {
                    int cj[3] = {ci[0] + s0, ci[1] + s1, ci[2] + s2};
                    double shift[3];
                    for (int k = 0; k < 3; ++k) {
                        shift[k] = 0.0;
                        if (cj[k] < 0) { cj[k] += nc; shift[k] = -L; }
                        if (cj[k] >= nc) { cj[k] -= nc; shift[k] = L; }
                    }
                    int c = (cj[0] * nc + cj[1]) * nc + cj[2];
                    for (int j = head[c]; j >= 0; j = next[j]) {
                        if (j <= i) continue;
                        double d0 = x[3 * i + 0] - (x[3 * j + 0] + shift[0]);
                        double d1 = x[3 * i + 1] - (x[3 * j + 1] + shift[1]);
                        double d2 = x[3 * i + 2] - (x[3 * j + 2] + shift[2]);
                        pair_term(d0, d1, d2, rc, eps, i, j, F, &U, &W, NULL);
                    }
                }
    }
    free(head);
    free(next);
    *U_out = U;
    *W_out = W;
    return 0;
}

/* ---------------------------------------------------------------------------
 * Embedded-atom form (appendix, Eq. Etot):
 *   E_pot = 1/2 sum_{i != j} V(r_ij) + sum_i F(rhobar_i),
 *   rhobar_i = sum_{j != i} f(r_ij)   (the density other atoms superpose at i).
 * The paper's Cu tables are not available; the functions are an analytic
 * stand-in of the Finnis-Sinclair / Sutton-Chen family in reduced units
 * (energy eps, length a = the lattice parameter of the fitted crystal):
 *   V(r) = r^-9,  f(r) = r^-6,  F(rhobar) = -c sqrt(rhobar),
 * with V and f truncated at rc in shifted-force form, g_s(r) = g(r) - g(rc)
 * - (r - rc) g'(rc), so that energies and forces are continuous at rc.
 * Forces, from E_pot's dependence on distances only, with d = x_i - x_j:
 *   f_ij = -[V_s'(r) + (F'(rhobar_i) + F'(rhobar_j)) f_s'(r)] d / r,
 *   V_s'(r) = -9 (r^-10 - rc^-10),  f_s'(r) = -6 (r^-7 - rc^-7),
 *   F'(rhobar) = -c / (2 sqrt(rhobar)).
 * The virial and the virial tensor take these pair forces exactly as in the
 * pair-potential case (Eq. stress), which holds for any energy that depends
 * on interatomic distances alone.
 * ------------------------------------------------------------------------- */
typedef struct {
    double rc, c;
    double *rhobar;   /* sweep 0 accumulates */
    const double *Fp; /* sweep 1 reads F'(rhobar) */
    double *F, U, W, *S;
} eam_acc;

static void eam_pair(eam_acc *A, int sweep, double dx, double dy, double dz, int i, int j)
{
    double r2 = dx * dx + dy * dy + dz * dz;
    double rc = A->rc;
    if (!(r2 < rc * rc)) return;
    double r = sqrt(r2);
    if (sweep == 0) {
        double fr = pow(r, -6.0) - pow(rc, -6.0) + 6.0 * pow(rc, -7.0) * (r - rc);
        A->rhobar[i] += fr;
        A->rhobar[j] += fr;
        return;
    }
    double dV = -9.0 * (pow(r, -10.0) - pow(rc, -10.0));
    double df = -6.0 * (pow(r, -7.0) - pow(rc, -7.0));
    double ff = -(dV + (A->Fp[i] + A->Fp[j]) * df) / r;
    A->U += pow(r, -9.0) - pow(rc, -9.0) + 9.0 * pow(rc, -10.0) * (r - rc);
    A->F[3 * i + 0] += ff * dx; A->F[3 * i + 1] += ff * dy; A->F[3 * i + 2] += ff * dz;
    A->F[3 * j + 0] -= ff * dx; A->F[3 * j + 1] -= ff * dy; A->F[3 * j + 2] -= ff * dz;
    A->W += ff * r2;
    if (A->S) {
        A->S[0] += ff * dx * dx; A->S[1] += ff * dy * dy; A->S[2] += ff * dz * dz;
        A->S[3] += ff * dx * dy; A->S[4] += ff * dx * dz; A->S[5] += ff * dy * dz;
    }
}

/* The pair set of orc_forces_tensor: all pairs i < j, minimum image when
 * rc <= L/2, else every image in {-1,0,1}^3. */
static void eam_sweep(eam_acc *A, int sweep, int N, double L, const double *x)
{
    int multi = A->rc > 0.5 * L;
    for (int i = 0; i < N; ++i)
        for (int j = i + 1; j < N; ++j) {
            double d0 = x[3 * i + 0] - x[3 * j + 0];
            double d1 = x[3 * i + 1] - x[3 * j + 1];
            double d2 = x[3 * i + 2] - x[3 * j + 2];
            if (!multi) {
                d0 -= L * nearbyint(d0 / L);
                d1 -= L * nearbyint(d1 / L);
                d2 -= L * nearbyint(d2 / L);
                eam_pair(A, sweep, d0, d1, d2, i, j);
            } else {
                for (int n0 = -1; n0 <= 1; ++n0)
                    for (int n1 = -1; n1 <= 1; ++n1)
                        for (int n2 = -1; n2 <= 1; ++n2)
                            eam_pair(A, sweep, d0 + n0 * L, d1 + n1 * L, d2 + n2 * L, i, j);
            }
        }
}

/* Forces, E_pot, W and (if S is not NULL) the virial tensor of the
 * embedded-atom form; rhobar (N doubles, may be NULL) receives the densities. */
void orc_forces_eam(int N, double L, double rc, double c, const double *x,
                    double *F, double *U_out, double *W_out, double *S, double *rhobar_out)
{
    double *rhobar = (double *)calloc((size_t)N, sizeof(double));
    double *Fp = (double *)malloc(sizeof(double) * (size_t)N);
    eam_acc A = {rc, c, rhobar, Fp, F, 0.0, 0.0, S};
    memset(F, 0, sizeof(double) * 3 * (size_t)N);
    if (S) memset(S, 0, sizeof(double) * 6);
    eam_sweep(&A, 0, N, L, x);
    double Uemb = 0.0;
    for (int i = 0; i < N; ++i) {
        Uemb += -c * sqrt(rhobar[i]);
        /* an atom with no neighbour in range has no pair that would use F' */
        Fp[i] = rhobar[i] > 0.0 ? -c / (2.0 * sqrt(rhobar[i])) : 0.0;
    }
    eam_sweep(&A, 1, N, L, x);
    *U_out = A.U + Uemb;
    *W_out = A.W;
    if (rhobar_out) memcpy(rhobar_out, rhobar, sizeof(double) * (size_t)N);
    free(rhobar);
    free(Fp);
}

/* The cell's material: LJTS with well depth eps, or the embedded-atom form. */
static void cell_forces(const orc_cell *cell, double eps, int N, double L, const double *x,
                        double *F, double *U, double *W, double *S)
{
    if (cell->potential == 1)
        orc_forces_eam(N, L, cell->rc, cell->eam_c, x, F, U, W, S, NULL);
    else
        orc_forces_tensor(N, L, cell->rc, eps, x, F, U, W, S);
}

/* Round a double to the nearest float and back. */
static double to_f32(double v) { return (double)(float)v; }

static double kinetic(int N, const double *v)
{
    double K = 0.0;
    for (int i = 0; i < 3 * N; ++i) K += 0.5 * v[i] * v[i];
    return K;
}

/* Cold energy: potential energy of the static lattice at rho (Sec. III, the
 * energy found with near-zero velocities; read as exactly zero velocities). */
double orc_ecold_cell(const orc_cell *cell, double eps)
{
    int n_c = cell->n_c;
    int N = 4 * n_c * n_c * n_c;
    double *x = (double *)malloc(sizeof(double) * 3 * N);
    double *F = (double *)malloc(sizeof(double) * 3 * N);
    double U, W;
    orc_lattice(n_c, cell->rho, x);
    for (int i = 0; i < 3 * N; ++i) x[i] = to_f32(x[i]);
    cell_forces(cell, eps, N, orc_box_length(n_c, cell->rho), x, F, &U, &W, NULL);
    free(x);
    free(F);
    return U;
}

double orc_ecold(int n_c, double rho, double rc, double eps)
{
    int N = 4 * n_c * n_c * n_c;
    double *x = (double *)malloc(sizeof(double) * 3 * N);
    double *F = (double *)malloc(sizeof(double) * 3 * N);
    double U, W;
    orc_lattice(n_c, rho, x);
    for (int i = 0; i < 3 * N; ++i) x[i] = to_f32(x[i]);
    orc_forces(N, orc_box_length(n_c, rho), rc, eps, x, F, &U, &W);
    free(x);
    free(F);
    return U;
}

/* ---------------------------------------------------------------------------
 * Lift (Sec. III): lattice, E_cold, first-guess temperature T0 = 2 E / N_DOF
 * with E = N e and N_DOF = 3N - 3, Gaussian velocities at T0 with the centre
 * of mass velocity removed, then velocities scaled so that the energy above
 * the cold lattice, K + (E_pot - E_cold), equals N e exactly (E_pot = E_cold
 * on the lattice). Positions and velocities are then rounded to float, the
 * storage precision of the device state, so both sides start from the same
 * bits. Returns E_cold.
 * ------------------------------------------------------------------------- */
double orc_lift(const orc_cell *cell, double eps, double *x, double *v)
{
    int n_c = cell->n_c;
    int N = 4 * n_c * n_c * n_c;
    double Ndof = 3.0 * N - 3.0;
    orc_lattice(n_c, cell->rho, x);
    for (int i = 0; i < 3 * N; ++i) x[i] = to_f32(x[i]);
    double Ecold = orc_ecold_cell(cell, eps);

    double T0 = 2.0 * N * cell->e / Ndof;
    double mean[3] = {0.0, 0.0, 0.0};
    for (int a = 0; a < N; ++a)
        for (int c = 0; c < 3; ++c) {
            v[3 * a + c] = orc_gauss(cell->seed, cell->cell_id, a, c) * sqrt(T0);
            mean[c] += v[3 * a + c];
        }
    for (int c = 0; c < 3; ++c) mean[c] /= N;
    for (int a = 0; a < N; ++a)
        for (int c = 0; c < 3; ++c) v[3 * a + c] -= mean[c];
    double K = kinetic(N, v);
    double lam = sqrt(N * cell->e / K);
    for (int i = 0; i < 3 * N; ++i) v[i] = to_f32(v[i] * lam);
    return Ecold;
}

/* Block standard error of the mean: the series is cut into B contiguous
 * blocks of equal length; SE = sqrt(sum_b (m_b - m)^2 / (B (B - 1))). */
void orc_block_stats(int n, const double *s, int B, double *mean, double *se)
{
    int bl = n / B;
    double m = 0.0;
    for (int k = 0; k < B * bl; ++k) m += s[k];
    m /= (double)(B * bl);
    double acc = 0.0;
    for (int b = 0; b < B; ++b) {
        double mb = 0.0;
        for (int k = 0; k < bl; ++k) mb += s[b * bl + k];
        mb /= bl;
        acc += (mb - m) * (mb - m);
    }
    *mean = m;
    *se = sqrt(acc / (B * (B - 1.0)));
}

static int in_schedule(const orc_sched *s, int k)
{
    for (int r = 0; r < s->n_rescale; ++r)
        if (s->rescale_steps[r] == k) return 1;
    return 0;
}

/* First scheduled step >= k, or -1. */
static int next_update(const orc_sched *s, int k)
{
    int best = -1;
    for (int r = 0; r < s->n_rescale; ++r)
        if (s->rescale_steps[r] >= k && (best < 0 || s->rescale_steps[r] < best)) best = s->rescale_steps[r];
    return best;
}

/* ---------------------------------------------------------------------------
 * Advance and restrict.
 * Microscopic model (Sec. II.B): velocity Verlet, positions wrapped into
 * [0, L) with floor after each drift.
 * Temperature update (Sec. III, Eq. Tcontribution): at scheduled steps the
 * kinetic energy is set to K_t = N e - (E_pot - E_cold) by scaling all
 * velocities with sqrt(K_t / K); under energy-conserving dynamics this is the
 * paper's update applied to the instantaneous E_pot. K_t <= 0 flags the cell.
 * Restriction (Sec. III, Eq. stress): P_k = (2 K_k + W_k) / (3 V) is one third
 * of the trace (kinetic part m v v, virial part r f), T_k = 2 K_k / N_DOF.
 * The full tensor of Eq. stress (kinetic m v v plus pair virial d f over V,
 * six components) is averaged over the window steps where E_pot is sampled.
 * Samples k = n - n_avg + 1 .. n are averaged; the standard error uses
 * contiguous blocks; P_rms is the RMS deviation of the instantaneous P from
 * its mean (the fluctuation measure of Sec. IV).
 * Observables of a rescale step are taken after the rescale.
 *
 * Thermostatted lifting and canonical production (ensemble 1; Sec. III with
 * the GJF integrator of Sec. II.B, unit mass, k_B = 1). One step is
 *   x' = x + b dt v + (b dt^2 / 2) f + (b dt / 2) beta
 *   v' = a v + (dt / 2) (a f + f') + b beta
 * with c = gamma dt / 2, b = 1 / (1 + c), a = (1 - c) / (1 + c) and beta a
 * Gaussian vector of variance 2 gamma T_th dt per component (orc_noise3 for
 * the step). T_th starts at the first guess 2 N e / N_DOF (all energy
 * kinetic). At each scheduled step s the temperature update of
 * Eq. Tcontribution uses the potential energy sampled over the second half of
 * the segment since the previous update (steps k > mid, mid = prev +
 * (s - prev) / 2, taken at steps divisible by energy_every and at s itself;
 * the instantaneous value if there is none): T = 2 (N e - (<E_pot> - E_cold))
 * / N_DOF; velocities are scaled to that temperature and it becomes T_th.
 * The energy-drift status does not apply (energy is not conserved).
 *
 * State (x, v) is advanced in place. Records: K, U, W, P, T for steps
 * 0..n_steps (arrays of n_steps + 1, may be NULL) and forces for steps
 * 0..n_recF-1 (recF of n_recF * N * 3, may be NULL).
 * ------------------------------------------------------------------------- */
void orc_run(const orc_cell *cell, const orc_sched *sch, double Ecold_total,
             double *x, double *v,
             double *recK, double *recU, double *recW, double *recP, double *recT,
             int n_recF, double *recF, orc_result *res)
{
    int n_c = cell->n_c;
    int N = 4 * n_c * n_c * n_c;
    double L = orc_box_length(n_c, cell->rho);
    double V = L * L * L;
    double Ndof = 3.0 * N - 3.0;
    double dt = cell->dt;
    int n = sch->n_steps;
    int w0 = n - sch->n_avg; /* last step before the averaging window */
    int status = 0;

    double *F = (double *)malloc(sizeof(double) * 3 * N);
    double *Pser = (double *)malloc(sizeof(double) * (sch->n_avg > 0 ? sch->n_avg : 1));
    double *Tser = (double *)malloc(sizeof(double) * (sch->n_avg > 0 ? sch->n_avg : 1));
    double U, W, K;
    double sumU = 0.0;
    int nU = 0;
    double E_w0 = 0.0, E_n = 0.0;
    int nvt = sch->ensemble == 1;
    double T_th = 2.0 * N * cell->e / Ndof;
    double gc = 0.5 * sch->gamma * dt, gb = 1.0 / (1.0 + gc), ga = (1.0 - gc) / (1.0 + gc);
    double *beta = (double *)malloc(sizeof(double) * 3 * N);
    double *Fold = (double *)malloc(sizeof(double) * 3 * N);
    int prev = 0, segN = 0;
    double segU = 0.0;
    double S[6], sig[6] = {0, 0, 0, 0, 0, 0};
    int nS = 0;

    cell_forces(cell, sch->eps, N, L, x, F, &U, &W, S);
    K = kinetic(N, v);
    for (int k = 0; k <= n; ++k) {
        if (k > 0 && !nvt) {
            for (int i = 0; i < 3 * N; ++i) {
                v[i] += 0.5 * dt * F[i];
                x[i] += dt * v[i];
                x[i] -= L * floor(x[i] / L);
                if (x[i] >= L) x[i] = 0.0;
            }
            cell_forces(cell, sch->eps, N, L, x, F, &U, &W, S);
            for (int i = 0; i < 3 * N; ++i) v[i] += 0.5 * dt * F[i];
            K = kinetic(N, v);
        } else if (k > 0) {
            double sig = sqrt(2.0 * sch->gamma * T_th * dt);
            for (int a = 0; a < N; ++a) {
                double z[3];
                orc_noise3(cell->seed, cell->cell_id, a, k, cell->query, z);
                for (int c = 0; c < 3; ++c) beta[3 * a + c] = sig * z[c];
            }
            for (int i = 0; i < 3 * N; ++i) {
                x[i] += gb * dt * v[i] + 0.5 * gb * dt * dt * F[i] + 0.5 * gb * dt * beta[i];
                x[i] -= L * floor(x[i] / L);
                if (x[i] >= L) x[i] = 0.0;
                Fold[i] = F[i];
            }
            cell_forces(cell, sch->eps, N, L, x, F, &U, &W, S);
            for (int i = 0; i < 3 * N; ++i) v[i] = ga * v[i] + 0.5 * dt * (ga * Fold[i] + F[i]) + gb * beta[i];
            K = kinetic(N, v);
        }
        if (!isfinite(K) || !isfinite(U) || !isfinite(W)) {
            status |= ORC_NONFINITE;
            break;
        }
        if (nvt) {
            int s = next_update(sch, k);
            if (s >= 0 && k > prev + (s - prev) / 2 && (k % sch->energy_every == 0 || k == s)) {
                segU += U;
                segN += 1;
            }
        }
        if (in_schedule(sch, k) && !nvt) {
            double Kt = N * cell->e - (U - Ecold_total);
            if (Kt <= 0.0) {
                status |= ORC_BELOW_COLD;
            } else {
                double lam = sqrt(Kt / K);
                for (int i = 0; i < 3 * N; ++i) v[i] *= lam;
                K = kinetic(N, v);
            }
        } else if (in_schedule(sch, k)) {
            double Ubar = segN > 0 ? segU / segN : U;
            double Tn = 2.0 * (N * cell->e - (Ubar - Ecold_total)) / Ndof;
            if (Tn <= 0.0) {
                status |= ORC_BELOW_COLD;
            } else {
                double lam = sqrt(Tn / (2.0 * K / Ndof));
                for (int i = 0; i < 3 * N; ++i) v[i] *= lam;
                K = kinetic(N, v);
                T_th = Tn;
            }
            prev = k;
            segU = 0.0;
            segN = 0;
        }
        double P = (2.0 * K + W) / (3.0 * V);
        double T = 2.0 * K / Ndof;
        if (recK) recK[k] = K;
        if (recU) recU[k] = U;
        if (recW) recW[k] = W;
        if (recP) recP[k] = P;
        if (recT) recT[k] = T;
        if (recF && k < n_recF) memcpy(recF + (size_t)k * 3 * N, F, sizeof(double) * 3 * N);
        if (k == w0) E_w0 = K + U;
        if (k == n) E_n = K + U;
        if (k > w0) {
            Pser[k - w0 - 1] = P;
            Tser[k - w0 - 1] = T;
            if (k % sch->energy_every == 0 || k == n) {
                sumU += U;
                nU += 1;
                /* Eq. stress on the same sampled steps: (sum m v_a v_b + sum d_a f_b) / V */
                double kv[6] = {0, 0, 0, 0, 0, 0};
                for (int a = 0; a < N; ++a) {
                    const double *va = v + 3 * a;
                    kv[0] += va[0] * va[0]; kv[1] += va[1] * va[1]; kv[2] += va[2] * va[2];
                    kv[3] += va[0] * va[1]; kv[4] += va[0] * va[2]; kv[5] += va[1] * va[2];
                }
                for (int c = 0; c < 6; ++c) sig[c] += (kv[c] + S[c]) / V;
                nS += 1;
            }
        }
    }

    memset(res, 0, sizeof(*res));
    res->Ecold = Ecold_total / N;
    if (status & ORC_NONFINITE) {
        res->P = res->P_se = res->P_rms = res->T = res->T_se = NAN;
        res->Epot_mean = res->drift = NAN;
        for (int c = 0; c < 6; ++c) res->stress[c] = NAN;
    } else {
        orc_block_stats(sch->n_avg, Pser, sch->n_blocks, &res->P, &res->P_se);
        orc_block_stats(sch->n_avg, Tser, sch->n_blocks, &res->T, &res->T_se);
        double acc = 0.0;
        for (int k = 0; k < sch->n_avg; ++k) acc += (Pser[k] - res->P) * (Pser[k] - res->P);
        res->P_rms = sqrt(acc / sch->n_avg);
        res->Epot_mean = nU > 0 ? sumU / nU / N : NAN;
        res->drift = (E_n - E_w0) / N;
        if (!nvt && fabs(res->drift) > sch->drift_tol) status |= ORC_DRIFT;
        res->n_samples = sch->n_avg;
        for (int c = 0; c < 6; ++c) res->stress[c] = nS > 0 ? sig[c] / nS : NAN;
    }
    res->status = status;
    free(F);
    free(Pser);
    free(Tser);
    free(beta);
    free(Fold);
}
