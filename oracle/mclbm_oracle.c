/*
 * FP64 CPU oracle for the two-component pseudopotential lattice Boltzmann step
 * (Sedahmed et al., "Study of fluid displacement in three-dimensional porous
 * media with an improved multi-component pseudopotential lattice Boltzmann
 * method", Phys. Fluids 2022, arXiv 2207.01534).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct
 * reference that the HIP library is checked against.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it; the
 * product path never does.  It shares no code, header, table or constant with
 * the HIP library.
 *
 * Everything is double precision, two full population buffers, pull
 * streaming, naive loops, OpenMP over the (z, y) rows.  One step follows the paper's
 * model in this order:
 *   O1  component densities                    Sec. 2, Eq. (3)
 *   O2  virtual solid densities (IVSD)         Sec. 2, Eqs. (14)-(15) and the
 *                                              chi^(1)=1+xi, chi^(2)=1-xi rule
 *   O3  unified pseudopotential psi-hat        psi = rho (Eq. 11 text),
 *                                              s = phi * rho-tilde (Eq. 14)
 *   O4  total force per component              Eqs. (10), (11), (13)
 *   O5  common velocity                        Eqs. (4), (5), (8)
 *   O6  mixture relaxation time                Eqs. (6), (7)
 *   O7  forced SRT collision                   Eqs. (1), (2), (9)
 *   O8  streaming with halfway bounce-back     Eq. (1) left side; Sec. 3.2 and
 *                                              Sec. 4.1 (bounce-back at the
 *                                              fluid-solid interface)
 *
 * Readings taken where the paper is silent or garbled (each is listed with
 * its justification in the design notes of the repository):
 *   Eq. (7) sign: nu = c_s^2 (tau - 1/2).  Only the minus sign turns the
 *     printed relaxation-time pairs (3.5, 0.62) into the stated M = 25.
 *   Eq. (8): tau_s is common to numerator and denominator and cancels, so the
 *     equilibrium velocity is the barycentric one.
 *   Half-force shift: the common velocity used in f^eq, in S_i and reported
 *     as u includes + (F^(1)+F^(2)) / (2 rho).  With it every collision adds
 *     exactly F^tot of momentum at every node (the Guo forcing identity); the
 *     switch `half_force_shift = 0` gives the as-printed variant.
 *   psi at solid nodes in Eq. (11) is zero; solid neighbours enter only via
 *     Eq. (13), so one unified field psi-hat carries both sums.
 *   A solid node with no fluid neighbour (Eq. 15 denominator zero) gets
 *     rho-tilde = 0; no fluid node ever reads it.
 *   The same G_coh multiplies Eqs. (11) and (13).
 *   The body force is F^(sigma),b = rho^(sigma) g^(sigma).
 *   Eq. (12) sums over ordered pairs: P = c_s^2 rho + c_s^2 G rho1 rho2.
 *
 * Layout: populations f[sigma][i][idx], idx = x + nx*(y + ny*z), x fastest.
 * Fields: rho[sigma][idx], F[sigma][axis][idx], u[axis][idx].
 * Solid mask: uint8, nonzero = solid.  All directions are periodic unless
 * open_x is set.
 *
 * Open inlet/outlet planes (open_x = 1; Sec. 2, the inlet and outlet
 * conditions, and Sec. 4.1): x is not periodic; x = 0 is the inlet plane,
 * x = nx-1 the outlet plane (both must be fluid, as must x = 1 and x = nx-2).
 *   - Force sums at a boundary plane: a neighbour outside the domain takes
 *     psi-hat from its mirror image across the plane (x + e_i with the x
 *     component of e_i reversed), the pairing printed after Eq. (11).
 *   - IVSD sums skip neighbours outside the domain.
 *   - Streaming leaves the populations that would arrive from outside unset;
 *     after streaming each boundary node is rebuilt:
 *       inlet, component 1: non-equilibrium extrapolation (NEEM) to the
 *         imposed density rho_in from the neighbour x_f = (1, y, z):
 *         f_i = f_i(x_f) + feq_i(rho_in, u_f) - feq_i(rho1(x_f), u_f),
 *         u_f = (sum_sigma sum_i e_i f_i(x_f)) / (rho1 + rho2)(x_f);
 *       inlet, component 2: the five populations with e_x = +1 keep the
 *         values held in `frozen` (the initial state);
 *       outlet: the same with the roles swapped (component 2 to rho_out
 *         from x_f = (nx-2, y, z); component 1's e_x = -1 populations held).
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define Q 19
#define NC 2

typedef struct {
    int32_t nx, ny, nz;
    int32_t half_force_shift; /* 1: u includes +F/(2 rho) (default reading) */
    double tau[2];            /* tau^(1), tau^(2) */
    double G;                 /* G_coh, Eqs. (11) and (13) */
    double g[2][3];           /* body acceleration per component */
    int32_t open_x;           /* 1: open inlet (x = 0) and outlet (x = nx-1) planes */
    double rho_in;            /* component-1 density imposed at the inlet plane */
    double rho_out;           /* component-2 density imposed at the outlet plane */
    const double *frozen;     /* [2][Q][ny*nz]: populations held at the inlet
                                 (side 0, component 2) and outlet (side 1,
                                 component 1); only the entering directions used */
} orc_params;

/* D3Q19 velocity set and weights exactly as printed under Eq. (2). */
static const int EX[Q] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
static const int EY[Q] = {0, 0, 0, 1, -1, 0, 0, 1, 1, -1, -1, 0, 0, 0, 0, 1, -1, 1, -1};
static const int EZ[Q] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, 1, -1, -1, 1, 1, -1, -1};
static const double W[Q] = {1.0 / 3.0,
                            1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0,
                            1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0,
                            1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
static const double CS2 = 1.0 / 3.0; /* c_s^2 with dx = dt = 1 */

/* The opposite direction is found by search, not tabulated. */
static int opposite(int i)
{
    for (int k = 0; k < Q; ++k)
        if (EX[k] == -EX[i] && EY[k] == -EY[i] && EZ[k] == -EZ[i]) return k;
    return -1;
}

static size_t node(const orc_params *p, int x, int y, int z)
{
    return (size_t)x + (size_t)p->nx * ((size_t)y + (size_t)p->ny * (size_t)z);
}

/* Coordinate c + d on a periodic axis of length n, for |d| <= 1. */
static int wrap(int c, int d, int n)
{
    int v = c + d;
    if (v < 0) v += n;
    if (v >= n) v -= n;
    return v;
}

/* Periodic neighbour of (x,y,z) along direction i, scaled by sgn (+1 or -1). */
static size_t neighbour(const orc_params *p, int x, int y, int z, int i, int sgn)
{
    return node(p, wrap(x, sgn * EX[i], p->nx), wrap(y, sgn * EY[i], p->ny),
                wrap(z, sgn * EZ[i], p->nz));
}

/* 1 if x + sgn * e_i leaves the domain through an open x plane. */
static int outside(const orc_params *p, int x, int i, int sgn)
{
    int v = x + sgn * EX[i];
    return p->open_x && (v < 0 || v >= p->nx);
}

/* The node whose psi-hat stands in for x + e_i: the neighbour itself, or
 * across an open plane its mirror image (x component of e_i reversed). */
static size_t psi_neighbour(const orc_params *p, int x, int y, int z, int i)
{
    if (outside(p, x, i, +1))
        return node(p, x - EX[i], wrap(y, EY[i], p->ny), wrap(z, EZ[i], p->nz));
    return neighbour(p, x, y, z, i, +1);
}

static size_t nnodes(const orc_params *p) { return (size_t)p->nx * p->ny * p->nz; }

/* ---- per-node building blocks --------------------------------------- */

void orc_lattice(int32_t e_out[3 * Q], double w_out[Q], int32_t opp_out[Q])
{
    for (int i = 0; i < Q; ++i) {
        e_out[3 * i + 0] = EX[i];
        e_out[3 * i + 1] = EY[i];
        e_out[3 * i + 2] = EZ[i];
        w_out[i] = W[i];
        opp_out[i] = opposite(i);
    }
}

/* Eq. (7), minus-sign reading. */
double orc_viscosity(double tau) { return CS2 * (tau - 0.5); }

/* Eq. (6) with Eq. (7): mixture relaxation time. */
double orc_mixture_tau(const orc_params *p, double rho1, double rho2)
{
    double rho = rho1 + rho2;
    double nu = rho1 * orc_viscosity(p->tau[0]) + rho2 * orc_viscosity(p->tau[1]);
    return nu / (rho * CS2) + 0.5;
}

/* Eq. (2): second-order equilibrium of one component. */
void orc_equilibrium(double rho, const double u[3], double feq[Q])
{
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    for (int i = 0; i < Q; ++i) {
        double eu = EX[i] * u[0] + EY[i] * u[1] + EZ[i] * u[2];
        feq[i] = W[i] * rho * (1.0 + eu / CS2 + (eu * eu) / (2.0 * CS2 * CS2) - uu / (2.0 * CS2));
    }
}

/* Eq. (9): forcing source of one component. */
void orc_source(const double u[3], const double F[3], double S[Q])
{
    for (int i = 0; i < Q; ++i) {
        double e[3] = {EX[i], EY[i], EZ[i]};
        double eu = e[0] * u[0] + e[1] * u[1] + e[2] * u[2];
        double acc = 0.0;
        for (int a = 0; a < 3; ++a)
            acc += ((e[a] - u[a]) / CS2 + eu / (CS2 * CS2) * e[a]) * F[a];
        S[i] = W[i] * acc;
    }
}

/* Eq. (1) right side at one node: post-collision population. */
static double collide_one(double f, double feq, double S, double tau_s)
{
    return f - (f - feq) / tau_s + (1.0 - 1.0 / (2.0 * tau_s)) * S;
}

/* ---- lattice-wide phases ------------------------------------------- */

/* O1, Eq. (3): rho[s][idx]; zero at solid nodes. */
void orc_densities(const orc_params *p, const uint8_t *solid, const double *f, double *rho)
{
    size_t N = nnodes(p);
#pragma omp parallel for collapse(2) schedule(static)
    for (int z = 0; z < p->nz; ++z)
        for (int y = 0; y < p->ny; ++y)
            for (int x = 0; x < p->nx; ++x) {
                size_t n = node(p, x, y, z);
                for (int s = 0; s < NC; ++s) {
                    double r = 0.0;
                    if (!solid[n])
                        for (int i = 0; i < Q; ++i) r += f[((size_t)s * Q + i) * N + n];
                    rho[(size_t)s * N + n] = r;
                }
            }
}

/* O2-O3, Eqs. (14)-(15): unified pseudopotential psi[s][idx]. */
void orc_pseudopotential(const orc_params *p, const uint8_t *solid, const double *xi,
                         const double *rho, double *psi)
{
    size_t N = nnodes(p);
#pragma omp parallel for collapse(2) schedule(static)
    for (int z = 0; z < p->nz; ++z)
        for (int y = 0; y < p->ny; ++y)
            for (int x = 0; x < p->nx; ++x) {
                size_t n = node(p, x, y, z);
                if (!solid[n]) {
                    for (int s = 0; s < NC; ++s) psi[(size_t)s * N + n] = rho[(size_t)s * N + n];
                    continue;
                }
                double den = 0.0, num[NC] = {0.0, 0.0};
                for (int i = 1; i < Q; ++i) {
                    if (outside(p, x, i, +1)) continue;
                    size_t m = neighbour(p, x, y, z, i, +1);
                    double fluid = solid[m] ? 0.0 : 1.0; /* 1 - phi */
                    den += W[i] * fluid;
                    for (int s = 0; s < NC; ++s) num[s] += W[i] * rho[(size_t)s * N + m] * fluid;
                }
                double chi[NC] = {1.0 + xi[n], 1.0 - xi[n]};
                for (int s = 0; s < NC; ++s)
                    psi[(size_t)s * N + n] = den > 0.0 ? chi[s] * num[s] / den : 0.0;
            }
}

/* O4, Eqs. (10), (11), (13): F[s][a][idx] at fluid nodes, zero at solid. */
void orc_forces(const orc_params *p, const uint8_t *solid, const double *rho, const double *psi,
                double *F)
{
    size_t N = nnodes(p);
#pragma omp parallel for collapse(2) schedule(static)
    for (int z = 0; z < p->nz; ++z)
        for (int y = 0; y < p->ny; ++y)
            for (int x = 0; x < p->nx; ++x) {
                size_t n = node(p, x, y, z);
                for (int s = 0; s < NC; ++s) {
                    int sb = 1 - s; /* the other component */
                    double sum[3] = {0.0, 0.0, 0.0};
                    if (!solid[n])
                        for (int i = 1; i < Q; ++i) {
                            size_t m = psi_neighbour(p, x, y, z, i);
                            double ps = psi[(size_t)sb * N + m];
                            sum[0] += W[i] * ps * EX[i];
                            sum[1] += W[i] * ps * EY[i];
                            sum[2] += W[i] * ps * EZ[i];
                        }
                    double r = rho[(size_t)s * N + n];
                    for (int a = 0; a < 3; ++a)
                        F[((size_t)s * 3 + a) * N + n] =
                            solid[n] ? 0.0 : -p->G * r * sum[a] + r * p->g[s][a];
                }
            }
}

/* O5, Eqs. (4), (5), (8): common velocity u[a][idx]; zero at solid. */
void orc_velocity(const orc_params *p, const uint8_t *solid, const double *f, const double *rho,
                  const double *F, double *u)
{
    size_t N = nnodes(p);
#pragma omp parallel for collapse(2) schedule(static)
    for (int z = 0; z < p->nz; ++z)
        for (int y = 0; y < p->ny; ++y)
            for (int x = 0; x < p->nx; ++x) {
                size_t n = node(p, x, y, z);
                double mom[3] = {0.0, 0.0, 0.0}, rt = 0.0;
                if (!solid[n]) {
                    for (int s = 0; s < NC; ++s) {
                        rt += rho[(size_t)s * N + n];
                        for (int i = 0; i < Q; ++i) {
                            double fi = f[((size_t)s * Q + i) * N + n];
                            mom[0] += EX[i] * fi;
                            mom[1] += EY[i] * fi;
                            mom[2] += EZ[i] * fi;
                        }
                        if (p->half_force_shift)
                            for (int a = 0; a < 3; ++a) mom[a] += 0.5 * F[((size_t)s * 3 + a) * N + n];
                    }
                }
                for (int a = 0; a < 3; ++a) u[(size_t)a * N + n] = solid[n] ? 0.0 : mom[a] / rt;
            }
}

/* Eq. (12), ordered-pair reading: P[idx]; zero at solid. */
void orc_pressure(const orc_params *p, const uint8_t *solid, const double *rho, double *P)
{
    size_t N = nnodes(p);
    for (size_t n = 0; n < N; ++n) {
        double r1 = rho[n], r2 = rho[N + n];
        double pairs = r1 * r2 + r2 * r1; /* sum over (sigma, sigma-bar) */
        P[n] = solid[n] ? 0.0 : CS2 * (r1 + r2) + 0.5 * CS2 * p->G * pairs;
    }
}

/* Macroscopic fields of the state f at one time level (readouts). */
void orc_fields(const orc_params *p, const uint8_t *solid, const double *xi, const double *f,
                double *rho, double *psi, double *F, double *u)
{
    orc_densities(p, solid, f, rho);
    orc_pseudopotential(p, solid, xi, rho, psi);
    orc_forces(p, solid, rho, psi, F);
    orc_velocity(p, solid, f, rho, F, u);
}

/* Initial state: f_i = w_i rho^(sigma) (zero velocity); zero at solid. */
void orc_init_equilibrium(const orc_params *p, const uint8_t *solid, const double *rho, double *f)
{
    size_t N = nnodes(p);
    const double zero[3] = {0.0, 0.0, 0.0};
    for (size_t n = 0; n < N; ++n)
        for (int s = 0; s < NC; ++s) {
            double feq[Q];
            orc_equilibrium(solid[n] ? 0.0 : rho[(size_t)s * N + n], zero, feq);
            for (int i = 0; i < Q; ++i) f[((size_t)s * Q + i) * N + n] = feq[i];
        }
}

/*
 * Open-plane rebuild after streaming (open_x): NEEM for the imposed component
 * and the held populations of the other one, at every fluid node of the
 * inlet (x = 0) and outlet (x = nx-1) planes.
 */
void orc_open_rebuild(const orc_params *p, const uint8_t *solid, double *f)
{
    size_t N = nnodes(p);
    size_t A = (size_t)p->ny * p->nz;
    for (int side = 0; side < 2; ++side) {
        int xb = side ? p->nx - 1 : 0;
        int xf = side ? p->nx - 2 : 1;
        int sig = side ? 1 : 0;                 /* imposed component */
        int held = 1 - sig;                      /* component with held populations */
        int dir_in = side ? -1 : +1;             /* e_x of the entering directions */
        double rho_b = side ? p->rho_out : p->rho_in;
        for (int z = 0; z < p->nz; ++z)
            for (int y = 0; y < p->ny; ++y) {
                size_t nb = node(p, xb, y, z), nf = node(p, xf, y, z);
                if (solid[nb]) continue;
                double rf[NC] = {0.0, 0.0}, j[3] = {0.0, 0.0, 0.0};
                for (int s = 0; s < NC; ++s)
                    for (int i = 0; i < Q; ++i) {
                        double fi = f[((size_t)s * Q + i) * N + nf];
                        rf[s] += fi;
                        j[0] += EX[i] * fi;
                        j[1] += EY[i] * fi;
                        j[2] += EZ[i] * fi;
                    }
                double uf[3] = {j[0] / (rf[0] + rf[1]), j[1] / (rf[0] + rf[1]), j[2] / (rf[0] + rf[1])};
                double eb[Q], ef[Q];
                orc_equilibrium(rho_b, uf, eb);
                orc_equilibrium(rf[sig], uf, ef);
                for (int i = 0; i < Q; ++i)
                    f[((size_t)sig * Q + i) * N + nb] = f[((size_t)sig * Q + i) * N + nf] + eb[i] - ef[i];
                size_t a = (size_t)y + (size_t)p->ny * z;
                for (int i = 0; i < Q; ++i)
                    if (EX[i] == dir_in)
                        f[((size_t)held * Q + i) * N + nb] = p->frozen[((size_t)side * Q + i) * A + a];
            }
    }
}

/*
 * One time step, O1-O8.  f_in holds f(t) and is overwritten by the
 * post-collision populations; f_out receives f(t+1).  The scratch field
 * arrays (rho 2N, psi 2N, F 6N, u 3N) are caller-provided so that the last
 * step's fields can be inspected.
 */
void orc_step(const orc_params *p, const uint8_t *solid, const double *xi, double *f_in,
              double *f_out, double *rho, double *psi, double *F, double *u)
{
    size_t N = nnodes(p);
    orc_fields(p, solid, xi, f_in, rho, psi, F, u);

    /* O6-O7: collision in place at fluid nodes. */
#pragma omp parallel for collapse(2) schedule(static)
    for (int z = 0; z < p->nz; ++z)
        for (int y = 0; y < p->ny; ++y)
            for (int x = 0; x < p->nx; ++x) {
                size_t n = node(p, x, y, z);
                if (solid[n]) continue;
                double r1 = rho[n], r2 = rho[N + n];
                double tau_s = orc_mixture_tau(p, r1, r2);
                double uu[3] = {u[n], u[N + n], u[2 * N + n]};
                for (int s = 0; s < NC; ++s) {
                    double Fs[3] = {F[((size_t)s * 3 + 0) * N + n], F[((size_t)s * 3 + 1) * N + n],
                                    F[((size_t)s * 3 + 2) * N + n]};
                    double feq[Q], S[Q];
                    orc_equilibrium(rho[(size_t)s * N + n], uu, feq);
                    orc_source(uu, Fs, S);
                    for (int i = 0; i < Q; ++i) {
                        double *fi = &f_in[((size_t)s * Q + i) * N + n];
                        *fi = collide_one(*fi, feq[i], S[i], tau_s);
                    }
                }
            }

    /* O8: pull streaming with halfway bounce-back; solid nodes hold zeros. */
    int opp[Q];
    for (int i = 0; i < Q; ++i) opp[i] = opposite(i);
#pragma omp parallel for collapse(2) schedule(static)
    for (int z = 0; z < p->nz; ++z)
        for (int y = 0; y < p->ny; ++y)
            for (int x = 0; x < p->nx; ++x) {
                size_t n = node(p, x, y, z);
                for (int s = 0; s < NC; ++s)
                    for (int i = 0; i < Q; ++i) {
                        double v = 0.0;
                        if (!solid[n] && !outside(p, x, i, -1)) {
                            size_t src = neighbour(p, x, y, z, i, -1);
                            if (!solid[src])
                                v = f_in[((size_t)s * Q + i) * N + src];
                            else
                                v = f_in[((size_t)s * Q + opp[i]) * N + n];
                        }
                        f_out[((size_t)s * Q + i) * N + n] = v;
                    }
            }
    if (p->open_x) orc_open_rebuild(p, solid, f_out);
}

/*
 * nsteps steps starting from fa; the buffers alternate.  Returns 0 if the
 * final state is in fa and 1 if it is in fb.  The field arrays hold the
 * fields of the last step's starting state.
 */
int32_t orc_run(const orc_params *p, const uint8_t *solid, const double *xi, double *fa, double *fb,
                int32_t nsteps, double *rho, double *psi, double *F, double *u)
{
    double *cur = fa, *nxt = fb;
    for (int32_t t = 0; t < nsteps; ++t) {
        orc_step(p, solid, xi, cur, nxt, rho, psi, F, u);
        double *tmp = cur;
        cur = nxt;
        nxt = tmp;
    }
    return cur == fa ? 0 : 1;
}

/*
 * Diagnostics of a state (Sec. 4.1 water saturation and mass sums):
 *   out[0], out[1]: component masses over fluid nodes
 *   out[2]: S_w = fraction of fluid nodes where rho^(2) > rho^(1)
 *           (component 2 is the water / wetting phase; ties count as oil)
 *   out[3]: smooth non-wetting fraction, mean of rho1/(rho1+rho2)
 *   out[4]: max |u| over fluid nodes
 *   out[5]: number of non-finite population values at fluid nodes
 */
void orc_diagnostics(const orc_params *p, const uint8_t *solid, const double *f, const double *rho,
                     const double *u, double out[6])
{
    size_t N = nnodes(p);
    double m1 = 0.0, m2 = 0.0, nw = 0.0, snw = 0.0, nf = 0.0, umax = 0.0, bad = 0.0;
    for (size_t n = 0; n < N; ++n) {
        if (solid[n]) continue;
        double r1 = rho[n], r2 = rho[N + n];
        m1 += r1;
        m2 += r2;
        nf += 1.0;
        if (r2 > r1) nw += 1.0;
        snw += r1 / (r1 + r2);
        double um = sqrt(u[n] * u[n] + u[N + n] * u[N + n] + u[2 * N + n] * u[2 * N + n]);
        if (um > umax) umax = um;
        for (int s = 0; s < NC; ++s)
            for (int i = 0; i < Q; ++i)
                if (!isfinite(f[((size_t)s * Q + i) * N + n])) bad += 1.0;
    }
    out[0] = m1;
    out[1] = m2;
    out[2] = nf > 0 ? nw / nf : 0.0;
    out[3] = nf > 0 ? snw / nf : 0.0;
    out[4] = umax;
    out[5] = bad;
}

/*
 * Smooth non-wetting saturation over a region (the differentiable loss):
 * L = (1/|R|) sum over fluid x in R of rho1/(rho1+rho2).
 */
double orc_loss_snw(const orc_params *p, const uint8_t *solid, const uint8_t *region,
                    const double *f)
{
    size_t N = nnodes(p);
    double acc = 0.0, cnt = 0.0;
    for (size_t n = 0; n < N; ++n) {
        if (solid[n] || !region[n]) continue;
        double r[NC] = {0.0, 0.0};
        for (int s = 0; s < NC; ++s)
            for (int i = 0; i < Q; ++i) r[s] += f[((size_t)s * Q + i) * N + n];
        acc += r[0] / (r[0] + r[1]);
        cnt += 1.0;
    }
    return cnt > 0 ? acc / cnt : 0.0;
}

/* Number of OpenMP threads the lattice-wide loops use (1 without OpenMP). */
int32_t orc_num_threads(void)
{
#ifdef _OPENMP
    return (int32_t)omp_get_max_threads();
#else
    return 1;
#endif
}

/* Set the number of OpenMP threads of later calls (ignored without OpenMP). */
void orc_set_num_threads(int32_t n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads((int)n);
#else
    (void)n;
#endif
}
