/*
 * Plain FP64 CPU oracle for the multi-component Shan-Chen lattice Boltzmann
 * method with a coupled reactive advection-diffusion solute (CooLBM,
 * arXiv 2502.12955).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct
 * statement of what one time step computes.  Only the test suite, the smoke
 * check and the CPU-baseline leg of the benchmark may load it.  It shares no
 * code, header, table or constant with the HIP library: every lattice table
 * and every formula below is written out again from the paper.
 *
 * Notation follows the paper:
 *   f^s_i   flow populations of component s (s = 0..ncomp-1), i over D2Q9/D3Q19
 *   h_k     solute populations, k over D2Q5/D3Q7
 *   rho_s   component density, psi_s pseudo-potential, F^s total force
 *   u       barycentric velocity, tau_s, tau_d relaxation times
 *
 *   h_{k,CO2} populations of the optional product species (eq:reactCO2)
 *
 * Layout: node index n = x + nx*(y + ny*z); f[(s*Q + i)*N + n]; h[(sp*QS + k)*N + n]
 * for solute species sp (0: the reacting species O2, 1: the product CO2).
 * Solid nodes carry no populations (their slots are left untouched).
 *
 * Readings taken where the paper is silent or ambiguous:
 *   - psi of a solid node is 0; walls act only through the adhesion force.
 *   - Guo forcing is one option, the Shan-Chen velocity shift the other.
 *   - body force on component s is rho_s * accel.
 *   - D3Q7 solute lattice: rest weight J0, link weights (1-J0)/6; the 2-D
 *     D2Q5 lattice: J0 and (1-J0)/4.  Solute c_s^2 = sum_k W_k e_kx^2.
 *   - the solute is advected by the barycentric velocity with half force.
 *   - the wet-node reaction is applied per missing link.
 *   - the product is created at every reacting link at the O2 consumption
 *     rate k C_b of that link (one CO2 per O2, eq:react), entering through
 *     the link in the product's own flux convention.
 *   - inlet (x = 0) anti-bounce-back Dirichlet, outlet (x = nx-1) zero
 *     gradient, when the solute runs in inlet/outlet mode.
 *   - fluid voxels pinched between two solids along one axis are made solid
 *     before anything else (in inlet/outlet mode the planes beyond x = 0 and
 *     x = nx-1 count as solid for this test).
 *   - conjugate heat transfer: interface nodes are fluid nodes with a solid
 *     flow-lattice neighbour and carry both energy distributions; the
 *     counter-slip conditions are posed per node over its unknown links
 *     (details with orc_step_thermal below).
 *   - particle deposition: "near the substrate" means a solid neighbour along
 *     any flow-lattice link; the deposit does not remove particles from the
 *     fluid (the paper's update has no sink term); nodes that turn solid lose
 *     their populations, and the pinch rule is applied again afterwards.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int32_t lattice;   /* 0: D2Q9 flow + D2Q5 solute, 1: D3Q19 flow + D3Q7 solute */
    int32_t nx, ny, nz;
    int32_t ncomp;     /* 1 or 2 */
    int32_t forcing;   /* 0: Guo, 1: Shan-Chen velocity shift */
    int32_t solute;    /* 0: off, 1: periodic, 2: inlet at x=0 / outlet at x=nx-1 */
    int32_t pad_;
    double tau[2];
    double G[2][2];
    double G_ads[2];
    double rho0;
    double accel[3];
    double D, J0, k_wall, C_in;
    int32_t product;   /* 1: a second species (CO2) produced at the reacting walls */
    int32_t pad2_;
    double D2, C_in2;  /* its diffusivity and inlet concentration */
    const double* k_node; /* per-node reaction rate [N] (e.g. A exp(-E / R_u T(x))), or NULL: k_wall */
} orc_params;

/* ---------------------------------------------------------------------------
 * Lattice tables, typed in from the paper's tables of velocities and weights
 * (subsection "3D and 2D LBM Models"): D3Q19, D2Q9 (with w_4 = 1/9, the
 * printed 1/36 being inconsistent with normalisation), D2Q5.  D3Q7 takes the
 * first seven D3Q19 vectors.
 * ------------------------------------------------------------------------- */
static const int D3Q19_C[19][3] = {
    {0, 0, 0},
    {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1},
    {1, 1, 0}, {-1, -1, 0}, {1, 0, 1}, {-1, 0, -1}, {0, 1, 1}, {0, -1, -1},
    {1, -1, 0}, {-1, 1, 0}, {1, 0, -1}, {-1, 0, 1}, {0, 1, -1}, {0, -1, 1}};
static const double D3Q19_W[19] = {
    1.0 / 3.0,
    1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0,
    1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0,
    1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
static const int D2Q9_C[9][3] = {
    {0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {-1, 0, 0}, {0, -1, 0},
    {1, 1, 0}, {-1, 1, 0}, {-1, -1, 0}, {1, -1, 0}};
static const double D2Q9_W[9] = {
    4.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0,
    1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
static const int D2Q5_C[5][3] = {{0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {-1, 0, 0}, {0, -1, 0}};
static const int D3Q7_C[7][3] = {
    {0, 0, 0}, {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1}};

/* Speed of sound squared of the flow lattices (both D2Q9 and D3Q19). */
#define CS2 (1.0 / 3.0)

typedef struct {
    int Q;
    const int (*c)[3];
    const double* w;
    int opp[19];
} flow_lat;

typedef struct {
    int Q;
    const int (*c)[3];
    double w[7];
    double cs2;
    int opp[7];
} sol_lat;

static void fill_opp(int Q, const int (*c)[3], int* opp) {
    for (int i = 0; i < Q; ++i)
        for (int j = 0; j < Q; ++j)
            if (c[j][0] == -c[i][0] && c[j][1] == -c[i][1] && c[j][2] == -c[i][2]) opp[i] = j;
}

static flow_lat make_flow(int lattice) {
    flow_lat L;
    if (lattice == 1) { L.Q = 19; L.c = D3Q19_C; L.w = D3Q19_W; }
    else              { L.Q = 9;  L.c = D2Q9_C;  L.w = D2Q9_W; }
    fill_opp(L.Q, L.c, L.opp);
    return L;
}

static sol_lat make_sol(int lattice, double J0) {
    sol_lat S;
    if (lattice == 1) { S.Q = 7; S.c = D3Q7_C; }
    else              { S.Q = 5; S.c = D2Q5_C; }
    S.w[0] = J0;
    for (int k = 1; k < S.Q; ++k) S.w[k] = (1.0 - J0) / (double)(S.Q - 1);
    S.cs2 = 0.0;
    for (int k = 0; k < S.Q; ++k) S.cs2 += S.w[k] * S.c[k][0] * S.c[k][0];
    fill_opp(S.Q, S.c, S.opp);
    return S;
}

/* Threads of the OpenMP loops (the CPU-baseline leg times one thread and all
 * host cores); returns the count now in effect. */
#ifdef _OPENMP
#include <omp.h>
#endif
int orc_set_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}

/* Table export for the tests (velocities as int[Q][3], weights, opposites). */
int orc_flow_lattice(int lattice, int* c, double* w, int* opp) {
    flow_lat L = make_flow(lattice);
    for (int i = 0; i < L.Q; ++i) {
        for (int a = 0; a < 3; ++a) c[3 * i + a] = L.c[i][a];
        w[i] = L.w[i];
        opp[i] = L.opp[i];
    }
    return L.Q;
}

int orc_solute_lattice(int lattice, double J0, int* c, double* w, int* opp, double* cs2) {
    sol_lat S = make_sol(lattice, J0);
    for (int k = 0; k < S.Q; ++k) {
        for (int a = 0; a < 3; ++a) c[3 * k + a] = S.c[k][a];
        w[k] = S.w[k];
        opp[k] = S.opp[k];
    }
    *cs2 = S.cs2;
    return S.Q;
}

/* ---------------------------------------------------------------------------
 * Local formulas
 * ------------------------------------------------------------------------- */

/* Second-order equilibrium, eq:6: w_i rho [1 + c.v/cs2 + ((c.v)^2 - cs2 v.v)/(2 cs2^2)]. */
static double feq_i(const flow_lat* L, int i, double rho, const double v[3]) {
    double cu = L->c[i][0] * v[0] + L->c[i][1] * v[1] + L->c[i][2] * v[2];
    double uu = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
    return L->w[i] * rho * (1.0 + cu / CS2 + (cu * cu - CS2 * uu) / (2.0 * CS2 * CS2));
}

/* Guo forcing term, eq:1.21: w_i [c_a/cs2 + (c_a c_b - cs2 d_ab) u_b/cs2^2] F_a. */
static double guo_i(const flow_lat* L, int i, const double F[3], const double u[3]) {
    double cF = L->c[i][0] * F[0] + L->c[i][1] * F[1] + L->c[i][2] * F[2];
    double cu = L->c[i][0] * u[0] + L->c[i][1] * u[1] + L->c[i][2] * u[2];
    double uF = u[0] * F[0] + u[1] * F[1] + u[2] * F[2];
    return L->w[i] * (cF / CS2 + (cF * cu - CS2 * uF) / (CS2 * CS2));
}

/* Pseudo-potential, eq:1.11 / pseudo-potential_multicomponent. */
static double psi_of(double rho, double rho0) { return rho0 * (1.0 - exp(-rho / rho0)); }

/* Solute equilibrium, eq:therpopeq_species: W_k C (1 + e_k.u / cs2). */
static double heq_k(const sol_lat* S, int k, double C, const double u[3]) {
    double eu = S->c[k][0] * u[0] + S->c[k][1] * u[1] + S->c[k][2] * u[2];
    return S->w[k] * C * (1.0 + eu / S->cs2);
}

void orc_feq(int lattice, double rho, const double* v, double* out) {
    flow_lat L = make_flow(lattice);
    for (int i = 0; i < L.Q; ++i) out[i] = feq_i(&L, i, rho, v);
}

void orc_guo(int lattice, const double* F, const double* u, double* out) {
    flow_lat L = make_flow(lattice);
    for (int i = 0; i < L.Q; ++i) out[i] = guo_i(&L, i, F, u);
}

double orc_psi(double rho, double rho0) { return psi_of(rho, rho0); }

/* ---------------------------------------------------------------------------
 * Grid helpers
 * ------------------------------------------------------------------------- */
static int64_t nnodes(const orc_params* p) { return (int64_t)p->nx * p->ny * p->nz; }

static int wrap(int a, int n) { return ((a % n) + n) % n; }

static int64_t idx(const orc_params* p, int x, int y, int z) {
    return (int64_t)x + (int64_t)p->nx * ((int64_t)y + (int64_t)p->ny * z);
}

static void coords(const orc_params* p, int64_t n, int* x, int* y, int* z) {
    *x = (int)(n % p->nx);
    *y = (int)((n / p->nx) % p->ny);
    *z = (int)(n / ((int64_t)p->nx * p->ny));
}

/* Periodic neighbour x + d. */
static int64_t nbr(const orc_params* p, int64_t n, const int d[3]) {
    int x, y, z;
    coords(p, n, &x, &y, &z);
    return idx(p, wrap(x + d[0], p->nx), wrap(y + d[1], p->ny), wrap(z + d[2], p->nz));
}

/* Periodic neighbour x - d. */
static int64_t nbr_back(const orc_params* p, int64_t n, const int d[3]) {
    int m[3] = {-d[0], -d[1], -d[2]};
    return nbr(p, n, m);
}

/* ---------------------------------------------------------------------------
 * Geometry: pinch-fill to a fixed point, then link masks.
 * A fluid voxel is "pinched" when along some axis both neighbours are
 * blocked (solid, or beyond the x-seams in solute inlet/outlet mode).
 * ------------------------------------------------------------------------- */
static int blocked(const orc_params* p, const uint8_t* mask, int x, int y, int z) {
    if (p->solute == 2 && (x < 0 || x >= p->nx)) return 1;
    return mask[idx(p, wrap(x, p->nx), wrap(y, p->ny), wrap(z, p->nz))] != 0;
}

int64_t orc_pinch_fill(const orc_params* p, uint8_t* mask) {
    int64_t N = nnodes(p), total = 0;
    int naxes = (p->lattice == 1) ? 3 : 2;
    uint8_t* add = (uint8_t*)malloc((size_t)N);
    for (;;) {
        int64_t changed = 0;
        memset(add, 0, (size_t)N);
        for (int64_t n = 0; n < N; ++n) {
            if (mask[n]) continue;
            int x, y, z;
            coords(p, n, &x, &y, &z);
            for (int a = 0; a < naxes; ++a) {
                int d[3] = {0, 0, 0};
                d[a] = 1;
                if (blocked(p, mask, x + d[0], y + d[1], z + d[2]) &&
                    blocked(p, mask, x - d[0], y - d[1], z - d[2])) {
                    add[n] = 1;
                    break;
                }
            }
        }
        for (int64_t n = 0; n < N; ++n)
            if (add[n]) { mask[n] = 1; ++changed; }
        total += changed;
        if (!changed) break;
    }
    free(add);
    return total;
}

/* Bit i of flow_bits[n] set iff fluid node n has solid upstream node n - c_i
 * (periodic); bit k of solute_bits[n] set iff the solute link k is a wet
 * (reactive) link: upstream n - e_k is solid and not across an x-seam in
 * inlet/outlet mode.  Solid nodes get 0. */
void orc_link_masks(const orc_params* p, const uint8_t* mask, uint32_t* flow_bits,
                    uint32_t* solute_bits) {
    flow_lat L = make_flow(p->lattice);
    sol_lat S = make_sol(p->lattice, p->J0);
    int64_t N = nnodes(p);
    for (int64_t n = 0; n < N; ++n) {
        uint32_t fb = 0, sb = 0;
        if (!mask[n]) {
            for (int i = 0; i < L.Q; ++i)
                if (mask[nbr_back(p, n, L.c[i])]) fb |= 1u << i;
            int x, y, z;
            coords(p, n, &x, &y, &z);
            for (int k = 0; k < S.Q; ++k) {
                int sx = x - S.c[k][0];
                if (p->solute == 2 && (sx < 0 || sx >= p->nx)) continue;
                if (mask[nbr_back(p, n, S.c[k])]) sb |= 1u << k;
            }
        }
        flow_bits[n] = fb;
        solute_bits[n] = sb;
    }
}

/* ---------------------------------------------------------------------------
 * Initialisation: f^s_i = f^eq_i(rho_s, u), h_k = h^eq_k(C, u), no force term.
 * rho: [ncomp][N]; u: [3][N] or NULL (rest); C: [N] or NULL (zero).
 * The product species (if on) starts at zero: h = 0 in its planes.
 * ------------------------------------------------------------------------- */
void orc_init(const orc_params* p, const uint8_t* mask, const double* rho, const double* u,
              const double* C, double* f, double* h) {
    flow_lat L = make_flow(p->lattice);
    sol_lat S = make_sol(p->lattice, p->J0);
    int64_t N = nnodes(p);
    for (int64_t n = 0; n < N; ++n) {
        if (mask[n]) continue;
        double v[3] = {0, 0, 0};
        if (u) { v[0] = u[n]; v[1] = u[N + n]; v[2] = u[2 * N + n]; }
        for (int s = 0; s < p->ncomp; ++s)
            for (int i = 0; i < L.Q; ++i) f[((int64_t)s * L.Q + i) * N + n] = feq_i(&L, i, rho[(int64_t)s * N + n], v);
        if (p->solute && h) {
            double c0 = C ? C[n] : 0.0;
            for (int k = 0; k < S.Q; ++k) h[(int64_t)k * N + n] = heq_k(&S, k, c0, v);
            if (p->product)
                for (int k = 0; k < S.Q; ++k) h[(int64_t)(S.Q + k) * N + n] = 0.0;   /* no product at t = 0 */
        }
    }
}

/* ---------------------------------------------------------------------------
 * Step pieces
 * ------------------------------------------------------------------------- */

/* Phase 1: densities (eq:1.7) and pseudo-potentials of every node; solid -> 0. */
static void densities(const orc_params* p, const flow_lat* L, const uint8_t* mask,
                      const double* f, double* rho, double* psi) {
    int64_t N = nnodes(p);
#pragma omp parallel for schedule(static)
    for (int64_t n = 0; n < N; ++n) {
        for (int s = 0; s < p->ncomp; ++s) {
            double r = 0.0;
            if (!mask[n])
                for (int i = 0; i < L->Q; ++i) r += f[((int64_t)s * L->Q + i) * N + n];
            rho[(int64_t)s * N + n] = r;
            psi[(int64_t)s * N + n] = mask[n] ? 0.0 : psi_of(r, p->rho0);
        }
    }
}

/* Total force on component s at fluid node n:
 *   cohesion   eq:1.14   -psi_s(x) sum_t G_st sum_i w_i psi_t(x+c_i) c_i
 *   adhesion   eq:1.15   -G_ads,s rho_s(x) sum_i w_i s(x+c_i) c_i
 *   body force           rho_s(x) accel                                    */
static void force_at(const orc_params* p, const flow_lat* L, const uint8_t* mask,
                     const double* rho, const double* psi, int64_t n, double F[2][3]) {
    int64_t N = nnodes(p);
    for (int s = 0; s < p->ncomp; ++s) {
        double coh[3] = {0, 0, 0}, ads[3] = {0, 0, 0};
        for (int i = 1; i < L->Q; ++i) {
            int64_t m = nbr(p, n, L->c[i]);
            double sumG = 0.0;
            for (int t = 0; t < p->ncomp; ++t) sumG += p->G[s][t] * psi[(int64_t)t * N + m];
            double solid = mask[m] ? 1.0 : 0.0;
            for (int a = 0; a < 3; ++a) {
                coh[a] += L->w[i] * sumG * L->c[i][a];
                ads[a] += L->w[i] * solid * L->c[i][a];
            }
        }
        double ps = psi[(int64_t)s * N + n], rs = rho[(int64_t)s * N + n];
        for (int a = 0; a < 3; ++a)
            F[s][a] = -ps * coh[a] - p->G_ads[s] * rs * ads[a] + rs * p->accel[a];
    }
}

/* Barycentric velocity with half force, eq:1.19 (also the "actual velocity"
 * of the Shan-Chen scheme). */
static void bary_u(const orc_params* p, const flow_lat* L, const double* f, int64_t n,
                   const double* rho, double F[2][3], double u[3]) {
    int64_t N = nnodes(p);
    double rt = 0.0, m[3] = {0, 0, 0};
    for (int s = 0; s < p->ncomp; ++s) {
        rt += rho[(int64_t)s * N + n];
        for (int i = 0; i < L->Q; ++i) {
            double fi = f[((int64_t)s * L->Q + i) * N + n];
            for (int a = 0; a < 3; ++a) m[a] += L->c[i][a] * fi;
        }
        for (int a = 0; a < 3; ++a) m[a] += 0.5 * F[s][a];
    }
    for (int a = 0; a < 3; ++a) u[a] = m[a] / rt;
}

/* Post-collision populations of node n (flow: eq:1.16 with Guo eq:1.19-1.21 or
 * Shan-Chen eq:1.17-1.18; solute: eq:therpop_species). */
static void collide_at(const orc_params* p, const flow_lat* L, const sol_lat* S,
                       const uint8_t* mask, const double* f, const double* h,
                       const double* rho, const double* psi, int64_t n,
                       double fs[2][19], double hs[14]) {
    int64_t N = nnodes(p);
    double F[2][3];
    force_at(p, L, mask, rho, psi, n, F);
    double u[3];
    bary_u(p, L, f, n, rho, F, u);

    double ueq[2][3];
    if (p->forcing == 0) {
        for (int s = 0; s < p->ncomp; ++s)
            for (int a = 0; a < 3; ++a) ueq[s][a] = u[a];
    } else {
        /* u' = sum_s (j_s / tau_s) / sum_s (rho_s / tau_s), u^eq_s = u' + tau_s F_s / rho_s */
        double num[3] = {0, 0, 0}, den = 0.0;
        for (int s = 0; s < p->ncomp; ++s) {
            double j[3] = {0, 0, 0};
            for (int i = 0; i < L->Q; ++i) {
                double fi = f[((int64_t)s * L->Q + i) * N + n];
                for (int a = 0; a < 3; ++a) j[a] += L->c[i][a] * fi;
            }
            for (int a = 0; a < 3; ++a) num[a] += j[a] / p->tau[s];
            den += rho[(int64_t)s * N + n] / p->tau[s];
        }
        for (int s = 0; s < p->ncomp; ++s)
            for (int a = 0; a < 3; ++a)
                ueq[s][a] = num[a] / den + p->tau[s] * F[s][a] / rho[(int64_t)s * N + n];
    }

    for (int s = 0; s < p->ncomp; ++s) {
        double tau = p->tau[s], rs = rho[(int64_t)s * N + n];
        double lam = 1.0 - 1.0 / (2.0 * tau);
        for (int i = 0; i < L->Q; ++i) {
            double fi = f[((int64_t)s * L->Q + i) * N + n];
            double src = (p->forcing == 0) ? guo_i(L, i, F[s], u) : 0.0;
            fs[s][i] = fi - (fi - feq_i(L, i, rs, ueq[s])) / tau + lam * src;
        }
    }

    if (p->solute) {
        /* species 0 (O2) and, with the product, species 1 (CO2): the same
         * collision (eq:therpop_species) with each species' own tau_d */
        for (int sp = 0; sp <= (p->product ? 1 : 0); ++sp) {
            double tau_d = (sp ? p->D2 : p->D) / S->cs2 + 0.5;
            double C = 0.0;
            for (int k = 0; k < S->Q; ++k) C += h[(int64_t)(sp * S->Q + k) * N + n];
            for (int k = 0; k < S->Q; ++k) {
                double hk = h[(int64_t)(sp * S->Q + k) * N + n];
                hs[sp * S->Q + k] = hk - (hk - heq_k(S, k, C, u)) / tau_d;
            }
        }
    }
}

/* Value of flow population i at fluid node y after streaming (eq:5 with
 * halfway bounce-back: a link whose upstream node is solid returns the
 * node's own post-collision population of the opposite direction). */
static double flow_stream_value(const orc_params* p, const flow_lat* L, const uint8_t* mask,
                                const double* fstar, int s, int i, int64_t y) {
    int64_t N = nnodes(p);
    int64_t src = nbr_back(p, y, L->c[i]);
    if (mask[src]) return fstar[((int64_t)s * L->Q + L->opp[i]) * N + y];
    return fstar[((int64_t)s * L->Q + i) * N + src];
}

/* Reaction rate at the wall node y: the prescribed field, else the uniform k_wall. */
static double rate_at(const orc_params* p, int64_t y) { return p->k_node ? p->k_node[y] : p->k_wall; }

/* Value of solute population k of species sp at fluid node y after streaming.
 * Precedence: inlet/outlet seam > wet (reactive) link > plain pull.
 *   inlet  (x = 0, e_kx = +1):      h_k = 2 W_k C_in - h_kbar(y, t+1)
 *   outlet (x = nx-1, e_kx = -1):   h_k = h_k(nx-2, t+1) = h*_k(y)
 *   wet link (y - e_k solid), O2:   C_b = 2 h_in / (2 W_k + k tau/(tau - 1/2)),
 *                                   h_k = 2 W_k C_b - h_in,  h_in = h_kbar(y, t+1)
 *   wet link, product (CO2):        h_k = h_in + k tau2/(tau2 - 1/2) C_b
 * (eq:wetnode9 generalised to any missing link; the node sits on the wall.
 * The O2 rule moves k C_b out of the fluid through the link in the flux
 * convention (1 - 1/(2 tau)) (h_in - h_k); the product rule moves the same
 * k C_b in, eq:reactCO2, in its own species' convention.)
 * h_kbar(y, t+1) is always a plain value h*_kbar(y + e_k): pinch-fill
 * guarantees that y + e_k is a fluid node inside the domain. */
static double solute_stream_value(const orc_params* p, const sol_lat* S, const uint8_t* mask,
                                  const double* hstar, int sp, int k, int64_t y) {
    int64_t N = nnodes(p);
    int x, yy, z;
    coords(p, y, &x, &yy, &z);
    int kb = S->opp[k];
    int64_t base = (int64_t)sp * S->Q;
    if (p->solute == 2 && x == 0 && S->c[k][0] == 1) {
        double hin = hstar[(base + kb) * N + nbr(p, y, S->c[k])];
        return 2.0 * S->w[k] * (sp ? p->C_in2 : p->C_in) - hin;
    }
    if (p->solute == 2 && x == p->nx - 1 && S->c[k][0] == -1) {
        return hstar[(base + k) * N + y];
    }
    int64_t src = nbr_back(p, y, S->c[k]);
    if (mask[src]) {
        double tau_d = p->D / S->cs2 + 0.5;
        double hin0 = hstar[(int64_t)kb * N + nbr(p, y, S->c[k])];
        double kr = rate_at(p, y);
        double Cb = 2.0 * hin0 / (2.0 * S->w[k] + kr * tau_d / (tau_d - 0.5));
        if (sp == 0) return 2.0 * S->w[k] * Cb - hin0;
        double tau2 = p->D2 / S->cs2 + 0.5;
        double hin = hstar[(base + kb) * N + nbr(p, y, S->c[k])];
        return hin + kr * tau2 / (tau2 - 0.5) * Cb;
    }
    return hstar[(base + k) * N + src];
}

/* ---------------------------------------------------------------------------
 * One or more full time steps.  State: pre-collision populations at t.
 *   1. rho_s, psi_s of every node (densities of step t everywhere first)
 *   2. post-collision populations of every fluid node
 *   3. streaming (pull) with bounce-back, seams and wet links
 * ------------------------------------------------------------------------- */
void orc_step(const orc_params* p, const uint8_t* mask, double* f, double* h, int64_t nsteps) {
    flow_lat L = make_flow(p->lattice);
    sol_lat S = make_sol(p->lattice, p->J0);
    int64_t N = nnodes(p);
    int NC = p->ncomp;
    double* rho = (double*)calloc((size_t)(NC * N), sizeof(double));
    double* psi = (double*)calloc((size_t)(NC * N), sizeof(double));
    double* fstar = (double*)calloc((size_t)(NC * L.Q * N), sizeof(double));
    int NS = p->solute ? (p->product ? 2 : 1) : 0;   /* solute species */
    double* hstar = NS ? (double*)calloc((size_t)(NS * S.Q * N), sizeof(double)) : NULL;

    for (int64_t t = 0; t < nsteps; ++t) {
        densities(p, &L, mask, f, rho, psi);
#pragma omp parallel for schedule(static)
        for (int64_t n = 0; n < N; ++n) {
            if (mask[n]) continue;
            double fs[2][19], hs[14];
            collide_at(p, &L, &S, mask, f, h, rho, psi, n, fs, hs);
            for (int s = 0; s < NC; ++s)
                for (int i = 0; i < L.Q; ++i) fstar[((int64_t)s * L.Q + i) * N + n] = fs[s][i];
            for (int k = 0; k < NS * S.Q; ++k) hstar[(int64_t)k * N + n] = hs[k];
        }
#pragma omp parallel for schedule(static)
        for (int64_t n = 0; n < N; ++n) {
            if (mask[n]) continue;
            for (int s = 0; s < NC; ++s)
                for (int i = 0; i < L.Q; ++i)
                    f[((int64_t)s * L.Q + i) * N + n] = flow_stream_value(p, &L, mask, fstar, s, i, n);
            for (int sp = 0; sp < NS; ++sp)
                for (int k = 0; k < S.Q; ++k)
                    h[(int64_t)(sp * S.Q + k) * N + n] = solute_stream_value(p, &S, mask, hstar, sp, k, n);
        }
    }
    free(rho);
    free(psi);
    free(fstar);
    free(hstar);
}

/* ---------------------------------------------------------------------------
 * Particle deposition (sec:particle_deposition, eq:surface_deposition), applied
 * after a full step.  The reacting solute species (planes 0..QS-1 of h) is the
 * particle mass fraction C_p.
 *   1. every fluid node n next to the substrate (some flow-lattice neighbour
 *      n + c_i, i >= 1, is solid; periodic wrap) adds DP times the sum of its
 *      particle populations after streaming to its deposit:
 *        C_ps(n, t+1) = C_ps(n, t) + DP * sum_k h_k(n, t+1)
 *   2. every fluid node whose deposit exceeds 1 turns solid (all at once);
 *   3. the pinch rule of the geometry is applied again to the new mask;
 *   4. every node that turned solid in 2 or 3 loses its populations and its
 *      deposit (set to 0).
 * mask, f, h and Cps ([N]) are updated in place; returns the number of nodes
 * that turned solid.
 * ------------------------------------------------------------------------- */
int64_t orc_deposit(const orc_params* p, uint8_t* mask, double* f, double* h, double* Cps, double DP) {
    flow_lat L = make_flow(p->lattice);
    sol_lat S = make_sol(p->lattice, p->J0);
    int64_t N = nnodes(p);
    int NC = p->ncomp;
    int NS = p->solute ? (p->product ? 2 : 1) : 0;
    uint8_t* before = (uint8_t*)malloc((size_t)N);
    memcpy(before, mask, (size_t)N);
    for (int64_t n = 0; n < N; ++n) {
        if (before[n]) continue;
        int near = 0;
        for (int i = 1; i < L.Q; ++i)
            if (before[nbr(p, n, L.c[i])]) near = 1;
        if (!near) continue;
        double C = 0.0;
        for (int k = 0; k < S.Q; ++k) C += h[(int64_t)k * N + n];
        Cps[n] += DP * C;
    }
    for (int64_t n = 0; n < N; ++n)
        if (!before[n] && Cps[n] > 1.0) mask[n] = 1;
    orc_pinch_fill(p, mask);
    int64_t count = 0;
    for (int64_t n = 0; n < N; ++n) {
        if (!mask[n] || before[n]) continue;
        ++count;
        for (int j = 0; j < NC * L.Q; ++j) f[(int64_t)j * N + n] = 0.0;
        for (int j = 0; j < NS * S.Q; ++j) h[(int64_t)j * N + n] = 0.0;
        Cps[n] = 0.0;
    }
    free(before);
    return count;
}

/* Post-step populations at selected fluid nodes only, from the state at t.
 * Needs post-collision values at the nodes' upstream neighbours, which are
 * computed one by one from the densities of the whole field.
 * f_out: [count][ncomp*Q], h_out: [count][QS * species] (may be NULL without solute). */
void orc_step_nodes(const orc_params* p, const uint8_t* mask, const double* f, const double* h,
                    const int64_t* nodes, int64_t count, double* f_out, double* h_out) {
    flow_lat L = make_flow(p->lattice);
    sol_lat S = make_sol(p->lattice, p->J0);
    int64_t N = nnodes(p);
    int NC = p->ncomp;
    double* rho = (double*)calloc((size_t)(NC * N), sizeof(double));
    double* psi = (double*)calloc((size_t)(NC * N), sizeof(double));
    densities(p, &L, mask, f, rho, psi);

#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t q = 0; q < count; ++q) {
        int64_t y = nodes[q];
        int x, yy, z;
        coords(p, y, &x, &yy, &z);
        double fs[2][19], hs[14], fs_n[2][19], hs_n[14];
        collide_at(p, &L, &S, mask, f, h, rho, psi, y, fs, hs);
        for (int i = 0; i < L.Q; ++i) {
            int64_t src = nbr_back(p, y, L.c[i]);
            int solid = mask[src] != 0;
            if (!solid) collide_at(p, &L, &S, mask, f, h, rho, psi, src, fs_n, hs_n);
            for (int s = 0; s < NC; ++s)
                f_out[q * NC * L.Q + s * L.Q + i] = solid ? fs[s][L.opp[i]] : fs_n[s][i];
        }
        if (p->solute && h_out) {
            int NS = p->product ? 2 : 1, QT = NS * S.Q;
            for (int sp = 0; sp < NS; ++sp)
                for (int k = 0; k < S.Q; ++k) {
                    int kb = S.opp[k], b = sp * S.Q;
                    double v;
                    int64_t src = nbr_back(p, y, S.c[k]);
                    if (p->solute == 2 && x == 0 && S.c[k][0] == 1) {
                        collide_at(p, &L, &S, mask, f, h, rho, psi, nbr(p, y, S.c[k]), fs_n, hs_n);
                        v = 2.0 * S.w[k] * (sp ? p->C_in2 : p->C_in) - hs_n[b + kb];
                    } else if (p->solute == 2 && x == p->nx - 1 && S.c[k][0] == -1) {
                        v = hs[b + k];
                    } else if (mask[src]) {
                        double tau_d = p->D / S.cs2 + 0.5;
                        collide_at(p, &L, &S, mask, f, h, rho, psi, nbr(p, y, S.c[k]), fs_n, hs_n);
                        double kr = rate_at(p, y);
                        double Cb = 2.0 * hs_n[kb] / (2.0 * S.w[k] + kr * tau_d / (tau_d - 0.5));
                        if (sp == 0) {
                            v = 2.0 * S.w[k] * Cb - hs_n[kb];
                        } else {
                            double tau2 = p->D2 / S.cs2 + 0.5;
                            v = hs_n[b + kb] + kr * tau2 / (tau2 - 0.5) * Cb;
                        }
                    } else {
                        collide_at(p, &L, &S, mask, f, h, rho, psi, src, fs_n, hs_n);
                        v = hs_n[b + k];
                    }
                    h_out[q * QT + b + k] = v;
                }
        }
    }
    free(rho);
    free(psi);
}

/* Forces F^s at every node of the state (solid -> 0): [ncomp][3][N]. */
void orc_forces(const orc_params* p, const uint8_t* mask, const double* f, double* Fout) {
    flow_lat L = make_flow(p->lattice);
    int64_t N = nnodes(p);
    int NC = p->ncomp;
    double* rho = (double*)calloc((size_t)(NC * N), sizeof(double));
    double* psi = (double*)calloc((size_t)(NC * N), sizeof(double));
    densities(p, &L, mask, f, rho, psi);
    for (int64_t n = 0; n < N; ++n) {
        double F[2][3] = {{0, 0, 0}, {0, 0, 0}};
        if (!mask[n]) force_at(p, &L, mask, rho, psi, n, F);
        for (int s = 0; s < NC; ++s)
            for (int a = 0; a < 3; ++a) Fout[((int64_t)s * 3 + a) * N + n] = F[s][a];
    }
    free(rho);
    free(psi);
}

/* Macroscopic fields of the current (post-streaming) state: rho_s = sum_i f,
 * u = barycentric velocity with half force (eq:1.19, taken after streaming),
 * C = sum_k h_k per solute species.  Solid nodes -> 0.  rho: [ncomp][N], u: [3][N],
 * C: [species][N] or NULL. */
void orc_moments(const orc_params* p, const uint8_t* mask, const double* f, const double* h,
                 double* rho_out, double* u_out, double* C_out) {
    flow_lat L = make_flow(p->lattice);
    sol_lat S = make_sol(p->lattice, p->J0);
    int64_t N = nnodes(p);
    int NC = p->ncomp;
    double* rho = (double*)calloc((size_t)(NC * N), sizeof(double));
    double* psi = (double*)calloc((size_t)(NC * N), sizeof(double));
    densities(p, &L, mask, f, rho, psi);
    for (int64_t n = 0; n < N; ++n) {
        double u[3] = {0, 0, 0};
        if (!mask[n]) {
            double F[2][3];
            force_at(p, &L, mask, rho, psi, n, F);
            bary_u(p, &L, f, n, rho, F, u);
        }
        for (int s = 0; s < NC; ++s) rho_out[(int64_t)s * N + n] = mask[n] ? 0.0 : rho[(int64_t)s * N + n];
        for (int a = 0; a < 3; ++a) u_out[(int64_t)a * N + n] = u[a];
        if (C_out) {
            for (int sp = 0; sp <= (p->product ? 1 : 0); ++sp) {
                double C = 0.0;
                if (p->solute && !mask[n])
                    for (int k = 0; k < S.Q; ++k) C += h[(int64_t)(sp * S.Q + k) * N + n];
                C_out[(int64_t)sp * N + n] = C;
            }
        }
    }
    free(rho);
    free(psi);
}

/* ===========================================================================
 * Conjugate heat transfer (Reactive LBM subsection): internal-energy
 * distributions in the fluid (eq:therpop, eq:therpopeq) and in the solid
 * (eq:therpop_solid, eq:therpopeq_solid) on the flow lattice, coupled at the
 * interface by the thermal counter-slip conditions (eq:countSlipFluxCon,
 * eq:countSlipTempCon) with the reaction heat (eq:reacRate), iterated with
 * the wet-node reaction (eq:wetnode9) until the interface temperature settles
 * (the flowchart's C_b - T loop).
 *
 * Which nodes carry what:
 *   - every fluid node carries fluid energy populations g_i;
 *   - every solid node carries solid energy populations gs_i;
 *   - an interface node is a fluid node with a solid neighbour along some
 *     flow-lattice link; it carries both (the paper's double node on the
 *     interface, the same node the solute's wet-node rule acts on).
 * Streaming pulls g_i from x - c_i if that node is fluid, gs_i if it carries
 * solid populations; the remaining populations of an interface node are the
 * unknowns of the counter-slip conditions:
 *   M_f = { i : x - c_i solid }            fluid unknowns  g_i  = w_i X_f
 *   M_s = { i : x - c_i fluid, and either not an interface node (nothing
 *           streams gs_i) or x + c_i solid (gs_i would come in from across
 *           the fluid: the solid field does not pass through it) }
 *                                           solid unknowns  gs_i = w_i X_s
 * (the counter-slip form: unknowns proportional to their weights).  Reading
 * (ours) of the flat-wall conditions for any voxel interface:
 *   temperature   (Kn_f + W_f X_f) / (rho c_p)_f = (Kn_s + W_s X_s) / (rho c_p)_s
 *   heat flux     k_f (W_f' X_f - B_f) = k_s (A_s - W_s' X_s) + Hdot
 * with Kn the sums of the known populations, W = sum of w_i over the
 * unknowns, W' and B (A) over the unknowns whose opposite population is
 * known (B = sum of g_opp(i), A = sum of gs_opp(i)), k = 1 - 1/(2 tau_e),
 * Hdot = h_r sum over the node's wet solute links of k(T) C_b (eq:reacRate,
 * eq:wetnode9), k(T) = A exp(-E / (R_u T)).  For a flat wall with normal +y
 * in D2Q9 (M_f = {2, 5, 6}, M_s = {4, 7, 8}) eliminating X_f gives exactly
 * the printed eq:unknownpopTempS, and the temperature condition then gives
 * eq:unknownpopTempF.  The flux condition can always be posed except at a
 * node whose every missing fluid link has a solid on both sides (only
 * diagonal pairs: axis pinches are removed by the geometry rule); there the
 * temperature condition alone is used, the solid unknowns taking the local
 * solid equilibrium, no reaction heat is released, and the node is counted.
 * ========================================================================= */
typedef struct {
    double tau_ef, tau_es;   /* 3 alpha + 1/2 of fluid and solid */
    double rhocp_f, rhocp_s; /* rho c_p of fluid and solid */
    double h_r;              /* heat released per unit of O2 consumed */
    double A, E_over_R;      /* k(T) = A exp(-E_over_R / T) at the interface */
    double T_tol;            /* relative tolerance of the interface iteration */
    int32_t T_maxit;         /* its iteration cap */
    int32_t pad_;
} orc_thermal;

/* Node classes: holds_solid[n] = 1 for solid and interface nodes,
 * iface[n] = 1 for interface nodes. */
void orc_thermal_nodes(const orc_params* p, const uint8_t* mask, uint8_t* holds_solid, uint8_t* iface) {
    flow_lat L = make_flow(p->lattice);
    int64_t N = nnodes(p);
    for (int64_t n = 0; n < N; ++n) {
        int any = 0;
        if (!mask[n])
            for (int i = 1; i < L.Q; ++i)
                if (mask[nbr_back(p, n, L.c[i])]) any = 1;
        iface[n] = (uint8_t)any;
        holds_solid[n] = (uint8_t)(mask[n] || any);
    }
}

/* Energy equilibrium of the fluid, eq:therpopeq, with E = rho_f eps_f = sum g:
 * w_i E [1 + c.u/cs2 + (c.u)^2/(2 cs2^2) - u.u/(2 cs2)]. */
static double geq_i(const flow_lat* L, int i, double E, const double u[3]) {
    double cu = L->c[i][0] * u[0] + L->c[i][1] * u[1] + L->c[i][2] * u[2];
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    return L->w[i] * E * (1.0 + cu / CS2 + cu * cu / (2.0 * CS2 * CS2) - uu / (2.0 * CS2));
}

/* Initial energy populations at temperature T [N]: fluid g = g^eq(rho_f c_p,f T, u),
 * solid (and interface) gs = w_i rho_s c_p,s T; Ti = T at every node. */
void orc_thermal_init(const orc_params* p, const orc_thermal* th, const uint8_t* mask, const double* T,
                      const double* u, double* g, double* gs, double* Ti) {
    flow_lat L = make_flow(p->lattice);
    int64_t N = nnodes(p);
    uint8_t* hs = (uint8_t*)malloc((size_t)N);
    uint8_t* itf = (uint8_t*)malloc((size_t)N);
    orc_thermal_nodes(p, mask, hs, itf);
    for (int64_t n = 0; n < N; ++n) {
        double v[3] = {0, 0, 0};
        if (u) { v[0] = u[n]; v[1] = u[N + n]; v[2] = u[2 * N + n]; }
        for (int i = 0; i < L.Q; ++i) {
            g[(int64_t)i * N + n] = mask[n] ? 0.0 : geq_i(&L, i, th->rhocp_f * T[n], v);
            gs[(int64_t)i * N + n] = hs[n] ? L.w[i] * th->rhocp_s * T[n] : 0.0;
        }
        Ti[n] = T[n];
    }
    free(hs);
    free(itf);
}

/* Counter-slip solve at interface node y (see the block comment above).  g, gs
 * hold the streamed known populations and receive the unknowns; h (solute,
 * after streaming) receives the wet-link populations of both species with the
 * rate at the settled temperature.  Ti[y]: start value in, settled value out.
 * Returns the iterations used; *degenerate = 1 if the flux condition could not
 * be posed; *settled = 1 if the tolerance was met. */
static int interface_solve(const orc_params* p, const orc_thermal* th, const flow_lat* L, const sol_lat* S,
                           const uint8_t* mask, const uint8_t* hs, const uint32_t* wet, double* g, double* gs,
                           double* h, double* Ti, int64_t y, int* degenerate, int* settled) {
    int64_t N = nnodes(p);
    int Q = L->Q;
    int mf[19], ms[19];
    for (int i = 0; i < Q; ++i) {
        int64_t src = nbr_back(p, y, L->c[i]);
        int64_t dst = nbr(p, y, L->c[i]);
        mf[i] = (i > 0) && mask[src];
        /* solid unknown: nothing streams it (the upstream node is pure fluid),
         * or it streams in from a fluid node across the node from a solid one
         * (the solid field does not pass through the fluid) */
        ms[i] = (i > 0) && !mask[src] && (!hs[src] || mask[dst]);
    }
    double Knf = 0, Kns = 0, Wf = 0, Ws = 0, Wfp = 0, Wsp = 0, Bf = 0, As = 0;
    for (int i = 0; i < Q; ++i) {
        int o = L->opp[i];
        if (mf[i]) {
            Wf += L->w[i];
            if (!mf[o]) { Wfp += L->w[i]; Bf += g[(int64_t)o * N + y]; }
        } else {
            Knf += g[(int64_t)i * N + y];
        }
        if (ms[i]) {
            Ws += L->w[i];
            if (!ms[o]) { Wsp += L->w[i]; As += gs[(int64_t)o * N + y]; }
        } else {
            Kns += gs[(int64_t)i * N + y];
        }
    }
    double kf = 1.0 - 0.5 / th->tau_ef, ks = 1.0 - 0.5 / th->tau_es;
    double cfs = th->rhocp_f / th->rhocp_s;
    double det = Wf * ks * Wsp + cfs * Ws * kf * Wfp;
    *degenerate = !(det > 0.0);

    /* solute wet links of this node: h_in = h_opp(k) after streaming */
    int nwet = 0, kw[7];
    double hin[7];
    double tau_d = p->D / S->cs2 + 0.5;
    if (p->solute)
        for (int k = 1; k < S->Q; ++k)
            if (wet[y] & (1u << k)) { kw[nwet] = k; hin[nwet] = h[(int64_t)S->opp[k] * N + y]; ++nwet; }

    double T = Ti[y], Xf = 0, Xs = 0, kr = 0, Cb[7];
    int it = 0;
    *settled = 0;
    while (it < th->T_maxit) {
        ++it;
        kr = th->A * exp(-th->E_over_R / T);
        double Hdot = 0.0;
        for (int q = 0; q < nwet; ++q) {
            int k = kw[q];
            Cb[q] = 2.0 * hin[q] / (2.0 * S->w[k] + kr * tau_d / (tau_d - 0.5));
            Hdot += th->h_r * kr * Cb[q];
        }
        if (!*degenerate) {
            Xs = (Wf * (ks * As + kf * Bf + Hdot) - kf * Wfp * (cfs * Kns - Knf)) / det;
        } else {
            Xs = Ws > 0.0 ? Kns / (1.0 - Ws) : 0.0;
        }
        Xf = (cfs * (Kns + Ws * Xs) - Knf) / Wf;
        double Tn = (Knf + Wf * Xf) / th->rhocp_f;
        int done = fabs(Tn - T) <= th->T_tol * fabs(Tn);
        T = Tn;
        if (done) { *settled = 1; break; }
    }
    for (int i = 0; i < Q; ++i) {
        if (mf[i]) g[(int64_t)i * N + y] = L->w[i] * Xf;
        if (ms[i]) gs[(int64_t)i * N + y] = L->w[i] * Xs;
    }
    Ti[y] = T;
    /* wet-link populations with the rate of the last iteration: O2 (eq:wetnode9)
     * and the product (eq:reactCO2, same convention as without heat) */
    for (int q = 0; q < nwet; ++q) {
        int k = kw[q];
        h[(int64_t)k * N + y] = 2.0 * S->w[k] * Cb[q] - hin[q];
        if (p->product) {
            double tau2 = p->D2 / S->cs2 + 0.5;
            double hin2 = h[(int64_t)(S->Q + S->opp[k]) * N + y];
            h[(int64_t)(S->Q + k) * N + y] = hin2 + kr * tau2 / (tau2 - 0.5) * Cb[q];
        }
    }
    return it;
}

/* Full time steps with conjugate heat transfer.  Flow and solute as orc_step,
 * except that the wet-link populations of the solute come from the interface
 * solve (their rate follows the interface temperature); then the energy
 * populations:
 *   1. fluid g: BGK towards g^eq(sum g, u) with tau_ef, u the barycentric
 *      velocity with half force of this step (the solute's);
 *      solid gs: BGK towards w_i sum gs with tau_es (eq:therpop_solid);
 *   2. streaming (pull) of the known populations;
 *   3. interface solve at every interface node (counter-slip + reaction).
 * g, gs: [Q][N]; Ti: [N] interface temperatures (start values of the
 * iteration, carried from step to step).  stats (may be NULL): [0] total
 * iterations, [1] interface solves that did not settle, [2] degenerate
 * interface nodes (of the last step). */
void orc_step_thermal(const orc_params* p, const orc_thermal* th, const uint8_t* mask, double* f, double* h,
                      double* g, double* gs, double* Ti, int64_t nsteps, int64_t* stats) {
    flow_lat L = make_flow(p->lattice);
    sol_lat S = make_sol(p->lattice, p->J0);
    int64_t N = nnodes(p);
    int NC = p->ncomp, Q = L.Q;
    int NS = p->solute ? (p->product ? 2 : 1) : 0;
    double* rho = (double*)calloc((size_t)(NC * N), sizeof(double));
    double* psi = (double*)calloc((size_t)(NC * N), sizeof(double));
    double* fstar = (double*)calloc((size_t)(NC * Q * N), sizeof(double));
    double* hstar = NS ? (double*)calloc((size_t)(NS * S.Q * N), sizeof(double)) : NULL;
    double* gstar = (double*)calloc((size_t)(Q * N), sizeof(double));
    double* gsstar = (double*)calloc((size_t)(Q * N), sizeof(double));
    uint8_t* hs = (uint8_t*)malloc((size_t)N);
    uint8_t* itf = (uint8_t*)malloc((size_t)N);
    uint32_t* fb = (uint32_t*)malloc((size_t)N * sizeof(uint32_t));
    uint32_t* wet = (uint32_t*)malloc((size_t)N * sizeof(uint32_t));
    orc_thermal_nodes(p, mask, hs, itf);
    orc_link_masks(p, mask, fb, wet);
    int64_t iters = 0, unsettled = 0, degen = 0;

    for (int64_t t = 0; t < nsteps; ++t) {
        densities(p, &L, mask, f, rho, psi);
#pragma omp parallel for schedule(static)
        for (int64_t n = 0; n < N; ++n) {
            if (!mask[n]) {
                double fs[2][19], hsn[14], F[2][3], u[3];
                collide_at(p, &L, &S, mask, f, h, rho, psi, n, fs, hsn);
                for (int s = 0; s < NC; ++s)
                    for (int i = 0; i < Q; ++i) fstar[((int64_t)s * Q + i) * N + n] = fs[s][i];
                for (int k = 0; k < NS * S.Q; ++k) hstar[(int64_t)k * N + n] = hsn[k];
                force_at(p, &L, mask, rho, psi, n, F);
                bary_u(p, &L, f, n, rho, F, u);
                double E = 0.0;
                for (int i = 0; i < Q; ++i) E += g[(int64_t)i * N + n];
                for (int i = 0; i < Q; ++i) {
                    double gi = g[(int64_t)i * N + n];
                    gstar[(int64_t)i * N + n] = gi - (gi - geq_i(&L, i, E, u)) / th->tau_ef;
                }
            }
            if (hs[n]) {
                double Es = 0.0;
                for (int i = 0; i < Q; ++i) Es += gs[(int64_t)i * N + n];
                for (int i = 0; i < Q; ++i) {
                    double gi = gs[(int64_t)i * N + n];
                    gsstar[(int64_t)i * N + n] = gi - (gi - L.w[i] * Es) / th->tau_es;
                }
            }
        }
#pragma omp parallel for schedule(static)
        for (int64_t n = 0; n < N; ++n) {
            if (!mask[n]) {
                for (int s = 0; s < NC; ++s)
                    for (int i = 0; i < Q; ++i)
                        f[((int64_t)s * Q + i) * N + n] = flow_stream_value(p, &L, mask, fstar, s, i, n);
                for (int sp = 0; sp < NS; ++sp)
                    for (int k = 0; k < S.Q; ++k) {
                        /* wet links are left to the interface solve (their rate needs T) */
                        int64_t src = nbr_back(p, n, S.c[k]);
                        int x, yy, z;
                        coords(p, n, &x, &yy, &z);
                        int seam = p->solute == 2 && ((x == 0 && S.c[k][0] == 1) || (x == p->nx - 1 && S.c[k][0] == -1));
                        if (!seam && mask[src]) continue;
                        h[(int64_t)(sp * S.Q + k) * N + n] = solute_stream_value(p, &S, mask, hstar, sp, k, n);
                    }
                for (int i = 0; i < Q; ++i) {
                    int64_t src = nbr_back(p, n, L.c[i]);
                    if (!mask[src]) g[(int64_t)i * N + n] = gstar[(int64_t)i * N + src];
                }
            }
            if (hs[n])
                for (int i = 0; i < Q; ++i) {
                    int64_t src = nbr_back(p, n, L.c[i]);
                    if (hs[src]) gs[(int64_t)i * N + n] = gsstar[(int64_t)i * N + src];
                }
        }
        degen = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : iters, unsettled, degen)
        for (int64_t n = 0; n < N; ++n) {
            if (!itf[n]) continue;
            int dg = 0, ok = 0;
            iters += interface_solve(p, th, &L, &S, mask, hs, wet, g, gs, h, Ti, n, &dg, &ok);
            unsettled += !ok;
            degen += dg;
        }
    }
    if (stats) { stats[0] = iters; stats[1] = unsettled; stats[2] = degen; }
    free(rho); free(psi); free(fstar); free(hstar); free(gstar); free(gsstar);
    free(hs); free(itf); free(fb); free(wet);
}

/* Temperature field: fluid nodes (interface included) E_f / (rho c_p)_f,
 * solid nodes E_s / (rho c_p)_s.  T: [N]. */
void orc_temperature(const orc_params* p, const orc_thermal* th, const uint8_t* mask, const double* g,
                     const double* gs, double* T) {
    flow_lat L = make_flow(p->lattice);
    int64_t N = nnodes(p);
    for (int64_t n = 0; n < N; ++n) {
        double E = 0.0;
        for (int i = 0; i < L.Q; ++i) E += mask[n] ? gs[(int64_t)i * N + n] : g[(int64_t)i * N + n];
        T[n] = E / (mask[n] ? th->rhocp_s : th->rhocp_f);
    }
}
