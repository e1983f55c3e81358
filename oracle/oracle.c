/*
 * FP64 CPU oracle of the transient coupled EM-thermal-mechanical method
 * (arXiv 2603.07038, Sec. II).  TEST INFRASTRUCTURE ONLY: only the test suite,
 * the smoke check and the benchmark's CPU-baseline leg may load this file's
 * library.  It shares no code, header, table or helper with the HIP library.
 *
 * Everything is written in the plainest form: natural (unpadded) per-component
 * arrays, one loop per formula, FP64 throughout, no blocking or fusion.
 *
 * Array layouts (x fastest):
 *   cells  c(i,j,k)  = (k*ny + j)*nx + i                 nx*ny*nz
 *   nodes  n(i,j,k)  = (k*(ny+1) + j)*(nx+1) + i         (nx+1)(ny+1)(nz+1)
 *   x-edge (i,j,k)   = (k*(ny+1) + j)*nx + i             nx(ny+1)(nz+1)
 *   y-edge (i,j,k)   = (k*ny + j)*(nx+1) + i             (nx+1)ny(nz+1)
 *   z-edge (i,j,k)   = (k*(ny+1) + j)*(nx+1) + i         (nx+1)(ny+1)nz
 *   displacement     = 3*node + component (interleaved)
 * An x-edge (i,j,k) joins nodes (i,j,k) and (i+1,j,k); likewise for y, z.
 *
 * Material table rows: eps_r, sigma0, tcr, k, rho_cp, E, nu, cte, void.
 * Boundary codes per face (-x,+x,-y,+y,-z,+z): 0 = PMC, 1 = PEC.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_EPS0 8.8541878128e-12
#define OR_MU0 1.25663706212e-6
#define OR_C0 299792458.0
#define NPROP 9

typedef struct {
    int nx, ny, nz;
    double *dx, *dy, *dz;   /* primal widths */
    double *hx, *hy, *hz;   /* node-centred (dual) widths, half cells at the ends */
    uint8_t *mat;
    double *props;
    int n_mat;
    int bc[6];
    /* ports */
    int n_ports;
    int *pdir, *pi, *pj, *pk, *pwave;
    double *pweight, *pg;
    double *gport[3];       /* summed lumped conductance per edge */
} grid_t;

/* ---------- indexing ---------------------------------------------------- */
static inline int64_t CI(const grid_t *g, int i, int j, int k) { return ((int64_t)k * g->ny + j) * g->nx + i; }
static inline int64_t NI(const grid_t *g, int i, int j, int k) { return ((int64_t)k * (g->ny + 1) + j) * (g->nx + 1) + i; }
static inline int64_t XI(const grid_t *g, int i, int j, int k) { return ((int64_t)k * (g->ny + 1) + j) * g->nx + i; }
static inline int64_t YI(const grid_t *g, int i, int j, int k) { return ((int64_t)k * g->ny + j) * (g->nx + 1) + i; }
static inline int64_t ZI(const grid_t *g, int i, int j, int k) { return ((int64_t)k * (g->ny + 1) + j) * (g->nx + 1) + i; }

int64_t or_n_edges(const void *h, int dir) {
    const grid_t *g = (const grid_t *)h;
    if (dir == 0) return (int64_t)g->nx * (g->ny + 1) * (g->nz + 1);
    if (dir == 1) return (int64_t)(g->nx + 1) * g->ny * (g->nz + 1);
    return (int64_t)(g->nx + 1) * (g->ny + 1) * g->nz;
}
int64_t or_n_nodes(const void *h) {
    const grid_t *g = (const grid_t *)h;
    return (int64_t)(g->nx + 1) * (g->ny + 1) * (g->nz + 1);
}

static double prop(const grid_t *g, int64_t c, int col) { return g->props[(int)g->mat[c] * NPROP + col]; }

static double *dual(const double *d, int n) {
    double *h = (double *)calloc((size_t)n + 1, sizeof(double));
    for (int i = 0; i < n; ++i) { h[i] += 0.5 * d[i]; h[i + 1] += 0.5 * d[i]; }
    return h;
}

static double *dupd(const double *s, size_t n) { double *d = (double *)malloc(n * sizeof(double)); memcpy(d, s, n * sizeof(double)); return d; }

void *or_create(int nx, int ny, int nz, const double *dx, const double *dy, const double *dz,
                const uint8_t *mat, const double *props, int n_mat, const int *em_bc) {
    grid_t *g = (grid_t *)calloc(1, sizeof(grid_t));
    g->nx = nx; g->ny = ny; g->nz = nz;
    g->dx = dupd(dx, nx); g->dy = dupd(dy, ny); g->dz = dupd(dz, nz);
    g->hx = dual(dx, nx); g->hy = dual(dy, ny); g->hz = dual(dz, nz);
    size_t nc = (size_t)nx * ny * nz;
    g->mat = (uint8_t *)malloc(nc); memcpy(g->mat, mat, nc);
    g->props = dupd(props, (size_t)n_mat * NPROP); g->n_mat = n_mat;
    for (int f = 0; f < 6; ++f) g->bc[f] = em_bc[f];
    for (int d = 0; d < 3; ++d) g->gport[d] = (double *)calloc((size_t)or_n_edges(g, d), sizeof(double));
    return g;
}

void or_destroy(void *h) {
    grid_t *g = (grid_t *)h;
    if (!g) return;
    free(g->dx); free(g->dy); free(g->dz); free(g->hx); free(g->hy); free(g->hz);
    free(g->mat); free(g->props);
    free(g->pdir); free(g->pi); free(g->pj); free(g->pk); free(g->pwave); free(g->pweight); free(g->pg);
    for (int d = 0; d < 3; ++d) free(g->gport[d]);
    free(g);
}

static int64_t edge_index(const grid_t *g, int d, int i, int j, int k) {
    return d == 0 ? XI(g, i, j, k) : d == 1 ? YI(g, i, j, k) : ZI(g, i, j, k);
}

/* Port edges: a current density weight*J_w(t) impressed on the edge and a
 * lumped conductance g (Norton form of a resistive source) added to the
 * edge conductivity in the update (Eq. 1 excitation term). */
void or_set_ports(void *h, int n, const uint8_t *dir, const int *pi, const int *pj, const int *pk,
                  const int *wave, const double *weight, const double *gp) {
    grid_t *g = (grid_t *)h;
    g->n_ports = n;
    g->pdir = (int *)malloc(sizeof(int) * (n + 1)); g->pi = (int *)malloc(sizeof(int) * (n + 1));
    g->pj = (int *)malloc(sizeof(int) * (n + 1)); g->pk = (int *)malloc(sizeof(int) * (n + 1));
    g->pwave = (int *)malloc(sizeof(int) * (n + 1));
    g->pweight = (double *)malloc(sizeof(double) * (n + 1)); g->pg = (double *)malloc(sizeof(double) * (n + 1));
    for (int d = 0; d < 3; ++d) memset(g->gport[d], 0, sizeof(double) * (size_t)or_n_edges(g, d));
    for (int p = 0; p < n; ++p) {
        g->pdir[p] = dir[p]; g->pi[p] = pi[p]; g->pj[p] = pj[p]; g->pk[p] = pk[p];
        g->pwave[p] = wave[p]; g->pweight[p] = weight[p]; g->pg[p] = gp[p];
        g->gport[dir[p]][edge_index(g, dir[p], pi[p], pj[p], pk[p])] += gp[p];
    }
}

/* ---------- time step (Eq. 2, CFL) -------------------------------------- */
/* Largest stable explicit step of the vacuum wave equation on the finest
 * spacing, scaled by the Courant number. */
double or_cfl_dt(const void *h, double cfl) {
    const grid_t *g = (const grid_t *)h;
    double mx = 1e300, my = 1e300, mz = 1e300;
    for (int i = 0; i < g->nx; ++i) mx = fmin(mx, g->dx[i]);
    for (int j = 0; j < g->ny; ++j) my = fmin(my, g->dy[j]);
    for (int k = 0; k < g->nz; ++k) mz = fmin(mz, g->dz[k]);
    return cfl / (OR_C0 * sqrt(1.0 / (mx * mx) + 1.0 / (my * my) + 1.0 / (mz * mz)));
}

/* ---------- edge materials (diagonal matrices D_eps, D_sigma(T), D_k) --- */
/* Each edge property is the mean of the up-to-four cells that touch the edge,
 * weighted by the quarter of the edge's dual area that lies in each cell.
 * sigma follows Eq. (6) per cell at the edge-midpoint temperature rise. */
typedef struct { double eps, sig, kth, area, len; } edge_mat_t;

static edge_mat_t edge_mat(const grid_t *g, int d, int i, int j, int k, double theta_e) {
    edge_mat_t m = {0, 0, 0, 0, 0};
    int a0, a1, b0, b1;  /* transverse cell ranges */
    double wsum = 0;
    if (d == 0) {
        m.len = g->dx[i]; m.area = g->hy[j] * g->hz[k];
        a0 = j - 1; a1 = j; b0 = k - 1; b1 = k;
        for (int kk = b0; kk <= b1; ++kk) for (int jj = a0; jj <= a1; ++jj) {
            if (jj < 0 || jj >= g->ny || kk < 0 || kk >= g->nz) continue;
            double w = 0.25 * g->dy[jj] * g->dz[kk];
            int64_t c = CI(g, i, jj, kk);
            m.eps += w * prop(g, c, 0);
            m.sig += w * prop(g, c, 1) / (1.0 + prop(g, c, 2) * theta_e);
            m.kth += w * prop(g, c, 3);
            wsum += w;
        }
    } else if (d == 1) {
        m.len = g->dy[j]; m.area = g->hx[i] * g->hz[k];
        for (int kk = k - 1; kk <= k; ++kk) for (int ii = i - 1; ii <= i; ++ii) {
            if (ii < 0 || ii >= g->nx || kk < 0 || kk >= g->nz) continue;
            double w = 0.25 * g->dx[ii] * g->dz[kk];
            int64_t c = CI(g, ii, j, kk);
            m.eps += w * prop(g, c, 0);
            m.sig += w * prop(g, c, 1) / (1.0 + prop(g, c, 2) * theta_e);
            m.kth += w * prop(g, c, 3);
            wsum += w;
        }
    } else {
        m.len = g->dz[k]; m.area = g->hx[i] * g->hy[j];
        for (int jj = j - 1; jj <= j; ++jj) for (int ii = i - 1; ii <= i; ++ii) {
            if (ii < 0 || ii >= g->nx || jj < 0 || jj >= g->ny) continue;
            double w = 0.25 * g->dx[ii] * g->dy[jj];
            int64_t c = CI(g, ii, jj, k);
            m.eps += w * prop(g, c, 0);
            m.sig += w * prop(g, c, 1) / (1.0 + prop(g, c, 2) * theta_e);
            m.kth += w * prop(g, c, 3);
            wsum += w;
        }
    }
    m.eps = OR_EPS0 * m.eps / wsum;
    m.sig /= wsum;
    m.kth /= wsum;
    return m;
}

static double theta_mid(const grid_t *g, const double *th, int d, int i, int j, int k) {
    if (!th) return 0.0;
    double a = th[NI(g, i, j, k)];
    double b = d == 0 ? th[NI(g, i + 1, j, k)] : d == 1 ? th[NI(g, i, j + 1, k)] : th[NI(g, i, j, k + 1)];
    return 0.5 * (a + b);
}

/* Tangential edges on PEC faces are held at zero. */
static int pec_edge(const grid_t *g, int d, int i, int j, int k) {
    const int *b = g->bc;
    if (d != 0 && ((i == 0 && b[0]) || (i == g->nx && b[1]))) return 1;
    if (d != 1 && ((j == 0 && b[2]) || (j == g->ny && b[3]))) return 1;
    if (d != 2 && ((k == 0 && b[4]) || (k == g->nz && b[5]))) return 1;
    return 0;
}

/* ---------- curl-curl (S = curl mu^-1 curl, Sec. II-A) -------------------
 * Magnetic intensity on each primal face = circulation of e around the face
 * divided by mu0 times the face area.  The curl of h at an edge is taken on
 * the edge's dual face; faces outside the domain carry h = 0, which is the
 * PMC (natural) truncation.  The result is (S e) per unit edge volume
 * L*A_dual; S itself is that times L*A_dual and is symmetric. */
static double hz_face(const grid_t *g, const double *ex, const double *ey, int i, int j, int k) {
    /* z-normal face of cell column (i,j) at node plane k */
    if (i < 0 || i >= g->nx || j < 0 || j >= g->ny) return 0.0;
    double circ = ex[XI(g, i, j, k)] * g->dx[i] + ey[YI(g, i + 1, j, k)] * g->dy[j]
                - ex[XI(g, i, j + 1, k)] * g->dx[i] - ey[YI(g, i, j, k)] * g->dy[j];
    return circ / (OR_MU0 * g->dx[i] * g->dy[j]);
}
static double hx_face(const grid_t *g, const double *ey, const double *ez, int i, int j, int k) {
    /* x-normal face at node plane i of cell (j,k) */
    if (j < 0 || j >= g->ny || k < 0 || k >= g->nz) return 0.0;
    double circ = ey[YI(g, i, j, k)] * g->dy[j] + ez[ZI(g, i, j + 1, k)] * g->dz[k]
                - ey[YI(g, i, j, k + 1)] * g->dy[j] - ez[ZI(g, i, j, k)] * g->dz[k];
    return circ / (OR_MU0 * g->dy[j] * g->dz[k]);
}
static double hy_face(const grid_t *g, const double *ez, const double *ex, int i, int j, int k) {
    /* y-normal face at node plane j of cell (i,k) */
    if (i < 0 || i >= g->nx || k < 0 || k >= g->nz) return 0.0;
    double circ = ez[ZI(g, i, j, k)] * g->dz[k] + ex[XI(g, i, j, k + 1)] * g->dx[i]
                - ez[ZI(g, i + 1, j, k)] * g->dz[k] - ex[XI(g, i, j, k)] * g->dx[i];
    return circ / (OR_MU0 * g->dz[k] * g->dx[i]);
}

static double curlcurl_edge(const grid_t *g, const double *ex, const double *ey, const double *ez,
                            int d, int i, int j, int k) {
    if (d == 0)
        return (hz_face(g, ex, ey, i, j, k) - hz_face(g, ex, ey, i, j - 1, k)) / g->hy[j]
             - (hy_face(g, ez, ex, i, j, k) - hy_face(g, ez, ex, i, j, k - 1)) / g->hz[k];
    if (d == 1)
        return (hx_face(g, ey, ez, i, j, k) - hx_face(g, ey, ez, i, j, k - 1)) / g->hz[k]
             - (hz_face(g, ex, ey, i, j, k) - hz_face(g, ex, ey, i - 1, j, k)) / g->hx[i];
    return (hy_face(g, ez, ex, i, j, k) - hy_face(g, ez, ex, i - 1, j, k)) / g->hx[i]
         - (hx_face(g, ey, ez, i, j, k) - hx_face(g, ey, ez, i, j - 1, k)) / g->hy[j];
}

/* (S e) per unit edge volume on every edge (zero on PEC edges). */
void or_curlcurl(const void *h, const double *ex, const double *ey, const double *ez,
                 double *sx, double *sy, double *sz) {
    const grid_t *g = (const grid_t *)h;
    double *out[3] = {sx, sy, sz};
    for (int d = 0; d < 3; ++d) {
        int ni = g->nx + (d != 0), nj = g->ny + (d != 1), nk = g->nz + (d != 2);
#pragma omp parallel for collapse(2) schedule(static)
        for (int k = 0; k < nk; ++k)
            for (int j = 0; j < nj; ++j)
                for (int i = 0; i < ni; ++i)
                    out[d][edge_index(g, d, i, j, k)] =
                        pec_edge(g, d, i, j, k) ? 0.0 : curlcurl_edge(g, ex, ey, ez, d, i, j, k);
    }
}

/* Edge length times dual area (the per-edge volume weight), and eps, sigma
 * per edge: exposed for tests that assemble the operators densely. */
void or_edge_coeffs(const void *h, const double *theta, int d, double *vol, double *eps, double *sig,
                    double *kth, uint8_t *pec) {
    const grid_t *g = (const grid_t *)h;
    int ni = g->nx + (d != 0), nj = g->ny + (d != 1), nk = g->nz + (d != 2);
    for (int k = 0; k < nk; ++k)
        for (int j = 0; j < nj; ++j)
            for (int i = 0; i < ni; ++i) {
                int64_t e = edge_index(g, d, i, j, k);
                edge_mat_t m = edge_mat(g, d, i, j, k, theta_mid(g, theta, d, i, j, k));
                if (vol) vol[e] = m.len * m.area;
                if (eps) eps[e] = m.eps;
                if (sig) sig[e] = m.sig;
                if (kth) kth[e] = m.kth;
                if (pec) pec[e] = (uint8_t)pec_edge(g, d, i, j, k);
            }
}

/* ---------- EM update, Eq. (2)-(3) --------------------------------------
 * Per edge, divided by the edge volume:
 *   (eps + a) e^{n+1} = 2 eps e^n - dt^2 (S e^n) - (eps - a) e^{n-1} - dt^2 (dJ/dt)^n
 * with a = dt*sigma(T^n)/2 (sigma including any port conductance) and
 * dt^2 (dJ/dt)^n = dt (J^{n+1/2} - J^{n-1/2}).
 * J_new / J_old are the per-wave excitation values at t_{n+1/2}, t_{n-1/2}. */
void or_em_step(const void *h, double dt, const double *theta,
                const double *exm, const double *eym, const double *ezm,
                const double *ex, const double *ey, const double *ez,
                double *exn, double *eyn, double *ezn, const double *J_new, const double *J_old) {
    const grid_t *g = (const grid_t *)h;
    double *jd[3];
    for (int d = 0; d < 3; ++d) jd[d] = (double *)calloc((size_t)or_n_edges(g, d), sizeof(double));
    for (int p = 0; p < g->n_ports; ++p) {
        int w = g->pwave[p];
        jd[g->pdir[p]][edge_index(g, g->pdir[p], g->pi[p], g->pj[p], g->pk[p])] +=
            g->pweight[p] * (J_new[w] - J_old[w]);
    }
    const double *em[3] = {exm, eym, ezm}, *ec[3] = {ex, ey, ez};
    double *en[3] = {exn, eyn, ezn};
    for (int d = 0; d < 3; ++d) {
        int ni = g->nx + (d != 0), nj = g->ny + (d != 1), nk = g->nz + (d != 2);
#pragma omp parallel for collapse(2) schedule(static)
        for (int k = 0; k < nk; ++k)
            for (int j = 0; j < nj; ++j)
                for (int i = 0; i < ni; ++i) {
                    int64_t e = edge_index(g, d, i, j, k);
                    if (pec_edge(g, d, i, j, k)) { en[d][e] = 0.0; continue; }
                    edge_mat_t m = edge_mat(g, d, i, j, k, theta_mid(g, theta, d, i, j, k));
                    double a = 0.5 * dt * (m.sig + g->gport[d][e]);
                    double s = curlcurl_edge(g, ex, ey, ez, d, i, j, k);
                    en[d][e] = (2.0 * m.eps * ec[d][e] - dt * dt * s - (m.eps - a) * em[d][e] - dt * jd[d][e])
                               / (m.eps + a);
                }
    }
    for (int d = 0; d < 3; ++d) free(jd[d]);
}

/* ---------- Joule source P = D_sigma e^2 (Sec. II-A) --------------------
 * Node form: each edge's power sigma_e(T^n) e_e^2 * L*A_dual is split half to
 * each end node and divided by the node's volume hx*hy*hz.  Only material
 * conductivity heats the package (port conductances model the source). */
void or_joule(const void *h, const double *theta, const double *ex, const double *ey, const double *ez,
              double *P) {
    const grid_t *g = (const grid_t *)h;
    const double *e[3] = {ex, ey, ez};
    int64_t nn = or_n_nodes(g);
    memset(P, 0, sizeof(double) * (size_t)nn);
    for (int d = 0; d < 3; ++d) {
        int ni = g->nx + (d != 0), nj = g->ny + (d != 1), nk = g->nz + (d != 2);
        for (int k = 0; k < nk; ++k)
            for (int j = 0; j < nj; ++j)
                for (int i = 0; i < ni; ++i) {
                    int64_t ei = edge_index(g, d, i, j, k);
                    edge_mat_t m = edge_mat(g, d, i, j, k, theta_mid(g, theta, d, i, j, k));
                    double half = 0.5 * m.sig * e[d][ei] * e[d][ei] * m.len * m.area;
                    P[NI(g, i, j, k)] += half;
                    P[NI(g, i + (d == 0), j + (d == 1), k + (d == 2))] += half;
                }
    }
    for (int k = 0; k <= g->nz; ++k)
        for (int j = 0; j <= g->ny; ++j)
            for (int i = 0; i <= g->nx; ++i) P[NI(g, i, j, k)] /= g->hx[i] * g->hy[j] * g->hz[k];
}

/* Total dissipated power sum_e sigma_e(T) e_e^2 L A_dual [W]. */
double or_joule_total(const void *h, const double *theta, const double *ex, const double *ey, const double *ez) {
    const grid_t *g = (const grid_t *)h;
    const double *e[3] = {ex, ey, ez};
    double tot = 0;
    for (int d = 0; d < 3; ++d) {
        int ni = g->nx + (d != 0), nj = g->ny + (d != 1), nk = g->nz + (d != 2);
        for (int k = 0; k < nk; ++k)
            for (int j = 0; j < nj; ++j)
                for (int i = 0; i < ni; ++i) {
                    int64_t ei = edge_index(g, d, i, j, k);
                    edge_mat_t m = edge_mat(g, d, i, j, k, theta_mid(g, theta, d, i, j, k));
                    tot += m.sig * e[d][ei] * e[d][ei] * m.len * m.area;
                }
    }
    return tot;
}

/* ---------- thermal, Eq. (4)-(5) ------------------------------------------
 * Node finite volume on the same grid: capacity C_n V_n is rho*c_p summed
 * over the node's cell octants; conduction between the two nodes of an edge
 * is k_e A_dual / L.  Forward Euler over dt_th with the mean Joule source
 * Pbar (per unit volume) held over the step; adiabatic (zero-flux) faces. */
void or_heat_capacity(const void *h, double *CV) {
    const grid_t *g = (const grid_t *)h;
    for (int k = 0; k <= g->nz; ++k)
        for (int j = 0; j <= g->ny; ++j)
            for (int i = 0; i <= g->nx; ++i) {
                double s = 0;
                for (int kk = k - 1; kk <= k; ++kk) for (int jj = j - 1; jj <= j; ++jj) for (int ii = i - 1; ii <= i; ++ii) {
                    if (ii < 0 || ii >= g->nx || jj < 0 || jj >= g->ny || kk < 0 || kk >= g->nz) continue;
                    s += prop(g, CI(g, ii, jj, kk), 4) * 0.125 * g->dx[ii] * g->dy[jj] * g->dz[kk];
                }
                CV[NI(g, i, j, k)] = s;
            }
}

static double cond_edge(const grid_t *g, int d, int i, int j, int k) {
    edge_mat_t m = edge_mat(g, d, i, j, k, 0.0);
    return m.kth * m.area / m.len;
}

void or_thermal_step(const void *h, double dt_th, const double *theta, const double *pbar, double *out) {
    const grid_t *g = (const grid_t *)h;
    int64_t nn = or_n_nodes(g);
    double *CV = (double *)malloc(sizeof(double) * (size_t)nn);
    or_heat_capacity(g, CV);
#pragma omp parallel for collapse(2) schedule(static)
    for (int k = 0; k <= g->nz; ++k)
        for (int j = 0; j <= g->ny; ++j)
            for (int i = 0; i <= g->nx; ++i) {
                int64_t n = NI(g, i, j, k);
                double t0 = theta[n], flux = 0;
                if (i > 0) flux += cond_edge(g, 0, i - 1, j, k) * (t0 - theta[NI(g, i - 1, j, k)]);
                if (i < g->nx) flux += cond_edge(g, 0, i, j, k) * (t0 - theta[NI(g, i + 1, j, k)]);
                if (j > 0) flux += cond_edge(g, 1, i, j - 1, k) * (t0 - theta[NI(g, i, j - 1, k)]);
                if (j < g->ny) flux += cond_edge(g, 1, i, j, k) * (t0 - theta[NI(g, i, j + 1, k)]);
                if (k > 0) flux += cond_edge(g, 2, i, j, k - 1) * (t0 - theta[NI(g, i, j, k - 1)]);
                if (k < g->nz) flux += cond_edge(g, 2, i, j, k) * (t0 - theta[NI(g, i, j, k + 1)]);
                double V = g->hx[i] * g->hy[j] * g->hz[k];
                out[n] = t0 + dt_th / CV[n] * (pbar[n] * V - flux);
            }
    free(CV);
}

/* ---------- discrete EM energy ------------------------------------------
 * W^{n+1/2} = 1/2 [ (e^{n+1}-e^n)^T D_eps (e^{n+1}-e^n) / dt^2 + e^{n+1 T} S e^n ],
 * conserved exactly by Eq. (2) without loss or source. */
double or_em_energy(const void *h, double dt, const double *ex0, const double *ey0, const double *ez0,
                    const double *ex1, const double *ey1, const double *ez1) {
    const grid_t *g = (const grid_t *)h;
    const double *e0[3] = {ex0, ey0, ez0}, *e1[3] = {ex1, ey1, ez1};
    double w = 0;
    for (int d = 0; d < 3; ++d) {
        int ni = g->nx + (d != 0), nj = g->ny + (d != 1), nk = g->nz + (d != 2);
        for (int k = 0; k < nk; ++k)
            for (int j = 0; j < nj; ++j)
                for (int i = 0; i < ni; ++i) {
                    if (pec_edge(g, d, i, j, k)) continue;
                    int64_t ei = edge_index(g, d, i, j, k);
                    edge_mat_t m = edge_mat(g, d, i, j, k, 0.0);
                    double dd = (e1[d][ei] - e0[d][ei]) / dt;
                    double s = curlcurl_edge(g, ex0, ey0, ez0, d, i, j, k);
                    w += m.len * m.area * (m.eps * dd * dd + e1[d][ei] * s);
                }
    }
    return 0.5 * w;
}

/* ---------- coupled march (Sec. II-A schedule) ---------------------------
 * Steps n0 .. n0+n_steps-1.  Each EM step uses sigma(T) of the current
 * temperature and adds its Joule power P^{n+1} to the block sum psum.  After
 * every R-th step the thermal update advances T over R*dt with the block mean
 * (R = 1 is the paper's synchronous schedule).  Histories every `stride`
 * steps: [step, W^{n+1/2}, cumulative Joule energy, max rise, probes...].
 * State is in/out: (e^n, e^{n-1}) in (ex,ey,ez),(exm,eym,ezm), theta, psum,
 * and *ejoule (cumulative dissipated energy). */
int or_run(void *h, double dt, int64_t n0, int64_t n_steps, int R, const double *J_half, int n_waves,
           int64_t n_samples, double *ex, double *ey, double *ez, double *exm, double *eym, double *ezm,
           double *theta, double *psum, double *ejoule, int stride, int n_probes, const int64_t *probes,
           double *hist, int64_t hist_cap) {
    grid_t *g = (grid_t *)h;
    int64_t ne[3] = {or_n_edges(g, 0), or_n_edges(g, 1), or_n_edges(g, 2)};
    int64_t nn = or_n_nodes(g);
    double *en[3], *P = (double *)malloc(sizeof(double) * (size_t)nn), *tn = (double *)malloc(sizeof(double) * (size_t)nn);
    double *pmean = (double *)malloc(sizeof(double) * (size_t)nn);
    for (int d = 0; d < 3; ++d) en[d] = (double *)malloc(sizeof(double) * (size_t)ne[d]);
    double *Jn = (double *)calloc((size_t)n_waves + 1, sizeof(double)), *Jo = (double *)calloc((size_t)n_waves + 1, sizeof(double));
    double *cur[3] = {ex, ey, ez}, *prv[3] = {exm, eym, ezm};
    int64_t rec = 0;
    for (int64_t n = n0; n < n0 + n_steps; ++n) {
        for (int w = 0; w < n_waves; ++w) {
            Jn[w] = (n + 1 < n_samples) ? J_half[(int64_t)w * n_samples + n + 1] : 0.0;
            Jo[w] = (n < n_samples) ? J_half[(int64_t)w * n_samples + n] : 0.0;
        }
        or_em_step(g, dt, theta, prv[0], prv[1], prv[2], cur[0], cur[1], cur[2], en[0], en[1], en[2], Jn, Jo);
        or_joule(g, theta, en[0], en[1], en[2], P);
        *ejoule += dt * or_joule_total(g, theta, en[0], en[1], en[2]);
        for (int64_t i = 0; i < nn; ++i) psum[i] += P[i];
        double W = (stride > 0 && (n + 1) % stride == 0) ? or_em_energy(g, dt, cur[0], cur[1], cur[2], en[0], en[1], en[2]) : 0.0;
        for (int d = 0; d < 3; ++d) { memcpy(prv[d], cur[d], sizeof(double) * (size_t)ne[d]); memcpy(cur[d], en[d], sizeof(double) * (size_t)ne[d]); }
        if ((n + 1) % R == 0) {
            for (int64_t i = 0; i < nn; ++i) pmean[i] = psum[i] / R;
            or_thermal_step(g, R * dt, theta, pmean, tn);
            memcpy(theta, tn, sizeof(double) * (size_t)nn);
            memset(psum, 0, sizeof(double) * (size_t)nn);
        }
        if (stride > 0 && (n + 1) % stride == 0 && hist && rec < hist_cap) {
            double *row = hist + rec * (4 + n_probes);
            double tmax = 0;
            for (int64_t i = 0; i < nn; ++i) tmax = fmax(tmax, theta[i]);
            row[0] = (double)(n + 1); row[1] = W; row[2] = *ejoule; row[3] = tmax;
            for (int p = 0; p < n_probes; ++p) {
                const int64_t *q = probes + 4 * p;
                int f = (int)q[0], i = (int)q[1], j = (int)q[2], k = (int)q[3];
                row[4 + p] = f == 3 ? theta[NI(g, i, j, k)] : cur[f][edge_index(g, f, i, j, k)];
            }
            ++rec;
        }
    }
    for (int d = 0; d < 3; ++d) free(en[d]);
    free(P); free(tn); free(pmean); free(Jn); free(Jo);
    return (int)rec;
}

/* ======================= thermo-mechanics, Eq. (7)-(9) ===================
 * HEX8 elements on the box cells, 2x2x2 Gauss quadrature.  Local node
 * a = ax + 2 ay + 4 az sits at (i+ax, j+ay, k+az).  Voigt order
 * [xx, yy, zz, xy, yz, zx] with engineering shear strains.  Void cells carry
 * no stiffness; fixed DOFs are given by a per-node 3-bit mask. */
static void elasticity_D(double E, double nu, double D[6][6]) {
    double lam = E * nu / ((1 + nu) * (1 - 2 * nu)), mu = E / (2 * (1 + nu));
    memset(D, 0, sizeof(double) * 36);
    for (int a = 0; a < 3; ++a) for (int b = 0; b < 3; ++b) D[a][b] = lam + (a == b ? 2 * mu : 0);
    D[3][3] = D[4][4] = D[5][5] = mu;
}

/* Shape functions and strain-displacement matrix B (6 x 24) at natural
 * coordinates (xi, eta, zeta) of a box of size hx*hy*hz. */
static void hex8_B(double xi, double eta, double zeta, double hx, double hy, double hz, double N[8], double B[6][24]) {
    memset(B, 0, sizeof(double) * 6 * 24);
    for (int a = 0; a < 8; ++a) {
        double sa = (a & 1) ? 1 : -1, ta = (a & 2) ? 1 : -1, ua = (a & 4) ? 1 : -1;
        N[a] = 0.125 * (1 + sa * xi) * (1 + ta * eta) * (1 + ua * zeta);
        double dx = 0.125 * sa * (1 + ta * eta) * (1 + ua * zeta) * 2.0 / hx;
        double dy = 0.125 * ta * (1 + sa * xi) * (1 + ua * zeta) * 2.0 / hy;
        double dz = 0.125 * ua * (1 + sa * xi) * (1 + ta * eta) * 2.0 / hz;
        B[0][3 * a + 0] = dx;
        B[1][3 * a + 1] = dy;
        B[2][3 * a + 2] = dz;
        B[3][3 * a + 0] = dy; B[3][3 * a + 1] = dx;
        B[4][3 * a + 1] = dz; B[4][3 * a + 2] = dy;
        B[5][3 * a + 0] = dz; B[5][3 * a + 2] = dx;
    }
}

static void cell_nodes(const grid_t *g, int i, int j, int k, int64_t nodes[8]) {
    for (int a = 0; a < 8; ++a) nodes[a] = NI(g, i + (a & 1), j + ((a >> 1) & 1), k + ((a >> 2) & 1));
}

/* Element stiffness Ke (24x24, Eq. 8 left side) and thermal load fe (Eq. 8
 * right side, eps_T = cte * dT(gauss point) [1,1,1,0,0,0]) of cell (i,j,k);
 * theta8 holds the temperature rise of the cell's 8 nodes (may be NULL). */
void or_hex8_element(const void *h, int i, int j, int k, const double *theta8, double *Ke, double *fe) {
    const grid_t *g = (const grid_t *)h;
    int64_t c = CI(g, i, j, k);
    if (Ke) memset(Ke, 0, sizeof(double) * 576);
    if (fe) memset(fe, 0, sizeof(double) * 24);
    if (prop(g, c, 8) != 0.0) return;
    double D[6][6], B[6][24], N[8];
    elasticity_D(prop(g, c, 5), prop(g, c, 6), D);
    double cte = prop(g, c, 7);
    double hx = g->dx[i], hy = g->dy[j], hz = g->dz[k], detJ = hx * hy * hz / 8.0;
    const double gp = 1.0 / sqrt(3.0);
    for (int q = 0; q < 8; ++q) {
        hex8_B((q & 1) ? gp : -gp, (q & 2) ? gp : -gp, (q & 4) ? gp : -gp, hx, hy, hz, N, B);
        double DB[6][24];
        for (int r = 0; r < 6; ++r)
            for (int col = 0; col < 24; ++col) {
                double s = 0;
                for (int m = 0; m < 6; ++m) s += D[r][m] * B[m][col];
                DB[r][col] = s;
            }
        if (Ke)
            for (int r = 0; r < 24; ++r)
                for (int col = 0; col < 24; ++col) {
                    double s = 0;
                    for (int m = 0; m < 6; ++m) s += B[m][r] * DB[m][col];
                    Ke[r * 24 + col] += s * detJ;
                }
        if (fe && theta8) {
            double th = 0;
            for (int a = 0; a < 8; ++a) th += N[a] * theta8[a];
            double epsT[6] = {cte * th, cte * th, cte * th, 0, 0, 0};
            double sig[6];
            for (int r = 0; r < 6; ++r) { sig[r] = 0; for (int m = 0; m < 6; ++m) sig[r] += D[r][m] * epsT[m]; }
            for (int r = 0; r < 24; ++r) {
                double s = 0;
                for (int m = 0; m < 6; ++m) s += B[m][r] * sig[m];
                fe[r] += s * detJ;
            }
        }
    }
}

/* Fixed-DOF mask per node (bit 0/1/2 = x/y/z).  mech_bc 0: kinematic
 * three-point mount on the bottom face (Sec. III-B): the node nearest the
 * centre fixed in x,y,z; the node on the +x edge at the centre's y fixed in
 * y,z; the node on the +y edge at the centre's x fixed in z.  mech_bc 1: every
 * bottom node fixed.  In both, nodes touched only by void cells are fixed. */
static int nearest_mid(const double *d, int n) {
    double x = 0, tot = 0;
    for (int i = 0; i < n; ++i) tot += d[i];
    double mid = 0.5 * tot, best = 1e300;
    int bi = 0;
    for (int i = 0; i <= n; ++i) {
        double dist = fabs(x - mid);
        if (dist < best) { best = dist; bi = i; }
        if (i < n) x += d[i];
    }
    return bi;
}

void or_mech_mask(const void *h, int mech_bc, uint8_t *mask) {
    const grid_t *g = (const grid_t *)h;
    for (int k = 0; k <= g->nz; ++k)
        for (int j = 0; j <= g->ny; ++j)
            for (int i = 0; i <= g->nx; ++i) {
                int solid = 0;
                for (int kk = k - 1; kk <= k; ++kk) for (int jj = j - 1; jj <= j; ++jj) for (int ii = i - 1; ii <= i; ++ii) {
                    if (ii < 0 || ii >= g->nx || jj < 0 || jj >= g->ny || kk < 0 || kk >= g->nz) continue;
                    if (prop(g, CI(g, ii, jj, kk), 8) == 0.0) solid = 1;
                }
                mask[NI(g, i, j, k)] = solid ? 0 : 7;
            }
    if (mech_bc == 1) {
        for (int j = 0; j <= g->ny; ++j) for (int i = 0; i <= g->nx; ++i) mask[NI(g, i, j, 0)] = 7;
    } else {
        int ic = nearest_mid(g->dx, g->nx), jc = nearest_mid(g->dy, g->ny);
        mask[NI(g, ic, jc, 0)] |= 7;
        mask[NI(g, g->nx, jc, 0)] |= 6;
        mask[NI(g, ic, g->ny, 0)] |= 4;
    }
}

/* Global thermal load f (3 per node), zero on fixed DOFs. */
void or_mech_rhs(const void *h, const double *theta, const uint8_t *mask, double *f) {
    const grid_t *g = (const grid_t *)h;
    int64_t nn = or_n_nodes(g);
    memset(f, 0, sizeof(double) * 3 * (size_t)nn);
    for (int k = 0; k < g->nz; ++k)
        for (int j = 0; j < g->ny; ++j)
            for (int i = 0; i < g->nx; ++i) {
                int64_t nd[8];
                double th8[8], fe[24];
                cell_nodes(g, i, j, k, nd);
                for (int a = 0; a < 8; ++a) th8[a] = theta[nd[a]];
                or_hex8_element(g, i, j, k, th8, NULL, fe);
                for (int a = 0; a < 8; ++a) for (int c = 0; c < 3; ++c) f[3 * nd[a] + c] += fe[3 * a + c];
            }
    for (int64_t n = 0; n < nn; ++n) for (int c = 0; c < 3; ++c) if (mask[n] >> c & 1) f[3 * n + c] = 0;
}

/* y = K q on the free DOFs (fixed rows return 0; q is taken as zero on fixed
 * DOFs).  Element matrices from a per-cell cache when given, else computed.
 * Cells are swept in 8 parity colours so no two threads share a node. */
static void mech_apply_impl(const grid_t *g, const uint8_t *mask, const double *q, double *y, const double *Kcache) {
    int64_t nn = or_n_nodes(g);
    memset(y, 0, sizeof(double) * 3 * (size_t)nn);
    for (int color = 0; color < 8; ++color) {
        int ci = color & 1, cj = (color >> 1) & 1, ck = (color >> 2) & 1;
#pragma omp parallel for collapse(2) schedule(dynamic, 1)
        for (int k = ck; k < g->nz; k += 2)
            for (int j = cj; j < g->ny; j += 2)
                for (int i = ci; i < g->nx; i += 2) {
                    int64_t c = CI(g, i, j, k);
                    if (prop(g, c, 8) != 0.0) continue;
                    double Kl[576];
                    const double *Ke = Kcache ? Kcache + 576 * c : Kl;
                    if (!Kcache) or_hex8_element(g, i, j, k, NULL, Kl, NULL);
                    int64_t nd[8];
                    cell_nodes(g, i, j, k, nd);
                    double qe[24];
                    for (int a = 0; a < 8; ++a) for (int cc = 0; cc < 3; ++cc)
                        qe[3 * a + cc] = (mask[nd[a]] >> cc & 1) ? 0.0 : q[3 * nd[a] + cc];
                    for (int r = 0; r < 24; ++r) {
                        double s = 0;
                        for (int col = 0; col < 24; ++col) s += Ke[r * 24 + col] * qe[col];
                        y[3 * nd[r / 3] + r % 3] += s;
                    }
                }
    }
    for (int64_t n = 0; n < nn; ++n) for (int c = 0; c < 3; ++c) if (mask[n] >> c & 1) y[3 * n + c] = 0;
}

void or_mech_apply(const void *h, const uint8_t *mask, const double *q, double *y) {
    mech_apply_impl((const grid_t *)h, mask, q, y, NULL);
}

/* Jacobi-preconditioned CG on K q = f over the free DOFs, stopping when the
 * true residual satisfies ||f - K q||_2 <= rtol ||f||_2.  q holds the initial
 * guess on entry.  Returns the iteration count, or -1 without convergence. */
int or_mech_solve(const void *h, const double *theta, const uint8_t *mask, double rtol, int maxit,
                  double *q, double *relres) {
    const grid_t *g = (const grid_t *)h;
    int64_t nn = or_n_nodes(g), nd = 3 * nn, ncell = (int64_t)g->nx * g->ny * g->nz;
    double *K = (double *)malloc(sizeof(double) * 576 * (size_t)ncell);
    for (int k = 0; k < g->nz; ++k) for (int j = 0; j < g->ny; ++j) for (int i = 0; i < g->nx; ++i)
        or_hex8_element(g, i, j, k, NULL, K + 576 * CI(g, i, j, k), NULL);
    double *f = (double *)malloc(sizeof(double) * nd), *r = (double *)malloc(sizeof(double) * nd);
    double *z = (double *)malloc(sizeof(double) * nd), *p = (double *)malloc(sizeof(double) * nd);
    double *Ap = (double *)malloc(sizeof(double) * nd), *dinv = (double *)calloc(nd, sizeof(double));
    or_mech_rhs(g, theta, mask, f);
    /* diagonal of K */
    for (int k = 0; k < g->nz; ++k) for (int j = 0; j < g->ny; ++j) for (int i = 0; i < g->nx; ++i) {
        int64_t c = CI(g, i, j, k), ndl[8];
        cell_nodes(g, i, j, k, ndl);
        for (int r2 = 0; r2 < 24; ++r2) dinv[3 * ndl[r2 / 3] + r2 % 3] += K[576 * c + r2 * 24 + r2];
    }
    for (int64_t a = 0; a < nd; ++a) {
        int fixed = mask[a / 3] >> (a % 3) & 1;
        dinv[a] = (fixed || dinv[a] == 0.0) ? 0.0 : 1.0 / dinv[a];
        if (fixed) q[a] = 0.0;
    }
    double fn = 0;
    for (int64_t a = 0; a < nd; ++a) fn += f[a] * f[a];
    fn = sqrt(fn);
    int it = 0, conv = 0;
    double rn = 0;
    if (fn == 0.0) { memset(q, 0, sizeof(double) * nd); if (relres) *relres = 0; goto done_ok; }
    for (;;) {
        /* (re)start from the true residual */
        mech_apply_impl(g, mask, q, Ap, K);
        rn = 0;
        for (int64_t a = 0; a < nd; ++a) { r[a] = f[a] - Ap[a]; rn += r[a] * r[a]; }
        rn = sqrt(rn);
        if (rn <= rtol * fn) { conv = 1; break; }
        if (it >= maxit) break;
        double rz = 0;
        for (int64_t a = 0; a < nd; ++a) { z[a] = dinv[a] * r[a]; p[a] = z[a]; rz += r[a] * z[a]; }
        while (it < maxit) {
            mech_apply_impl(g, mask, p, Ap, K);
            double pAp = 0;
            for (int64_t a = 0; a < nd; ++a) pAp += p[a] * Ap[a];
            double alpha = rz / pAp, rr = 0;
            for (int64_t a = 0; a < nd; ++a) { q[a] += alpha * p[a]; r[a] -= alpha * Ap[a]; rr += r[a] * r[a]; }
            ++it;
            if (sqrt(rr) <= rtol * fn) break;
            double rz2 = 0;
            for (int64_t a = 0; a < nd; ++a) { z[a] = dinv[a] * r[a]; rz2 += r[a] * z[a]; }
            double beta = rz2 / rz;
            rz = rz2;
            for (int64_t a = 0; a < nd; ++a) p[a] = z[a] + beta * p[a];
        }
    }
    if (relres) *relres = rn / fn;
done_ok:
    free(K); free(f); free(r); free(z); free(p); free(Ap); free(dinv);
    return conv || fn == 0.0 ? it : -1;
}

/* Stress at the element centroid, sigma = D (B(0) q_e - cte*dT_c [1,1,1,0,0,0])
 * with dT_c the centroid (mean nodal) rise, and Eq. (9) von Mises.  Void
 * cells give 0.  sig6 (6 per cell, optional) receives the stress vector. */
void or_von_mises(const void *h, const double *theta, const double *q, double *vm, double *sig6) {
    const grid_t *g = (const grid_t *)h;
#pragma omp parallel for collapse(2) schedule(static)
    for (int k = 0; k < g->nz; ++k)
        for (int j = 0; j < g->ny; ++j)
            for (int i = 0; i < g->nx; ++i) {
                int64_t c = CI(g, i, j, k);
                if (prop(g, c, 8) != 0.0) { vm[c] = 0; if (sig6) memset(sig6 + 6 * c, 0, 48); continue; }
                double D[6][6], B[6][24], N[8], eps[6] = {0}, s[6];
                elasticity_D(prop(g, c, 5), prop(g, c, 6), D);
                hex8_B(0, 0, 0, g->dx[i], g->dy[j], g->dz[k], N, B);
                int64_t nd[8];
                cell_nodes(g, i, j, k, nd);
                double th = 0;
                for (int a = 0; a < 8; ++a) th += N[a] * theta[nd[a]];
                for (int r = 0; r < 6; ++r)
                    for (int col = 0; col < 24; ++col) eps[r] += B[r][col] * q[3 * nd[col / 3] + col % 3];
                double cte = prop(g, c, 7);
                for (int r = 0; r < 3; ++r) eps[r] -= cte * th;
                for (int r = 0; r < 6; ++r) { s[r] = 0; for (int m = 0; m < 6; ++m) s[r] += D[r][m] * eps[m]; }
                double a1 = s[0] - s[1], a2 = s[1] - s[2], a3 = s[2] - s[0];
                vm[c] = sqrt(0.5 * (a1 * a1 + a2 * a2 + a3 * a3 + 6.0 * (s[3] * s[3] + s[4] * s[4] + s[5] * s[5])));
                if (sig6) for (int r = 0; r < 6; ++r) sig6[6 * c + r] = s[r];
            }
}

int or_num_threads(void) {
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}
