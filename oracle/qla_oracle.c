/*
 * Plain FP64 CPU oracle for the qubit lattice algorithm (QLA) time step for the
 * 2D Maxwell equations in an isotropic inhomogeneous dielectric n(x, y).
 *
 * TEST INFRASTRUCTURE ONLY. Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg load this code. It shares nothing with the GPU
 * library: no headers, helpers, tables or kernels.
 *
 * The oracle is the algorithm itself, written operator by operator in the
 * paper's order and notation, one full-lattice pass per operator, FP64
 * throughout:
 *   - qubit vector Q = (q0..q5) = (n Ex, n Ey, n Ez, Bx, By, Bz), Eq. (3b3);
 *   - collision C_x, Eq. (2e3), angles Eq. (2e4); collision C_y, Eq. (2e8);
 *   - streaming S^{+-x}_{14}, S^{+-x}_{25}, Eq. (2e5), and their y analogues
 *     S^{+-y}_{03}, S^{+-y}_{25} (Section IV);
 *   - U_x, Eq. (2e6); U_y, Eq. (2e9): products of 16 operators, the rightmost
 *     applied first;
 *   - potentials V_x, V_y, Eqs. (2e11)-(2e13);
 *   - the full step Q(t + dt) = V_y V_x U_y U_x Q(t), Eq. (2e14);
 *   - the energy ||Q||^2, Eq. (A13).
 * Each 6x6 operator is built as the dense matrix printed in the paper and
 * applied as a dense matrix-vector product at every site.
 *
 * Readings of points the paper leaves open (each also listed in the design
 * notes):
 *   - S^{+-}: the streamed amplitude at x takes the value found at x +- 1 cell
 *     (Eq. 2e5 writes q(x +- delta)); the lattice is periodic in x and y.
 *   - Each collision and potential uses the refractive index of the site it
 *     acts on (collisions are on-site, Section V-A).
 *   - The garbled pair "{q_, q4}" of Section IV is {q1, q4}, from Eq. (2e5).
 *   - dn/dx, dn/dy in Eq. (2e13): centred differences of the sampled n,
 *     (n[x+1] - n[x-1]) / (2 delta), periodic.
 *   - Potential mode V_PAPER: Eqs. (2e11)-(2e12) with two printed-entry
 *     corrections: V_x row q5 is (0, +sin b0, 0, 0, 0, cos b0), which is what
 *     the LCU sum (2f1)-(2f4) gives and what the source term of Eq. (2d6)
 *     needs; V_y row q3 is (0, 0, sin b3, cos b3, 0, 0), so that V_y = I at
 *     b3 = 0 and the source term of Eq. (2d4) has its printed sign.
 *   - Potential mode V_SKEW_HALF (default): the unitary collision-shaped
 *     potentials V_x = C_x(theta1 -> +b0/2, theta2 -> -b2/2) and
 *     V_y = C_y(theta0 -> +b1/2, theta2 -> -b3/2). With site-dependent angles
 *     the unitary U_x recovers the symmetrised operator
 *     (1/2)[(1/n) d/dx + d/dx (1/n)]; these half-angle rotations add exactly
 *     the skew remainder that turns it into the Maxwell form of
 *     Eqs. (2d1)-(2d6). The test suite pins this by second-order convergence
 *     to a spectral solution of Eqs. (2d1)-(2d6).
 *   - V_NONE: potentials off (the homogeneous-medium scheme of Eq. 2e10).
 *   - V_BSTREAM (beyond the paper, E_z triple): U_x and U_y built only from the sets
 *     of Eqs. (2e6) and (2e9) that stream the B-qubit of the pair (S14 along x, S03
 *     along y), each used twice, and no potentials. A set that streams the B-qubit puts
 *     the angle of the E-qubit's site on the neighbour pair, which to first order
 *     gives dt q2 = (1/n) d q4 and dt q4 = d(q2 / n): the Maxwell form of
 *     Eqs. (2d3)-(2d5) without a potential. Pinned by the same convergence and
 *     Fresnel tests as V_SKEW_HALF.
 */
#include <math.h>
#include <stddef.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

enum { V_SKEW_HALF = 0, V_PAPER = 1, V_NONE = 2, V_BSTREAM = 3 };

/* Operator codes for single-operator application (tests drive these). */
enum {
    OP_CX = 0, OP_CX_DAG, OP_CY, OP_CY_DAG,
    OP_S14_PX, OP_S14_MX, OP_S25_PX, OP_S25_MX,
    OP_S03_PY, OP_S03_MY, OP_S25_PY, OP_S25_MY,
    OP_VX, OP_VY, OP_UX, OP_UY, OP_STEP,
    OP_COUNT
};

/* Eq. (2e6) exactly as printed, left to right; the rightmost factor acts first. */
static const int UX_AS_PRINTED[16] = {
    OP_S25_PX, OP_CX_DAG, OP_S25_MX, OP_CX,
    OP_S14_MX, OP_CX_DAG, OP_S14_PX, OP_CX,
    OP_S25_MX, OP_CX, OP_S25_PX, OP_CX_DAG,
    OP_S14_PX, OP_CX, OP_S14_MX, OP_CX_DAG,
};

/* Eq. (2e9) exactly as printed, left to right; the rightmost factor acts first. */
static const int UY_AS_PRINTED[16] = {
    OP_S25_PY, OP_CY_DAG, OP_S25_MY, OP_CY,
    OP_S03_MY, OP_CY_DAG, OP_S03_PY, OP_CY,
    OP_S25_MY, OP_CY, OP_S25_PY, OP_CY_DAG,
    OP_S03_PY, OP_CY, OP_S03_MY, OP_CY_DAG,
};

/* V_BSTREAM (a scheme beyond the paper, for the E_z triple): the sets of Eq. (2e6) that
 * stream the E-qubit q2 (S25) are replaced by copies of the neighbouring sets that
 * stream the B-qubit q4 (S14), which couple the same neighbour pairs with the same
 * rotation sense; likewise in Eq. (2e9) with S03. No potentials. Same notation as
 * above: as printed, the rightmost factor acts first. In acting order the x sets are
 * (C+, S14-, C, S14+) twice, then (C, S14+, C+, S14-) twice. */
static const int UX_BSTREAM[16] = {
    OP_S14_MX, OP_CX_DAG, OP_S14_PX, OP_CX,
    OP_S14_MX, OP_CX_DAG, OP_S14_PX, OP_CX,
    OP_S14_PX, OP_CX, OP_S14_MX, OP_CX_DAG,
    OP_S14_PX, OP_CX, OP_S14_MX, OP_CX_DAG,
};
static const int UY_BSTREAM[16] = {
    OP_S03_MY, OP_CY_DAG, OP_S03_PY, OP_CY,
    OP_S03_MY, OP_CY_DAG, OP_S03_PY, OP_CY,
    OP_S03_PY, OP_CY, OP_S03_MY, OP_CY_DAG,
    OP_S03_PY, OP_CY, OP_S03_MY, OP_CY_DAG,
};

typedef double mat6[6][6];

/* Lattices smaller than this run each pass on one thread (fork/join would dominate). */
#define PARALLEL_MIN_SITES 8192

/* Per-site cosines and sines of every angle a step needs. */
typedef struct {
    double *base;      /* one allocation holding every array below */
    double *ct, *st;   /* collision angle theta = delta / (4 n), Eq. (2e4) */
    double *cbx, *sbx; /* potential angle along x (beta_2 = beta_0, or its half) */
    double *cby, *sby; /* potential angle along y (beta_3 = beta_1, or its half) */
} site_angles;

static size_t site(int nx, int x, int y) { return (size_t)y * (size_t)nx + (size_t)x; }
static int wrap(int i, int n) { return ((i % n) + n) % n; }

/* Eq. (2e3) with c1 = cos theta1, s1 = sin theta1, c2 = cos theta2, s2 = sin theta2. */
static void collision_x(double c1, double s1, double c2, double s2, mat6 M)
{
    memset(M, 0, sizeof(mat6));
    M[0][0] = 1.0;
    M[1][1] = c1;  M[1][5] = -s1;
    M[2][2] = c2;  M[2][4] = -s2;
    M[3][3] = 1.0;
    M[4][2] = s2;  M[4][4] = c2;
    M[5][1] = s1;  M[5][5] = c1;
}

/* Eq. (2e8) with c0 = cos theta0, s0 = sin theta0, c2 = cos theta2, s2 = sin theta2. */
static void collision_y(double c0, double s0, double c2, double s2, mat6 M)
{
    memset(M, 0, sizeof(mat6));
    M[0][0] = c0;  M[0][5] = s0;
    M[1][1] = 1.0;
    M[2][2] = c2;  M[2][3] = s2;
    M[3][2] = -s2; M[3][3] = c2;
    M[4][4] = 1.0;
    M[5][0] = -s0; M[5][5] = c0;
}

/* Eq. (2e11), row q5 with +sin b0 (LCU sum, Eqs. 2f1-2f4). */
static void potential_x_paper(double cb0, double sb0, double cb2, double sb2, mat6 M)
{
    memset(M, 0, sizeof(mat6));
    M[0][0] = 1.0;
    M[1][1] = 1.0;
    M[2][2] = 1.0;
    M[3][3] = 1.0;
    M[4][2] = -sb2; M[4][4] = cb2;
    M[5][1] = sb0;  M[5][5] = cb0;
}

/* Eq. (2e12), row q3 = (0, 0, sin b3, cos b3, 0, 0). */
static void potential_y_paper(double cb1, double sb1, double cb3, double sb3, mat6 M)
{
    memset(M, 0, sizeof(mat6));
    M[0][0] = 1.0;
    M[1][1] = 1.0;
    M[2][2] = 1.0;
    M[3][2] = sb3;  M[3][3] = cb3;
    M[4][4] = 1.0;
    M[5][0] = -sb1; M[5][5] = cb1;
}

/* y <- M x (or M^T x) at every site; the six planes are q[c * N + s]. */
static void apply_local(int nx, int ny, double *q, const site_angles *A, int op, int vmode)
{
    const size_t N = (size_t)nx * (size_t)ny;
    if (op != OP_CX && op != OP_CX_DAG && op != OP_CY && op != OP_CY_DAG && op != OP_VX &&
        op != OP_VY)
        return;
#pragma omp parallel for schedule(static) if (N >= PARALLEL_MIN_SITES)
    for (int y = 0; y < ny; ++y) {
        for (int x = 0; x < nx; ++x) {
            const size_t s = site(nx, x, y);
            mat6 M;
            int transpose = 0;
            switch (op) {
            case OP_CX: case OP_CX_DAG:
                collision_x(A->ct[s], A->st[s], A->ct[s], A->st[s], M);
                transpose = (op == OP_CX_DAG);
                break;
            case OP_CY: case OP_CY_DAG:
                collision_y(A->ct[s], A->st[s], A->ct[s], A->st[s], M);
                transpose = (op == OP_CY_DAG);
                break;
            case OP_VX:
                if (vmode == V_PAPER)
                    potential_x_paper(A->cbx[s], A->sbx[s], A->cbx[s], A->sbx[s], M);
                else /* skew-half: C_x with theta1 = +b0/2, theta2 = -b2/2 */
                    collision_x(A->cbx[s], A->sbx[s], A->cbx[s], -A->sbx[s], M);
                break;
            case OP_VY:
                if (vmode == V_PAPER)
                    potential_y_paper(A->cby[s], A->sby[s], A->cby[s], A->sby[s], M);
                else /* skew-half: C_y with theta0 = +b1/2, theta2 = -b3/2 */
                    collision_y(A->cby[s], A->sby[s], A->cby[s], -A->sby[s], M);
                break;
            }
            double v[6], w[6];
            for (int c = 0; c < 6; ++c) v[c] = q[(size_t)c * N + s];
            for (int r = 0; r < 6; ++r) {
                double acc = 0.0;
                for (int c = 0; c < 6; ++c) acc += (transpose ? M[c][r] : M[r][c]) * v[c];
                w[r] = acc;
            }
            for (int c = 0; c < 6; ++c) q[(size_t)c * N + s] = w[c];
        }
    }
}

/* Streaming, Eq. (2e5): q_c(x, y) <- q_c(x + dx, y + dy) for the two listed components. */
static void stream(int nx, int ny, double *q, int ca, int cb, int dx, int dy, double *tmp)
{
    const size_t N = (size_t)nx * (size_t)ny;
    const int comps[2] = { ca, cb };
    for (int k = 0; k < 2; ++k) {
        double *p = q + (size_t)comps[k] * N;
#pragma omp parallel for schedule(static) if (N >= PARALLEL_MIN_SITES)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x)
                tmp[site(nx, x, y)] = p[site(nx, wrap(x + dx, nx), wrap(y + dy, ny))];
        memcpy(p, tmp, N * sizeof(double));
    }
}

static void apply_op(int op, int nx, int ny, double *q, const site_angles *A, int vmode,
                     double *tmp)
{
    switch (op) {
    case OP_S14_PX: stream(nx, ny, q, 1, 4, +1, 0, tmp); break;
    case OP_S14_MX: stream(nx, ny, q, 1, 4, -1, 0, tmp); break;
    case OP_S25_PX: stream(nx, ny, q, 2, 5, +1, 0, tmp); break;
    case OP_S25_MX: stream(nx, ny, q, 2, 5, -1, 0, tmp); break;
    case OP_S03_PY: stream(nx, ny, q, 0, 3, 0, +1, tmp); break;
    case OP_S03_MY: stream(nx, ny, q, 0, 3, 0, -1, tmp); break;
    case OP_S25_PY: stream(nx, ny, q, 2, 5, 0, +1, tmp); break;
    case OP_S25_MY: stream(nx, ny, q, 2, 5, 0, -1, tmp); break;
    case OP_VX: case OP_VY:
        if (vmode == V_NONE || vmode == V_BSTREAM) break;
        apply_local(nx, ny, q, A, op, vmode);
        break;
    case OP_UX: {
        const int *ops = vmode == V_BSTREAM ? UX_BSTREAM : UX_AS_PRINTED;
        for (int i = 15; i >= 0; --i) apply_op(ops[i], nx, ny, q, A, vmode, tmp);
        break;
    }
    case OP_UY: {
        const int *ops = vmode == V_BSTREAM ? UY_BSTREAM : UY_AS_PRINTED;
        for (int i = 15; i >= 0; --i) apply_op(ops[i], nx, ny, q, A, vmode, tmp);
        break;
    }
    case OP_STEP: /* Eq. (2e14): V_y V_x U_y U_x */
        apply_op(OP_UX, nx, ny, q, A, vmode, tmp);
        apply_op(OP_UY, nx, ny, q, A, vmode, tmp);
        apply_op(OP_VX, nx, ny, q, A, vmode, tmp);
        apply_op(OP_VY, nx, ny, q, A, vmode, tmp);
        break;
    default:
        apply_local(nx, ny, q, A, op, vmode);
        break;
    }
}

/* theta = delta / (4 n), Eq. (2e4); beta = delta^2 (dn/dx) / n^2, Eq. (2e13), with the
 * centred difference dn/dx = (n[x+1] - n[x-1]) / (2 delta). */
int qla_oracle_coefficients(int nx, int ny, double delta, const double *n,
                            double *theta, double *beta_x, double *beta_y)
{
    if (nx < 1 || ny < 1 || !(delta > 0.0) || !n) return -1;
#pragma omp parallel for schedule(static)
    for (int y = 0; y < ny; ++y) {
        for (int x = 0; x < nx; ++x) {
            const size_t s = site(nx, x, y);
            const double nn = n[s];
            const double dndx = (n[site(nx, wrap(x + 1, nx), y)] - n[site(nx, wrap(x - 1, nx), y)])
                                / (2.0 * delta);
            const double dndy = (n[site(nx, x, wrap(y + 1, ny))] - n[site(nx, x, wrap(y - 1, ny))])
                                / (2.0 * delta);
            if (theta) theta[s] = delta / (4.0 * nn);
            if (beta_x) beta_x[s] = delta * delta * dndx / (nn * nn);
            if (beta_y) beta_y[s] = delta * delta * dndy / (nn * nn);
        }
    }
    return 0;
}

static int build_angles(int nx, int ny, double delta, int vmode, const double *n, site_angles *A)
{
    const size_t N = (size_t)nx * (size_t)ny;
    double *buf = (double *)malloc(9 * N * sizeof(double));
    if (!buf) return -2;
    double *theta = buf, *bx = buf + N, *by = buf + 2 * N;
    A->base = buf;
    A->ct = buf + 3 * N; A->st = buf + 4 * N;
    A->cbx = buf + 5 * N; A->sbx = buf + 6 * N;
    A->cby = buf + 7 * N; A->sby = buf + 8 * N;
    qla_oracle_coefficients(nx, ny, delta, n, theta, bx, by);
    /* V_PAPER uses the full beta; V_SKEW_HALF rotates by half of it. */
    const double scale = (vmode == V_PAPER) ? 1.0 : 0.5;
#pragma omp parallel for schedule(static)
    for (long long s = 0; s < (long long)N; ++s) {
        A->ct[s] = cos(theta[s]);
        A->st[s] = sin(theta[s]);
        A->cbx[s] = cos(scale * bx[s]);
        A->sbx[s] = sin(scale * bx[s]);
        A->cby[s] = cos(scale * by[s]);
        A->sby[s] = sin(scale * by[s]);
    }
    return 0;
}

static int check_args(int nx, int ny, double delta, int vmode, const double *n, const double *q)
{
    if (nx < 1 || ny < 1 || !(delta > 0.0) || !n || !q) return -1;
    if (vmode != V_SKEW_HALF && vmode != V_PAPER && vmode != V_NONE && vmode != V_BSTREAM)
        return -1;
    return 0;
}

/* Apply one operator (an OP_* code) to the six planes q[6][ny][nx] in place. */
int qla_oracle_apply(int op, int nx, int ny, double delta, int vmode, const double *n, double *q)
{
    if (check_args(nx, ny, delta, vmode, n, q) || op < 0 || op >= OP_COUNT) return -1;
    site_angles A;
    if (build_angles(nx, ny, delta, vmode, n, &A)) return -2;
    double *tmp = (double *)malloc((size_t)nx * (size_t)ny * sizeof(double));
    if (!tmp) { free(A.base); return -2; }
    apply_op(op, nx, ny, q, &A, vmode, tmp);
    free(tmp);
    free(A.base);
    return 0;
}

/* Advance q[6][ny][nx] by `steps` full steps of Eq. (2e14). */
int qla_oracle_advance(int nx, int ny, double delta, int vmode, const double *n, double *q,
                       long long steps)
{
    if (check_args(nx, ny, delta, vmode, n, q) || steps < 0) return -1;
    site_angles A;
    if (build_angles(nx, ny, delta, vmode, n, &A)) return -2;
    double *tmp = (double *)malloc((size_t)nx * (size_t)ny * sizeof(double));
    if (!tmp) { free(A.base); return -2; }
    for (long long t = 0; t < steps; ++t) apply_op(OP_STEP, nx, ny, q, &A, vmode, tmp);
    free(tmp);
    free(A.base);
    return 0;
}

/* Energy, Eq. (A13): the sum of q_c^2 over all six components and all sites, without
 * the cell-area factor. Summed row by row in a fixed order. */
double qla_oracle_energy(int nx, int ny, const double *q)
{
    const size_t N = (size_t)nx * (size_t)ny;
    double total = 0.0;
    for (int c = 0; c < 6; ++c) {
        const double *p = q + (size_t)c * N;
        for (size_t s = 0; s < N; ++s) total += p[s] * p[s];
    }
    return total;
}

/* Initial Gaussian-envelope plane-wave packet in E_z (Section V, "QLA 2D Initial
 * Conditions"), paired with the magnetic field of a wave travelling one way along the
 * direction phi in a uniform medium:
 *   Ez0 = amp exp(-r^2 / (2 sigma^2)) cos(2 pi s / lam),
 *   q2 = n Ez0 (Eq. 3b3), q3 = Bx = q2 sin(phi), q4 = By = -q2 cos(phi).
 * s is the minimum-image displacement from (x0, y0) projected on the direction of
 * travel; r = s for a planar packet, else the full minimum-image distance. */
int qla_oracle_packet(int nx, int ny, const double *n, double x0, double y0, double sigma,
                      double lam, double phi, double amp, int planar, double *q)
{
    if (nx < 1 || ny < 1 || !n || !q || !(sigma > 0.0) || !(lam > 0.0)) return -1;
    const size_t N = (size_t)nx * (size_t)ny;
    const double kx = cos(phi), ky = sin(phi);
    const double pi = 3.14159265358979323846;
    for (int y = 0; y < ny; ++y) {
        double dy = (double)y - y0;
        dy -= (double)ny * floor(dy / (double)ny + 0.5);
        for (int x = 0; x < nx; ++x) {
            double dx = (double)x - x0;
            dx -= (double)nx * floor(dx / (double)nx + 0.5);
            const double s = dx * kx + dy * ky;
            const double r2 = planar ? s * s : dx * dx + dy * dy;
            const double ez = amp * exp(-r2 / (2.0 * sigma * sigma)) * cos(2.0 * pi * s / lam);
            const size_t i = site(nx, x, y);
            const double q2 = n[i] * ez;
            q[0 * N + i] = 0.0;
            q[1 * N + i] = 0.0;
            q[2 * N + i] = q2;
            q[3 * N + i] = q2 * ky;
            q[4 * N + i] = -q2 * kx;
            q[5 * N + i] = 0.0;
        }
    }
    return 0;
}

int qla_oracle_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
