/*
 * Seeded synthetic SPD stencil matrices and vectors (CSR, int32 indices, fp64 values).
 *
 * Input construction only: nothing here computes any part of the adaptive FSAI method.
 * Both the FP64 oracle and the HIP library read what these routines write.
 *
 * Random numbers: counter-based SplitMix64 (Steele, Lea, Flood, "Fast splittable
 * pseudorandom number generators", OOPSLA 2014).  The k-th draw of stream `key` is
 * mix(key + (k+1)*0x9E3779B97F4A7C15), where mix is SplitMix64's output function.
 * U(0,1) = (u >> 11) * 2^-53.  N(0,1) by Box-Muller.
 *
 * Row ordering is lexicographic, x fastest: node = x + nx*(y + ny*z); with three
 * degrees of freedom per node, row = 3*node + dof.  Columns are strictly ascending
 * within every row and every matrix is stored with both triangles.  The two triangles
 * are bitwise equal: every entry a_ij is computed by the same operations, in the same
 * order, as a_ji.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define SM64_GAMMA 0x9E3779B97F4A7C15ULL

static inline uint64_t sm64_mix(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* key of stream `stream` under seed `seed` */
uint64_t synth_key(uint64_t seed, uint64_t stream)
{
    return sm64_mix(seed * SM64_GAMMA + sm64_mix(stream + 0x632BE59BD9B4E019ULL));
}

/* k-th 64-bit draw of the stream with key `key` */
static inline uint64_t sm64_at(uint64_t key, uint64_t k)
{
    return sm64_mix(key + (k + 1) * SM64_GAMMA);
}

static inline double u01(uint64_t u) { return (double)(u >> 11) * 0x1.0p-53; }

/* one standard normal from draws 2k, 2k+1 of the stream (Box-Muller, cosine branch) */
static inline double normal_at(uint64_t key, uint64_t k)
{
    double u1 = 1.0 - u01(sm64_at(key, 2 * k));      /* (0, 1] */
    double u2 = u01(sm64_at(key, 2 * k + 1));
    return sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
}

void synth_uniform(uint64_t seed, uint64_t stream, int64_t n, double lo, double hi, double *out)
{
    uint64_t key = synth_key(seed, stream);
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < n; ++k)
        out[k] = lo + (hi - lo) * u01(sm64_at(key, (uint64_t)k));
}

void synth_raw(uint64_t seed, uint64_t stream, int64_t n, uint64_t *out)
{
    uint64_t key = synth_key(seed, stream);
    for (int64_t k = 0; k < n; ++k) out[k] = sm64_at(key, (uint64_t)k);
}

void synth_normal(uint64_t seed, uint64_t stream, int64_t n, double *out)
{
    uint64_t key = synth_key(seed, stream);
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < n; ++k) out[k] = normal_at(key, (uint64_t)k);
}

/* y = A x, plain row loop (used once to form b = A x_true) */
void synth_matvec(int32_t n, const int32_t *rp, const int32_t *ci, const double *val,
                  const double *x, double *y)
{
#pragma omp parallel for schedule(static)
    for (int32_t i = 0; i < n; ++i) {
        double s = 0.0;
        for (int32_t e = rp[i]; e < rp[i + 1]; ++e) s += val[e] * x[ci[e]];
        y[i] = s;
    }
}

/* ------------------------------------------------------------------------------------
 * 7-point finite-difference operator on an nx*ny*nz grid of unknowns, homogeneous
 * Dirichlet boundary eliminated.  Constant coefficients (cx, cy, cz):
 *   diagonal 2(cx+cy+cz), off-diagonal -c_d towards each interior neighbour along d.
 * ---------------------------------------------------------------------------------- */
int64_t synth_lap7_nnz(int32_t nx, int32_t ny, int32_t nz)
{
    int64_t n = (int64_t)nx * ny * nz;
    return n + 2 * ((int64_t)(nx - 1) * ny * nz + (int64_t)nx * (ny - 1) * nz +
                    (int64_t)nx * ny * (nz - 1));
}

static void lap7_fill(int32_t nx, int32_t ny, int32_t nz, int lognormal,
                      double cx, double cy, double cz, uint64_t key, double sigma,
                      int32_t *rp, int32_t *ci, double *val);

void synth_lap7(int32_t nx, int32_t ny, int32_t nz, double cx, double cy, double cz,
                int32_t *rp, int32_t *ci, double *val)
{
    lap7_fill(nx, ny, nz, 0, cx, cy, cz, 0, 0.0, rp, ci, val);
}

/* 7-point operator with log-normal edge conductances: every grid edge (including the
 * edges to the eliminated boundary) carries w = exp(sigma * xi), xi ~ N(0,1) drawn from
 * the edge's own counter; off-diagonal -w, diagonal = sum of the six edge weights. */
void synth_lap7_lognormal(int32_t nx, int32_t ny, int32_t nz, double sigma, uint64_t seed,
                          int32_t *rp, int32_t *ci, double *val)
{
    lap7_fill(nx, ny, nz, 1, 0, 0, 0, synth_key(seed, 7), sigma, rp, ci, val);
}

/* weight of the edge from lower endpoint (x,y,z) (interior coordinates, may be -1) along d */
static inline double edge_w(int32_t nx, int32_t ny, int32_t x, int32_t y, int32_t z, int d,
                            uint64_t key, double sigma)
{
    int64_t lin = (int64_t)(x + 1) + (int64_t)(nx + 2) * ((y + 1) + (int64_t)(ny + 2) * (z + 1));
    return exp(sigma * normal_at(key, (uint64_t)(3 * lin + d)));
}

static void lap7_fill(int32_t nx, int32_t ny, int32_t nz, int lognormal, double cx, double cy,
                      double cz, uint64_t key, double sigma, int32_t *rp, int32_t *ci, double *val)
{
    int64_t n = (int64_t)nx * ny * nz;
    /* row pointers: count neighbours */
    rp[0] = 0;
    for (int64_t r = 0; r < n; ++r) {
        int32_t x = (int32_t)(r % nx), y = (int32_t)((r / nx) % ny), z = (int32_t)(r / ((int64_t)nx * ny));
        int32_t c = 1 + (x > 0) + (x < nx - 1) + (y > 0) + (y < ny - 1) + (z > 0) + (z < nz - 1);
        rp[r + 1] = rp[r] + c;
    }
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < n; ++r) {
        int32_t x = (int32_t)(r % nx), y = (int32_t)((r / nx) % ny), z = (int32_t)(r / ((int64_t)nx * ny));
        double wzm, wym, wxm, wxp, wyp, wzp;
        if (lognormal) {
            wxm = edge_w(nx, ny, x - 1, y, z, 0, key, sigma);
            wxp = edge_w(nx, ny, x, y, z, 0, key, sigma);
            wym = edge_w(nx, ny, x, y - 1, z, 1, key, sigma);
            wyp = edge_w(nx, ny, x, y, z, 1, key, sigma);
            wzm = edge_w(nx, ny, x, y, z - 1, 2, key, sigma);
            wzp = edge_w(nx, ny, x, y, z, 2, key, sigma);
        } else {
            wxm = wxp = cx;
            wym = wyp = cy;
            wzm = wzp = cz;
        }
        double diag = ((wxm + wxp) + (wym + wyp)) + (wzm + wzp);
        int32_t e = rp[r];
        int64_t sx = 1, sy = nx, sz = (int64_t)nx * ny;
        if (z > 0) { ci[e] = (int32_t)(r - sz); val[e++] = -wzm; }
        if (y > 0) { ci[e] = (int32_t)(r - sy); val[e++] = -wym; }
        if (x > 0) { ci[e] = (int32_t)(r - sx); val[e++] = -wxm; }
        ci[e] = (int32_t)r; val[e++] = diag;
        if (x < nx - 1) { ci[e] = (int32_t)(r + sx); val[e++] = -wxp; }
        if (y < ny - 1) { ci[e] = (int32_t)(r + sy); val[e++] = -wyp; }
        if (z < nz - 1) { ci[e] = (int32_t)(r + sz); val[e++] = -wzp; }
    }
}

/* ------------------------------------------------------------------------------------
 * 27-point, 3 degrees of freedom per node: trilinear-hexahedron-like assembly on an
 * N^3 grid of interior nodes ((N+2)^3 with the Dirichlet boundary layer, eliminated).
 * Each of the (N+1)^3 cells e contributes c_e (I_8 - 11^T/8) (x) M_e over its 8 corner
 * nodes, with c_e = exp(sigma*xi_e), xi_e ~ N(0,1), M_e = I_3 + w_e w_e^T, w_e ~ N(0,I_3).
 * Every term is positive semi-definite and the boundary elimination removes the constant
 * null space, so the assembled matrix is SPD.  Node couplings form the 27-point stencil
 * with dense 3x3 blocks.
 * ---------------------------------------------------------------------------------- */
int64_t synth_elast27_nnz(int32_t N)
{
    int64_t p = 3 * (int64_t)N - 2;
    return 9 * p * p * p;
}

int synth_elast27(int32_t N, double sigma, uint64_t seed, int32_t *rp, int32_t *ci, double *val)
{
    int64_t nc1 = (int64_t)N + 1, ncell = nc1 * nc1 * nc1;
    double *cell = (double *)malloc(sizeof(double) * 7 * ncell); /* c, then M (xx,xy,xz,yy,yz,zz) */
    if (!cell) return 1;
    uint64_t key = synth_key(seed, 27);
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < ncell; ++e) {
        double xi = normal_at(key, 4 * (uint64_t)e + 0);
        double w0 = normal_at(key, 4 * (uint64_t)e + 1);
        double w1 = normal_at(key, 4 * (uint64_t)e + 2);
        double w2 = normal_at(key, 4 * (uint64_t)e + 3);
        double *c = cell + 7 * e;
        c[0] = exp(sigma * xi);
        c[1] = 1.0 + w0 * w0; c[2] = w0 * w1; c[3] = w0 * w2;
        c[4] = 1.0 + w1 * w1; c[5] = w1 * w2; c[6] = 1.0 + w2 * w2;
    }
    int64_t nnode = (int64_t)N * N * N;
    /* row pointers */
    rp[0] = 0;
    for (int64_t a = 0; a < nnode; ++a) {
        int32_t x = (int32_t)(a % N), y = (int32_t)((a / N) % N), z = (int32_t)(a / ((int64_t)N * N));
        int32_t cnt = (1 + (x > 0) + (x < N - 1)) * (1 + (y > 0) + (y < N - 1)) * (1 + (z > 0) + (z < N - 1));
        for (int d = 0; d < 3; ++d) rp[3 * a + d + 1] = rp[3 * a + d] + 3 * cnt;
    }
    static const int midx[3][3] = {{1, 2, 3}, {2, 4, 5}, {3, 5, 6}};
#pragma omp parallel for schedule(static)
    for (int64_t a = 0; a < nnode; ++a) {
        /* interior node coordinates 1..N inside the (N+2)^3 grid; cells 0..N */
        int32_t x = (int32_t)(a % N) + 1, y = (int32_t)((a / N) % N) + 1, z = (int32_t)(a / ((int64_t)N * N)) + 1;
        for (int d = 0; d < 3; ++d) {
            int32_t e = rp[3 * a + d];
            for (int dz = -1; dz <= 1; ++dz) {
                int32_t bz = z + dz;
                if (bz < 1 || bz > N) continue;
                for (int dy = -1; dy <= 1; ++dy) {
                    int32_t by = y + dy;
                    if (by < 1 || by > N) continue;
                    for (int dx = -1; dx <= 1; ++dx) {
                        int32_t bx = x + dx;
                        if (bx < 1 || bx > N) continue;
                        int64_t b = (int64_t)(bx - 1) + (int64_t)N * ((by - 1) + (int64_t)N * (bz - 1));
                        double coef = (dx == 0 && dy == 0 && dz == 0) ? 0.875 : -0.125;
                        /* shared cells: lower corners in {x-1,x} intersect {bx-1,bx}, per axis */
                        int32_t cx0 = (dx < 0) ? x - 1 : ((dx > 0) ? x : x - 1);
                        int32_t cx1 = (dx < 0) ? x - 1 : x;
                        int32_t cy0 = (dy < 0) ? y - 1 : ((dy > 0) ? y : y - 1);
                        int32_t cy1 = (dy < 0) ? y - 1 : y;
                        int32_t cz0 = (dz < 0) ? z - 1 : ((dz > 0) ? z : z - 1);
                        int32_t cz1 = (dz < 0) ? z - 1 : z;
                        for (int dp = 0; dp < 3; ++dp) {
                            double s = 0.0;
                            for (int32_t qz = cz0; qz <= cz1; ++qz)
                                for (int32_t qy = cy0; qy <= cy1; ++qy)
                                    for (int32_t qx = cx0; qx <= cx1; ++qx) {
                                        const double *c = cell + 7 * ((int64_t)qx + nc1 * ((int64_t)qy + nc1 * qz));
                                        double m = c[midx[d][dp]];
                                        s += c[0] * (coef * m);
                                    }
                            ci[e] = (int32_t)(3 * b + dp);
                            val[e] = s;
                            ++e;
                        }
                    }
                }
            }
        }
    }
    free(cell);
    return 0;
}
