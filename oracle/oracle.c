/*
 * FP64 CPU oracle of the physics-embedded cloth method (arXiv 2403.12820).
 *
 * TEST INFRASTRUCTURE ONLY. The tests, the smoke check and the CPU-baseline leg of
 * the benchmark call it; the product library never does. It shares no code, header,
 * table or constant with the GPU path.
 *
 * Plain loops in double precision, one cloth instance per call, written in the
 * order the paper states each step:
 *   - mass-spring step: section 3.1, eqs. (1) elastic spring force, (2) spring
 *     damping, (3) uniform pressure on the four nearest neighbours, (4) gravity
 *     and air drag, (5) semi-implicit Euler with the constraint operator
 *     (Dirichlet pins, and a sphere handled by intersection elimination with
 *     friction);
 *   - physics-embedded CNN cell: section 3.2, eq. (6) one shared convolution
 *     applied to the state and to its time derivative, eq. (7) linear, nonlinear
 *     (ISRU) and derivative branches summed into a velocity increment, then
 *     eq. (5) again as the embedded integrator (Fig. 2), with wind and the
 *     pressure of eq. (3) added as known external forces;
 *   - its exact reverse mode (section 3.2.1: gradient backpropagation), the
 *     data term of the eq. (8) loss and Adam (Table 1);
 *   - section 3.2's own cell read literally ("pair cell": twelve frozen
 *     neighbour-difference channels shared by the three axes, per-channel branch
 *     weights, eqs. 6 and 7) with its reverse mode;
 *   - FP64 diagnostics: position RMS error, energy, stretch ratio.
 * Readings of passages the paper leaves open are listed in the design notes.
 *
 * State layout: six planes [x0 x1 x2 v0 v1 v2], each row-major H x W (node p = i*W + j).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ mass-spring */

/* Section 3.1: springs of the 13-point stencil. Each node links to the 8 nodes of its
   3x3 block and to the 4 nodes two steps away in the cardinal directions (the skip
   links that give bending). Columns: row offset, column offset, family
   (0 structural, rest length h; 1 shear, rest length sqrt(2) h; 2 bend, rest length 2h). */
static const int OR_NB[12][3] = {
    {0, 1, 0}, {0, -1, 0}, {1, 0, 0}, {-1, 0, 0},
    {1, 1, 1}, {1, -1, 1}, {-1, 1, 1}, {-1, -1, 1},
    {0, 2, 2}, {0, -2, 2}, {2, 0, 2}, {-2, 0, 2}};

typedef struct {
    double k[3];  /* spring constant per family (E of eq. 1) */
    double mu;    /* damping coefficient of eq. (2) */
    double drag;  /* air-drag coefficient d of eq. (4) */
    double g[3];  /* gravity acceleration of eq. (4) */
    double dt;    /* time step of eq. (5) */
} or_ms_params;

static double or_dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

/* Eq. (3): pressure on node (i, j) from its four nearest neighbours. Going round the node
   through right (0,+1), down (+1,0), left (0,-1) and up (-1,0), every consecutive pair
   (j1, j2) whose two nodes lie on the grid adds pr (x_j1 - x_i) x (x_j2 - x_i). With rows
   running down the grid this is the clockwise order, and on the flat rest grid
   X = (j h, i h, 0) each pair gives +h^2 along z, so pr > 0 pushes along +z (against
   gravity). Adds scale * force to F. */
static void or_pressure(int H, int W, const double *s, int i, int j, double scale, double *F)
{
    static const int R[4][2] = {{0, 1}, {1, 0}, {0, -1}, {-1, 0}};
    const long n = (long)H * W, p = (long)i * W + j;
    for (int k = 0; k < 4; ++k) {
        const int i1 = i + R[k][0], j1 = j + R[k][1];
        const int i2 = i + R[(k + 1) % 4][0], j2 = j + R[(k + 1) % 4][1];
        if (i1 < 0 || i1 >= H || j1 < 0 || j1 >= W || i2 < 0 || i2 >= H || j2 < 0 || j2 >= W) continue;
        double a[3], b[3];
        for (int c = 0; c < 3; ++c) {
            a[c] = s[c * n + (long)i1 * W + j1] - s[c * n + p];
            b[c] = s[c * n + (long)i2 * W + j2] - s[c * n + p];
        }
        F[0] += scale * (a[1] * b[2] - a[2] * b[1]);
        F[1] += scale * (a[2] * b[0] - a[0] * b[2]);
        F[2] += scale * (a[0] * b[1] - a[1] * b[0]);
    }
}

/* Total force on each node, f[3][H*W]; pinned nodes get zero.
   f_i = m (g + a_ext) - d v_i + sum_j [ -k_j (r - L_j) x_ij / r - mu ((v_ij . x_ij)/r^2) x_ij ]
         + f_p,i (eq. 3, pressure pr)
   with x_ij = x_i - x_j, v_ij = v_i - v_j, r = |x_ij|. */
void or_ms_force(int H, int W, double h, double m, const double *a_ext, double pr, const or_ms_params *P,
                 const uint8_t *pin, const double *s, double *f)
{
    const long n = (long)H * W;
    const double L[3] = {h, sqrt(2.0) * h, 2.0 * h};
    for (int i = 0; i < H; ++i)
        for (int j = 0; j < W; ++j) {
            const long p = (long)i * W + j;
            double F[3] = {0.0, 0.0, 0.0};
            if (!pin[p]) {
                for (int a = 0; a < 3; ++a)
                    F[a] = m * (P->g[a] + a_ext[a]) - P->drag * s[(3 + a) * n + p]; /* eq. (4) + wind */
                for (int q = 0; q < 12; ++q) {
                    const int ii = i + OR_NB[q][0], jj = j + OR_NB[q][1];
                    if (ii < 0 || ii >= H || jj < 0 || jj >= W) continue; /* spring needs both ends */
                    const long pj = (long)ii * W + jj;
                    const int fam = OR_NB[q][2];
                    double xij[3], vij[3];
                    for (int a = 0; a < 3; ++a) {
                        xij[a] = s[a * n + p] - s[a * n + pj];
                        vij[a] = s[(3 + a) * n + p] - s[(3 + a) * n + pj];
                    }
                    const double r = sqrt(or_dot3(xij, xij));
                    if (r < 1e-12 * h) continue;
                    const double ce = -P->k[fam] * (r - L[fam]) / r;        /* eq. (1) */
                    const double cd = -P->mu * or_dot3(vij, xij) / (r * r); /* eq. (2) */
                    for (int a = 0; a < 3; ++a) F[a] += (ce + cd) * xij[a];
                }
                if (pr != 0.0) or_pressure(H, W, s, i, j, pr, F);
            }
            for (int a = 0; a < 3; ++a) f[a * n + p] = F[a];
        }
}

/* The position update of eq. (5), x' = x + dt v', for a free node, with the constraint operator C
   extended by a sphere (section 3.1: cloth-object collision handled by intersection elimination;
   the ball of the fourth scene absorbs the bounce and its friction resists relative motion).
   If x + dt v lies inside the sphere (|y - c| < R), the node moves to the nearest surface point
   c + R n, n = (y - c)/|y - c|, its inward normal velocity is removed and its tangential velocity
   is scaled by 1 - fric. sphere = {cx, cy, cz, R, fric}; NULL or R <= 0: no sphere. v is in/out. */
static void or_sphere_update(const double *sphere, double dt, const double *x, double *v, double *y)
{
    for (int a = 0; a < 3; ++a) y[a] = x[a] + dt * v[a];
    if (!sphere || !(sphere[3] > 0.0)) return;
    double d[3];
    for (int a = 0; a < 3; ++a) d[a] = y[a] - sphere[a];
    const double r = sqrt(or_dot3(d, d));
    if (!(r < sphere[3])) return;
    double nn[3] = {0.0, 0.0, 1.0};
    if (r > 0.0)
        for (int a = 0; a < 3; ++a) nn[a] = d[a] / r;
    const double vn = or_dot3(v, nn);
    for (int a = 0; a < 3; ++a) {
        const double vt = v[a] - vn * nn[a];
        v[a] = (1.0 - sphere[4]) * vt + (vn > 0.0 ? vn : 0.0) * nn[a];
        y[a] = sphere[a] + sphere[3] * nn[a];
    }
}

/* Reverse mode of or_sphere_update for a free node. Given the adjoints gy of the new position and
   gw of the new velocity, returns gx (adjoint of x) and gv (adjoint of the velocity v before the
   constraint). Outside the sphere y = x + dt v, v' = v. Inside, with u = x + dt v - c, r = |u|,
   n = u / r, s = v . n and k = max(s, 0) - (1 - fric) s:
     y = c + R n,   v' = (1 - fric) v + k n,
   so by the chain rule
     g_s = (gw . n)([s > 0] - (1 - fric)),   g_n = R gy + k gw + g_s v,
     gv = (1 - fric) gw + g_s n + dt g_u,   gx = g_u = (g_n - (n . g_n) n) / r
   (dn/du = (I - n n^T) / r; n is the constant (0, 0, 1) at r = 0, where g_u = 0). */
static void or_sphere_adjoint(const double *sphere, double dt, const double *x, const double *v,
                              const double *gy, const double *gw, double *gx, double *gv)
{
    for (int a = 0; a < 3; ++a) { gx[a] = gy[a]; gv[a] = gw[a] + dt * gy[a]; }
    if (!sphere || !(sphere[3] > 0.0)) return;
    double d[3];
    for (int a = 0; a < 3; ++a) d[a] = x[a] + dt * v[a] - sphere[a];
    const double r = sqrt(or_dot3(d, d));
    if (!(r < sphere[3])) return;
    double nn[3] = {0.0, 0.0, 1.0};
    if (r > 0.0)
        for (int a = 0; a < 3; ++a) nn[a] = d[a] / r;
    const double kf = 1.0 - sphere[4];
    const double s = or_dot3(v, nn);
    const double k = (s > 0.0 ? s : 0.0) - kf * s;
    const double gs = or_dot3(gw, nn) * ((s > 0.0 ? 1.0 : 0.0) - kf);
    double gn[3], gu[3];
    for (int a = 0; a < 3; ++a) gn[a] = sphere[3] * gy[a] + k * gw[a] + gs * v[a];
    const double ngn = or_dot3(nn, gn);
    for (int a = 0; a < 3; ++a) gu[a] = r > 0.0 ? (gn[a] - ngn * nn[a]) / r : 0.0;
    for (int a = 0; a < 3; ++a) {
        gx[a] = gu[a];
        gv[a] = kf * gw[a] + gs * nn[a] + dt * gu[a];
    }
}

/* Adjoint of eq. (5) at node p with the constraint: from g_next at p, adds dLoss/dx^k to the
   position rows of g_cur and returns in gdv the adjoint of the velocity before the constraint
   (v = v^k + dv + external terms; zero for a pinned node, whose v' = 0 and x' = x). v is that
   velocity (needed only with a sphere). */
static void or_store_node_adjoint(long n, long p, int pinned, double dt, const double *s, const double *v,
                                  const double *sphere, const double *g_next, double *g_cur, double *gdv)
{
    double x[3], gy[3], gw[3], gx[3];
    for (int a = 0; a < 3; ++a) {
        x[a] = s[a * n + p];
        gy[a] = g_next[a * n + p];
        gw[a] = g_next[(3 + a) * n + p];
    }
    if (pinned) {
        for (int a = 0; a < 3; ++a) { gx[a] = gy[a]; gdv[a] = 0.0; }
    } else {
        or_sphere_adjoint(sphere, dt, x, v, gy, gw, gx, gdv);
    }
    for (int a = 0; a < 3; ++a) g_cur[a * n + p] += gx[a];
}

/* Writes node p of eq. (5): velocity v' (zero when pinned) and position, with the sphere. */
static void or_store_node(long n, long p, int pinned, double dt, const double *s, double *v,
                          const double *sphere, double *out)
{
    double x[3], y[3];
    for (int a = 0; a < 3; ++a) x[a] = s[a * n + p];
    if (pinned) {
        for (int a = 0; a < 3; ++a) { v[a] = 0.0; y[a] = x[a] + dt * v[a]; }
    } else {
        or_sphere_update(sphere, dt, x, v, y);
    }
    for (int a = 0; a < 3; ++a) {
        out[(3 + a) * n + p] = v[a];
        out[a * n + p] = y[a];
    }
}

/* One step of eq. (5): v' = C(v + dt f / m), x' = x + dt v'; C zeroes pinned velocities and
   handles the sphere. */
void or_ms_step(int H, int W, double h, double m, const double *a_ext, double pr, const or_ms_params *P,
                const uint8_t *pin, const double *s, double *out, const double *sphere)
{
    const long n = (long)H * W;
    double *f = (double *)malloc(sizeof(double) * 3 * n);
    or_ms_force(H, W, h, m, a_ext, pr, P, pin, s, f);
    for (long p = 0; p < n; ++p) {
        double v[3];
        for (int a = 0; a < 3; ++a) v[a] = s[(3 + a) * n + p] + P->dt * f[a * n + p] / m;
        or_store_node(n, p, pin[p], P->dt, s, v, sphere, out);
    }
    free(f);
}

/* n_steps consecutive steps; s is overwritten with the final state. */
void or_ms_run(int H, int W, double h, double m, const double *a_ext, double pr, const or_ms_params *P,
               const uint8_t *pin, double *s, int n_steps, const double *sphere)
{
    const long n = (long)H * W;
    double *t = (double *)malloc(sizeof(double) * 6 * n);
    for (int k = 0; k < n_steps; ++k) {
        or_ms_step(H, W, h, m, a_ext, pr, P, pin, s, t, sphere);
        memcpy(s, t, sizeof(double) * 6 * n);
    }
    free(t);
}

/* ------------------------------------------------------------------ diagnostics */

/* Energy: kinetic + spring (each spring once) - potential of gravity and wind. */
double or_energy(int H, int W, double h, double m, const double *a_ext, const or_ms_params *P,
                 const double *s)
{
    const long n = (long)H * W;
    const double L[3] = {h, sqrt(2.0) * h, 2.0 * h};
    double e = 0.0;
    for (int i = 0; i < H; ++i)
        for (int j = 0; j < W; ++j) {
            const long p = (long)i * W + j;
            for (int a = 0; a < 3; ++a) {
                const double v = s[(3 + a) * n + p];
                e += 0.5 * m * v * v - m * (P->g[a] + a_ext[a]) * s[a * n + p];
            }
            for (int q = 0; q < 12; ++q) {
                /* count each spring once: take the offsets pointing "forward" */
                const int di = OR_NB[q][0], dj = OR_NB[q][1];
                if (!(di > 0 || (di == 0 && dj > 0))) continue;
                const int ii = i + di, jj = j + dj;
                if (ii < 0 || ii >= H || jj < 0 || jj >= W) continue;
                const long pj = (long)ii * W + jj;
                double d[3];
                for (int a = 0; a < 3; ++a) d[a] = s[a * n + p] - s[a * n + pj];
                const double r = sqrt(or_dot3(d, d)) - L[OR_NB[q][2]];
                e += 0.5 * P->k[OR_NB[q][2]] * r * r;
            }
        }
    return e;
}

/* Largest r / L over structural springs (fam_mask bit f selects family f). */
double or_max_stretch(int H, int W, double h, const double *s, int fam_mask)
{
    const long n = (long)H * W;
    const double L[3] = {h, sqrt(2.0) * h, 2.0 * h};
    double best = 0.0;
    for (int i = 0; i < H; ++i)
        for (int j = 0; j < W; ++j)
            for (int q = 0; q < 12; ++q) {
                const int fam = OR_NB[q][2];
                if (!((fam_mask >> fam) & 1)) continue;
                const int ii = i + OR_NB[q][0], jj = j + OR_NB[q][1];
                if (ii < 0 || ii >= H || jj < 0 || jj >= W) continue;
                double d[3];
                for (int a = 0; a < 3; ++a) d[a] = s[a * n + (long)i * W + j] - s[a * n + (long)ii * W + jj];
                const double r = sqrt(or_dot3(d, d)) / L[fam];
                if (r > best) best = r;
            }
    return best;
}

/* Sum over nodes of |x - x_ref|^2 (the caller divides and takes the root). */
double or_sq_pos_err(int H, int W, const double *s, const double *ref)
{
    const long n = (long)H * W;
    double acc = 0.0;
    for (long p = 0; p < n; ++p)
        for (int a = 0; a < 3; ++a) {
            const double d = s[a * n + p] - ref[a * n + p];
            acc += d * d;
        }
    return acc;
}

/* ------------------------------------------------------------------ CNN cell */

/* Parameter vector (row-major): conv K[Ch][6][3][3] | A[Ch][Ch] | B[Ch][Ch] |
   W_L[3][Ch] | W_N[3][Ch] | W_D[3][Ch] | b_L[3]. */
typedef struct { long K, A, B, WL, WN, WD, bL, total; } or_layout;

static or_layout or_theta_layout(int ch)
{
    or_layout l;
    l.K = 0;
    l.A = l.K + (long)ch * 54;
    l.B = l.A + (long)ch * ch;
    l.WL = l.B + (long)ch * ch;
    l.WN = l.WL + 3L * ch;
    l.WD = l.WN + 3L * ch;
    l.bL = l.WD + 3L * ch;
    l.total = l.bL + 3;
    return l;
}

long or_theta_size(int ch) { return or_theta_layout(ch).total; }

static int or_clamp(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

/* bfloat16 round-to-nearest-even of a float value, returned as double. The operands of the
   bf16 products are float32 values in the library, so the argument is first taken to float
   (round to nearest); bfloat16 keeps the upper 16 bits of the float32 encoding, and the lower
   16 are rounded away to nearest, ties to the even upper half (a carry may reach the exponent,
   and past the largest finite value it gives infinity). Infinities and NaNs pass unchanged. */
static double or_bf16(double x)
{
    float f = (float)x;
    uint32_t u;
    memcpy(&u, &f, 4);
    if ((u & 0x7f800000u) == 0x7f800000u) return x; /* inf / nan unchanged */
    u += 0x7fffu + ((u >> 16) & 1u);
    u &= 0xffff0000u;
    memcpy(&f, &u, 4);
    return (double)f;
}

/* The rounding above over an array, for the tests that pin it. */
void or_bf16_array(long n, const double *x, double *y)
{
    for (long t = 0; t < n; ++t) y[t] = or_bf16(x[t]);
}

/* ISRU with parameter alpha (section 3.2): sigma(z) = z / sqrt(1 + alpha z^2). */
static double or_isru(double z, double al) { return z / sqrt(1.0 + al * z * z); }
static double or_isru_d(double z, double al) { double t = 1.0 + al * z * z; return 1.0 / (t * sqrt(t)); }

/* Input operator of the convolution for node (i, j): for each channel c and tap
   o = (dy, dx) in {-1, 0, 1}^2 the neighbour q = clamp(i+dy, j+dx) is read; position
   channels give the two-point difference with the central point S_c(q) - S_c(p)
   (section 3.2: correlations of each neighbour with the centre), velocity channels the
   raw value S_c(q). u[c*9 + (dy+1)*3 + (dx+1)].
   'emu' != 0 emulates a float32 subtraction before the value is used. */
static void or_im2col(int H, int W, const double *s, int i, int j, double *u, int emu)
{
    const long n = (long)H * W;
    const long p = (long)i * W + j;
    for (int c = 0; c < 6; ++c)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                const long q = (long)or_clamp(i + dy, 0, H - 1) * W + or_clamp(j + dx, 0, W - 1);
                double v = s[c * n + q];
                if (c < 3) {
                    v -= s[c * n + p];
                    if (emu) v = (double)(float)v;
                }
                u[c * 9 + (dy + 1) * 3 + (dx + 1)] = v;
            }
}

/* Forward quantities of the cell at one node, kept for the reverse pass. */
typedef struct {
    double uk[54], ud[54];             /* im2col of S^k and of S^k - S^{k-1} */
    double phi[64], xi[64];            /* eq. (6): conv of the state and of its time difference */
    double a[64], b[64], z[64];        /* z = (A phi) * (B phi) */
    double gs[64], nn[64], dd[64];     /* sigma(phi), sigma(z), xi * sigma(phi) */
    double dv[3];                      /* eq. (7): L + N + D */
} or_node;

/* emu bit 0: round conv operands (im2col entries and K) to bf16;
   bit 1: round the operands of the two Ch x Ch maps (phi, A, B) to bf16;
   bit 2: round the head operands (phi, n, d and W_L, W_N, W_D) to bf16. */
static void or_cell_node(int H, int W, int ch, double alpha, const double *th, const or_layout *Lo,
                         const double *sk, const double *dS, int i, int j, int emu, or_node *o)
{
    const int e0 = emu & 1, e1 = (emu >> 1) & 1, e2 = (emu >> 2) & 1;
    or_im2col(H, W, sk, i, j, o->uk, e0);
    or_im2col(H, W, dS, i, j, o->ud, e0);
    if (e0)
        for (int t = 0; t < 54; ++t) { o->uk[t] = or_bf16(o->uk[t]); o->ud[t] = or_bf16(o->ud[t]); }
    for (int c = 0; c < ch; ++c) {
        double pk = 0.0, pd = 0.0;
        for (int t = 0; t < 54; ++t) {
            const double w = e0 ? or_bf16(th[Lo->K + (long)c * 54 + t]) : th[Lo->K + (long)c * 54 + t];
            pk += w * o->uk[t];
            pd += w * o->ud[t];
        }
        o->phi[c] = pk;
        o->xi[c] = pd;
    }
    for (int r = 0; r < ch; ++r) {
        double sa = 0.0, sb = 0.0;
        for (int c = 0; c < ch; ++c) {
            const double ph = e1 ? or_bf16(o->phi[c]) : o->phi[c];
            const double wa = th[Lo->A + (long)r * ch + c], wb = th[Lo->B + (long)r * ch + c];
            sa += (e1 ? or_bf16(wa) : wa) * ph;
            sb += (e1 ? or_bf16(wb) : wb) * ph;
        }
        o->a[r] = sa;
        o->b[r] = sb;
        o->z[r] = sa * sb;
    }
    for (int c = 0; c < ch; ++c) {
        o->gs[c] = or_isru(o->phi[c], alpha);
        o->nn[c] = or_isru(o->z[c], alpha);
        o->dd[c] = o->xi[c] * o->gs[c];
    }
    for (int r = 0; r < 3; ++r) {
        double acc = th[Lo->bL + r];
        for (int c = 0; c < ch; ++c) {
            double wl = th[Lo->WL + r * ch + c], wn = th[Lo->WN + r * ch + c], wd = th[Lo->WD + r * ch + c];
            double fp = o->phi[c], fn = o->nn[c], fd = o->dd[c];
            if (e2) {
                wl = or_bf16(wl); wn = or_bf16(wn); wd = or_bf16(wd);
                fp = or_bf16(fp); fn = or_bf16(fn); fd = or_bf16(fd);
            }
            acc += wl * fp + wn * fn + wd * fd;
        }
        o->dv[r] = acc;
    }
}

/* Time difference S^k - S^{k-1} of the six planes (emu: rounded like a float32 subtraction). */
static double *or_time_diff(long n, const double *sp, const double *sk, int emu)
{
    double *d = (double *)malloc(sizeof(double) * 6 * n);
    for (long t = 0; t < 6 * n; ++t) {
        d[t] = sk[t] - sp[t];
        if (emu) d[t] = (double)(float)d[t];
    }
    return d;
}

/* One frame of the framework (Fig. 2): the cell gives dv, then eq. (5) with the pins and the
   hard-encoded external forces, wind and pressure (eq. 3 at the positions of S^k, per unit
   mass pm = pr / m): v' = C(v + dv + dt a_ext + dt pm sum_pairs (x_j1 - x) x (x_j2 - x)),
   x' = x + dt v'. */
void or_cnn_forward(int H, int W, int ch, double alpha, double dt, const double *a_ext, double pm,
                    const uint8_t *pin, const double *theta, const double *s_prev,
                    const double *s_cur, double *s_next, int emu, double *dv_out, const double *sphere)
{
    const long n = (long)H * W;
    const or_layout Lo = or_theta_layout(ch);
    double *dS = or_time_diff(n, s_prev, s_cur, emu & 1);
    or_node *o = (or_node *)malloc(sizeof(or_node));
    for (int i = 0; i < H; ++i)
        for (int j = 0; j < W; ++j) {
            const long p = (long)i * W + j;
            or_cell_node(H, W, ch, alpha, theta, &Lo, s_cur, dS, i, j, emu, o);
            double fp[3] = {0.0, 0.0, 0.0};
            if (pm != 0.0) or_pressure(H, W, s_cur, i, j, dt * pm, fp);
            double v[3];
            for (int a = 0; a < 3; ++a) {
                if (dv_out) dv_out[a * n + p] = o->dv[a];
                v[a] = s_cur[(3 + a) * n + p] + o->dv[a] + dt * a_ext[a] + fp[a];
            }
            or_store_node(n, p, pin[p], dt, s_cur, v, sphere, s_next);
        }
    free(o);
    free(dS);
}

/* Adjoint of c (x_j1 - x) x (x_j2 - x) summed over the pairs of node (i, j) (eq. 3), for the
   adjoint gdv of the velocity it is added to: with A = x_j1 - x, B = x_j2 - x,
   d/dx_j1 = c B x gdv, d/dx_j2 = c gdv x A, d/dx = minus both. Accumulates into g (positions). */
static void or_pressure_adjoint(int H, int W, const double *s, int i, int j, double c, const double *gdv,
                                double *g)
{
    static const int R[4][2] = {{0, 1}, {1, 0}, {0, -1}, {-1, 0}};
    const long n = (long)H * W, p = (long)i * W + j;
    for (int k = 0; k < 4; ++k) {
        const int i1 = i + R[k][0], j1 = j + R[k][1];
        const int i2 = i + R[(k + 1) % 4][0], j2 = j + R[(k + 1) % 4][1];
        if (i1 < 0 || i1 >= H || j1 < 0 || j1 >= W || i2 < 0 || i2 >= H || j2 < 0 || j2 >= W) continue;
        const long q1 = (long)i1 * W + j1, q2 = (long)i2 * W + j2;
        double A[3], B[3];
        for (int a = 0; a < 3; ++a) {
            A[a] = s[a * n + q1] - s[a * n + p];
            B[a] = s[a * n + q2] - s[a * n + p];
        }
        const double g1[3] = {c * (B[1] * gdv[2] - B[2] * gdv[1]), c * (B[2] * gdv[0] - B[0] * gdv[2]),
                              c * (B[0] * gdv[1] - B[1] * gdv[0])};
        const double g2[3] = {c * (gdv[1] * A[2] - gdv[2] * A[1]), c * (gdv[2] * A[0] - gdv[0] * A[2]),
                              c * (gdv[0] * A[1] - gdv[1] * A[0])};
        for (int a = 0; a < 3; ++a) {
            g[a * n + q1] += g1[a];
            g[a * n + q2] += g2[a];
            g[a * n + p] -= g1[a] + g2[a];
        }
    }
}

/* Reverse mode of or_cnn_forward (emu = 0). Given g_next = dLoss/dS^{k+1}, accumulate
   dLoss/dS^k into g_cur, dLoss/dS^{k-1} into g_prev and dLoss/dtheta into g_theta. */
void or_cnn_backward(int H, int W, int ch, double alpha, double dt, const double *a_ext, double pm,
                     const uint8_t *pin, const double *theta, const double *s_prev, const double *s_cur,
                     const double *g_next, double *g_cur, double *g_prev, double *g_theta,
                     const double *sphere)
{
    const long n = (long)H * W;
    const or_layout Lo = or_theta_layout(ch);
    double *dS = or_time_diff(n, s_prev, s_cur, 0);
    or_node *o = (or_node *)malloc(sizeof(or_node));
    double gdv[3], gphi[64], gxi[64], gnn[64], gdd[64], gz[64], ga[64], gb[64], guk[54], gud[54];
    for (int i = 0; i < H; ++i)
        for (int j = 0; j < W; ++j) {
            const long p = (long)i * W + j;
            or_cell_node(H, W, ch, alpha, theta, &Lo, s_cur, dS, i, j, 0, o);
            /* eq. (5): x' = x + dt v', v' = C(v + dv + dt a + pressure), C = pins and sphere */
            double v[3] = {0.0, 0.0, 0.0};
            if (sphere) {
                double fp[3] = {0.0, 0.0, 0.0};
                if (pm != 0.0) or_pressure(H, W, s_cur, i, j, dt * pm, fp);
                for (int a = 0; a < 3; ++a) v[a] = s_cur[(3 + a) * n + p] + o->dv[a] + dt * a_ext[a] + fp[a];
            }
            or_store_node_adjoint(n, p, pin[p], dt, s_cur, v, sphere, g_next, g_cur, gdv);
            for (int a = 0; a < 3; ++a) g_cur[(3 + a) * n + p] += gdv[a];
            if (pm != 0.0) or_pressure_adjoint(H, W, s_cur, i, j, dt * pm, gdv, g_cur);
            /* eq. (7) heads */
            for (int c = 0; c < ch; ++c) { gphi[c] = 0.0; gnn[c] = 0.0; gdd[c] = 0.0; }
            for (int r = 0; r < 3; ++r) {
                g_theta[Lo.bL + r] += gdv[r];
                for (int c = 0; c < ch; ++c) {
                    g_theta[Lo.WL + r * ch + c] += gdv[r] * o->phi[c];
                    g_theta[Lo.WN + r * ch + c] += gdv[r] * o->nn[c];
                    g_theta[Lo.WD + r * ch + c] += gdv[r] * o->dd[c];
                    gphi[c] += theta[Lo.WL + r * ch + c] * gdv[r];
                    gnn[c] += theta[Lo.WN + r * ch + c] * gdv[r];
                    gdd[c] += theta[Lo.WD + r * ch + c] * gdv[r];
                }
            }
            /* derivative branch d = xi * sigma(phi); nonlinear branch n = sigma(z) */
            for (int c = 0; c < ch; ++c) {
                gxi[c] = gdd[c] * o->gs[c];
                gphi[c] += gdd[c] * o->xi[c] * or_isru_d(o->phi[c], alpha);
                gz[c] = gnn[c] * or_isru_d(o->z[c], alpha);
                ga[c] = gz[c] * o->b[c];
                gb[c] = gz[c] * o->a[c];
            }
            for (int r = 0; r < ch; ++r)
                for (int c = 0; c < ch; ++c) {
                    g_theta[Lo.A + (long)r * ch + c] += ga[r] * o->phi[c];
                    g_theta[Lo.B + (long)r * ch + c] += gb[r] * o->phi[c];
                    gphi[c] += theta[Lo.A + (long)r * ch + c] * ga[r] + theta[Lo.B + (long)r * ch + c] * gb[r];
                }
            /* eq. (6) conv */
            for (int t = 0; t < 54; ++t) { guk[t] = 0.0; gud[t] = 0.0; }
            for (int c = 0; c < ch; ++c)
                for (int t = 0; t < 54; ++t) {
                    const double w = theta[Lo.K + (long)c * 54 + t];
                    g_theta[Lo.K + (long)c * 54 + t] += gphi[c] * o->uk[t] + gxi[c] * o->ud[t];
                    guk[t] += w * gphi[c];
                    gud[t] += w * gxi[c];
                }
            /* adjoint of the input operator: the tap value of (c, o) came from S_c(q) and, for
               positions, minus S_c(p); the time difference is S^k - S^{k-1}. */
            for (int c = 0; c < 6; ++c)
                for (int dy = -1; dy <= 1; ++dy)
                    for (int dx = -1; dx <= 1; ++dx) {
                        const int t = c * 9 + (dy + 1) * 3 + (dx + 1);
                        const long q = (long)or_clamp(i + dy, 0, H - 1) * W + or_clamp(j + dx, 0, W - 1);
                        g_cur[c * n + q] += guk[t] + gud[t];
                        g_prev[c * n + q] -= gud[t];
                        if (c < 3) {
                            g_cur[c * n + p] -= guk[t] + gud[t];
                            g_prev[c * n + p] += gud[t];
                        }
                    }
        }
    free(o);
    free(dS);
}

/* ------------------------------------------------------------------ the paper's own cell */

/* Section 3.2 read literally ("pair cell"). Twelve channels, one per neighbour of the 13-point
   stencil, in the order of the springs above. The filter of channel c is predetermined: +s_c at
   its neighbour j, -s_c at the centre, zero (frozen) elsewhere, and the same 2-D filter acts on
   each axis. Eq. (6) applies it to x^k and to v^k:
     phi_c = s_c (x_j - x_i),  xi_c = s_c (v_j - v_i)   (3-vectors; zero when j is off the grid).
   Eq. (7), axis by axis, summed over the channels, bias once:
     dv = sum_c [ wL_c phi_c + wN_c sigma(phi_c) + wD_c xi_c * sigma(phi_c) ] + b_L.
   Then eq. (5) with pins, wind and pressure as for the other cell.
   theta: s[12] | wL[12] | wN[12] | wD[12] | bL[3]. */
enum { OR_PS = 0, OR_PWL = 12, OR_PWN = 24, OR_PWD = 36, OR_PBL = 48, OR_PTOTAL = 51 };
long or_pair_theta_size(void) { return OR_PTOTAL; }

static void or_pair_node(int H, int W, double alpha, const double *th, const double *s, int i, int j,
                         double *dv)
{
    const long n = (long)H * W, p = (long)i * W + j;
    for (int a = 0; a < 3; ++a) dv[a] = th[OR_PBL + a];
    for (int c = 0; c < 12; ++c) {
        const int ii = i + OR_NB[c][0], jj = j + OR_NB[c][1];
        if (ii < 0 || ii >= H || jj < 0 || jj >= W) continue;
        const long q = (long)ii * W + jj;
        for (int a = 0; a < 3; ++a) {
            const double phi = th[OR_PS + c] * (s[a * n + q] - s[a * n + p]);
            const double xi = th[OR_PS + c] * (s[(3 + a) * n + q] - s[(3 + a) * n + p]);
            const double sg = or_isru(phi, alpha);
            dv[a] += th[OR_PWL + c] * phi + th[OR_PWN + c] * sg + th[OR_PWD + c] * xi * sg;
        }
    }
}

/* One frame with the pair cell: v' = C(v + dv + dt a_ext + dt pm f_p(x)), x' = x + dt v'. */
void or_pair_forward(int H, int W, double alpha, double dt, const double *a_ext, double pm,
                     const uint8_t *pin, const double *theta, const double *s_cur, double *s_next,
                     double *dv_out, const double *sphere)
{
    const long n = (long)H * W;
    for (int i = 0; i < H; ++i)
        for (int j = 0; j < W; ++j) {
            const long p = (long)i * W + j;
            double dv[3], fp[3] = {0.0, 0.0, 0.0};
            or_pair_node(H, W, alpha, theta, s_cur, i, j, dv);
            if (pm != 0.0) or_pressure(H, W, s_cur, i, j, dt * pm, fp);
            double v[3];
            for (int a = 0; a < 3; ++a) {
                if (dv_out) dv_out[a * n + p] = dv[a];
                v[a] = s_cur[(3 + a) * n + p] + dv[a] + dt * a_ext[a] + fp[a];
            }
            or_store_node(n, p, pin[p], dt, s_cur, v, sphere, s_next);
        }
}

/* Reverse mode of or_pair_forward: g_next = dLoss/dS^{k+1} gives dLoss/dS^k (into g_cur) and
   dLoss/dtheta (into g_theta). */
void or_pair_backward(int H, int W, double alpha, double dt, const double *a_ext, double pm,
                      const uint8_t *pin, const double *theta, const double *s_cur, const double *g_next,
                      double *g_cur, double *g_theta, const double *sphere)
{
    const long n = (long)H * W;
    for (int i = 0; i < H; ++i)
        for (int j = 0; j < W; ++j) {
            const long p = (long)i * W + j;
            double gdv[3], v[3] = {0.0, 0.0, 0.0};
            if (sphere) {  /* the velocity before the constraint, as in or_pair_forward */
                double dv[3], fp[3] = {0.0, 0.0, 0.0};
                or_pair_node(H, W, alpha, theta, s_cur, i, j, dv);
                if (pm != 0.0) or_pressure(H, W, s_cur, i, j, dt * pm, fp);
                for (int a = 0; a < 3; ++a) v[a] = s_cur[(3 + a) * n + p] + dv[a] + dt * a_ext[a] + fp[a];
            }
            or_store_node_adjoint(n, p, pin[p], dt, s_cur, v, sphere, g_next, g_cur, gdv);
            for (int a = 0; a < 3; ++a) {
                g_cur[(3 + a) * n + p] += gdv[a];
                g_theta[OR_PBL + a] += gdv[a];
            }
            if (pm != 0.0) or_pressure_adjoint(H, W, s_cur, i, j, dt * pm, gdv, g_cur);
            for (int c = 0; c < 12; ++c) {
                const int ii = i + OR_NB[c][0], jj = j + OR_NB[c][1];
                if (ii < 0 || ii >= H || jj < 0 || jj >= W) continue;
                const long q = (long)ii * W + jj;
                const double sc = theta[OR_PS + c];
                for (int a = 0; a < 3; ++a) {
                    const double d = s_cur[a * n + q] - s_cur[a * n + p];
                    const double e = s_cur[(3 + a) * n + q] - s_cur[(3 + a) * n + p];
                    const double phi = sc * d, xi = sc * e;
                    const double sg = or_isru(phi, alpha), sgd = or_isru_d(phi, alpha);
                    g_theta[OR_PWL + c] += gdv[a] * phi;
                    g_theta[OR_PWN + c] += gdv[a] * sg;
                    g_theta[OR_PWD + c] += gdv[a] * xi * sg;
                    const double gphi = gdv[a] * (theta[OR_PWL + c] + (theta[OR_PWN + c] + theta[OR_PWD + c] * xi) * sgd);
                    const double gxi = gdv[a] * theta[OR_PWD + c] * sg;
                    g_theta[OR_PS + c] += gphi * d + gxi * e;
                    g_cur[a * n + q] += sc * gphi;
                    g_cur[a * n + p] -= sc * gphi;
                    g_cur[(3 + a) * n + q] += sc * gxi;
                    g_cur[(3 + a) * n + p] -= sc * gxi;
                }
            }
        }
}

/* ------------------------------------------------------------------ loss and Adam */

/* Data term of eq. (8), normalised per field: w / n_free * sum over free nodes of
   |x_hat - x|^2 / sx^2 + |v_hat - v|^2 / sv^2. Adds d/ds_hat into g (if non-null). */
double or_loss_mse(long n, const uint8_t *pin, long n_free, double sx, double sv, double w,
                   const double *s_hat, const double *s_true, double *g)
{
    double acc = 0.0;
    for (int c = 0; c < 6; ++c) {
        const double sc = c < 3 ? sx : sv;
        for (long p = 0; p < n; ++p) {
            if (pin[p]) continue;
            const double d = s_hat[c * n + p] - s_true[c * n + p];
            acc += d * d / (sc * sc);
            if (g) g[c * n + p] += w * 2.0 * d / (sc * sc * (double)n_free);
        }
    }
    return w * acc / (double)n_free;
}

/* Adam (Kingma and Ba), step t >= 1, bias-corrected. */
void or_adam(long n, double lr, double b1, double b2, double eps, int t, double *th, double *m,
             double *v, const double *g)
{
    for (long i = 0; i < n; ++i) {
        m[i] = b1 * m[i] + (1.0 - b1) * g[i];
        v[i] = b2 * v[i] + (1.0 - b2) * g[i] * g[i];
        const double mh = m[i] / (1.0 - pow(b1, t));
        const double vh = v[i] / (1.0 - pow(b2, t));
        th[i] -= lr * mh / (sqrt(vh) + eps);
    }
}
