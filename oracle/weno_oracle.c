/*
 * FP64 CPU oracle for Weighted Direction (WD) WENO 2x image zooming
 * (Crnkovic, Skific, Bosner, "WENO based adaptive image zooming algorithm",
 * arXiv 2312.00229).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * statement of what the GPU path computes.  Only the test-suite, the smoke
 * check and the CPU-baseline leg of the benchmark may load it.  It shares no
 * code, header or constant with the HIP library.
 *
 * Everything is written on the paper's fine grid (Section 3): original
 * samples sit at even/even fine indices (2I, 2J), the "x" points of phase 1
 * at odd/odd indices, the "+" points of phase 2 at mixed parity.  The fine
 * index i runs along the first array axis (image rows), j along the second.
 *
 * Readings of passages the paper leaves open (each one is a switch or a
 * documented default):
 *   - boundary: input samples outside the image are clamped to the edge;
 *     function tests instead pass an input that already extends >= 5 samples
 *     beyond the domain and crop the result;
 *   - direction vector d^gamma (eq. Vektor): one fine-grid step, i.e. length
 *     h*sqrt(2)/2 on the diagonals (phase 1) and h/2 on the axes (phase 2);
 *   - smoothness-indicator scale (eq. 2Dsmoothness): `si_mode` 0 uses the
 *     length of the integration interval (sqrt(2)h in phase 1, h in phase 2),
 *     `si_mode` 1 uses sqrt(2)h literally in both phases;
 *   - output: 2n x 2m samples, the last fine row and column computed by the
 *     same formulas on the padded grid; the paper's (2n-1)x(2m-1) grid is the
 *     leading crop;
 *   - algorithms 1 and 2 loop over all four directions k = 0..3.
 *
 * Build: gcc -O2 -fopenmp -shared -fPIC weno_oracle.c -o libweno_oracle.so -lm
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    double beta;   /* exponent of the nonlinear weights, eq. (alpha)              */
    double keps;   /* K_eps, eps_h = K_eps h^2 (Section 2, eq. IzrazOmega)        */
    double h;      /* coarse (input) grid spacing                                  */
    double nbw;    /* neighbour-indicator weight; < 0 selects h^2/8, the value in
                      the proof of Theorem 1 (eq. DDiffOrder) that reproduces
                      Table 1 row 2; eqs. 2DsmoothnessFinal and tezine print
                      h^2/4, which callers pass explicitly                        */
    int si_mode;   /* 0: interval-length scale, 1: literal sqrt(2)h scale          */
} weno_oracle_params;

#define WO_OK 0
#define WO_EINVAL -1
#define WO_ENOMEM -2

/* Fine-grid margin around the 2n x 2m output: phase-2 points need +-1 for
 * their neighbour indicators and +-3 for their stencils, phase-1 points +-2
 * and +-3 again, which reaches 9 fine cells; 12 leaves slack. */
#define FM 12

typedef struct {
    int rows, cols; /* 2n + 2FM, 2m + 2FM */
    double* a;
} fgrid;

static int fg_alloc(fgrid* g, int n, int m)
{
    g->rows = 2 * n + 2 * FM;
    g->cols = 2 * m + 2 * FM;
    g->a = (double*)calloc((size_t)g->rows * (size_t)g->cols, sizeof(double));
    return g->a ? 0 : -1;
}

static void fg_free(fgrid* g)
{
    free(g->a);
    g->a = NULL;
}

/* element at fine index (i, j); i, j may be negative down to -FM */
#define AT(g, i, j) ((g).a[(size_t)((i) + FM) * (size_t)(g).cols + (size_t)((j) + FM)])

static int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }
static int is_odd(int v) { return (v % 2 + 2) % 2 == 1; }

/* ---------------------------------------------------------------------------
 * One-dimensional building blocks (Section 2 and eqs. p, 2Dsmoothness).
 *
 * A stencil S^gamma = {c - d, c + d, c + 3d} holds samples a, b, c.  With the
 * local coordinate t = (x - c)/|d| the nodes are t = -1, 1, 3 and the
 * interpolating quadratic in Newton form is
 *     q(t) = a + f1 (t + 1) + f2 (t + 1)(t - 1),
 *     f1 = (b - a)/2,  f2 = (c - 2b + a)/8.
 * ------------------------------------------------------------------------- */
static void newton_coeffs(double a, double b, double c, double* f1, double* f2)
{
    *f1 = (b - a) / 2.0;
    *f2 = ((c - b) / 2.0 - (b - a) / 2.0) / 4.0;
}

/* value of the stencil quadratic at its centre point c (t = 0), eq. (p) */
static double candidate(double a, double b, double c)
{
    double f1, f2;
    newton_coeffs(a, b, c, &f1, &f2);
    return a + f1 * (0.0 + 1.0) + f2 * (0.0 + 1.0) * (0.0 - 1.0);
}

/* Smoothness indicator, eq. (2Dsmoothness):
 *   SI = sum_{l=1,2} int_{c-d}^{c+d} scale^(2l-1) (d^l q / dx^l)^2 dx,
 * with x = c + t|d| (so dx = |d| dt, d/dx = (1/|d|) d/dt):
 *   dq/dt = f1 + 2 f2 t,  d2q/dt2 = 2 f2,
 *   int_{-1}^{1} (f1 + 2 f2 t)^2 dt = 2 f1^2 + (8/3) f2^2,
 *   int_{-1}^{1} (2 f2)^2 dt = 8 f2^2. */
static double indicator(double a, double b, double c, double step, double scale)
{
    double f1, f2;
    newton_coeffs(a, b, c, &f1, &f2);
    double i1 = (2.0 * f1 * f1 + (8.0 / 3.0) * f2 * f2) / step;   /* int (q')^2 dx  */
    double i2 = (8.0 * f2 * f2) / (step * step * step);           /* int (q'')^2 dx */
    return scale * i1 + scale * scale * scale * i2;
}

/* partial derivatives of candidate() and indicator() with respect to (a, b, c) */
static void candidate_grad(double g[3])
{
    /* q(0) = a + f1 - f2; df1/d(a,b,c) = (-1/2, 1/2, 0); df2 = (1/8, -1/4, 1/8) */
    g[0] = 1.0 - 0.5 - 0.125;
    g[1] = 0.5 + 0.25;
    g[2] = -0.125;
}

static void indicator_grad(double a, double b, double c, double step, double scale, double g[3])
{
    double f1, f2;
    newton_coeffs(a, b, c, &f1, &f2);
    double dS_df1 = scale * (4.0 * f1) / step;
    double dS_df2 = scale * ((16.0 / 3.0) * f2) / step
                  + scale * scale * scale * (16.0 * f2) / (step * step * step);
    g[0] = dS_df1 * (-0.5) + dS_df2 * 0.125;
    g[1] = dS_df1 * (0.5) + dS_df2 * (-0.25);
    g[2] = dS_df2 * 0.125;
}

/* ---------------------------------------------------------------------------
 * Directions, eq. (defgammak): gamma_k = gamma_0 + k pi/2.  On the fine grid
 * d^gamma is one fine step (si, sj) with si = sign(cos gamma), sj = sign(sin
 * gamma) on the diagonals and (cos, sin) on the axes.
 * ------------------------------------------------------------------------- */
static const int DIAG[4][2] = {{1, 1}, {-1, 1}, {-1, -1}, {1, -1}}; /* gamma_0 = pi/4 */
static const int AXIS[4][2] = {{1, 0}, {0, 1}, {-1, 0}, {0, -1}};   /* gamma_0 = 0    */

/* neighbour offsets of the combined indicator D:
 *   phase 1, eq. (2DsmoothnessFinal): (0,+-2), (+-2,0)
 *   phase 2, eq. (tezine):             (+-1,+-1) */
static const int NB1[4][2] = {{0, 2}, {2, 0}, {0, -2}, {-2, 0}};
static const int NB2[4][2] = {{1, 1}, {-1, -1}, {-1, 1}, {1, -1}};

typedef struct {
    int n, m;
    double beta, eps, nbw;
    double step1, step2, scale1, scale2;
    fgrid F;       /* fine-grid values: originals, then x points, then + points */
    fgrid P[4];    /* candidate values p^gamma_k at the current phase's points  */
    fgrid S[4];    /* smoothness indicators SI^gamma_k                          */
    fgrid T[4];    /* eps + D^gamma_k                                           */
} wo_state;

static void st_free(wo_state* s)
{
    fg_free(&s->F);
    for (int k = 0; k < 4; ++k) {
        fg_free(&s->P[k]);
        fg_free(&s->S[k]);
        fg_free(&s->T[k]);
    }
}

static int st_init(wo_state* s, const double* V, int n, int m, const weno_oracle_params* p)
{
    memset(s, 0, sizeof(*s));
    s->n = n;
    s->m = m;
    s->beta = p->beta;
    s->eps = p->keps * p->h * p->h;
    s->nbw = p->nbw < 0.0 ? p->h * p->h / 8.0 : p->nbw;
    s->step1 = sqrt(2.0) / 2.0 * p->h;
    s->step2 = p->h / 2.0;
    if (p->si_mode == 1) {
        s->scale1 = sqrt(2.0) * p->h;
        s->scale2 = sqrt(2.0) * p->h;
    } else {
        s->scale1 = 2.0 * s->step1;
        s->scale2 = 2.0 * s->step2;
    }
    int bad = fg_alloc(&s->F, n, m);
    for (int k = 0; k < 4; ++k) {
        bad |= fg_alloc(&s->P[k], n, m);
        bad |= fg_alloc(&s->S[k], n, m);
        bad |= fg_alloc(&s->T[k], n, m);
    }
    if (bad) {
        st_free(s);
        return WO_ENOMEM;
    }
    /* originals at even/even fine indices, padded by clamping to the edge */
    for (int i = -FM; i < 2 * n + FM; ++i) {
        if (is_odd(i)) continue;
        for (int j = -FM; j < 2 * m + FM; ++j) {
            if (is_odd(j)) continue;
            int I = clampi(i / 2, 0, n - 1);
            int J = clampi(j / 2, 0, m - 1);
            AT(s->F, i, j) = V[(size_t)I * (size_t)m + (size_t)J];
        }
    }
    return WO_OK;
}

/* Does fine point (i, j) belong to the class handled by `phase`?
 * phase 1: odd/odd ("x"); phase 2: mixed parity ("+"). */
static int in_class(int phase, int i, int j)
{
    if (phase == 1) return is_odd(i) && is_odd(j);
    return is_odd(i) != is_odd(j);
}

/* candidates and indicators of every point of the class within fine range [lo, hi) */
static void stencil_pass(wo_state* s, int phase, int lo, int hi_i, int hi_j)
{
    const int (*dir)[2] = phase == 1 ? DIAG : AXIS;
    double step = phase == 1 ? s->step1 : s->step2;
    double scale = phase == 1 ? s->scale1 : s->scale2;
    #pragma omp parallel for schedule(static)
    for (int i = lo; i < hi_i; ++i) {
        for (int j = lo; j < hi_j; ++j) {
            if (!in_class(phase, i, j)) continue;
            for (int k = 0; k < 4; ++k) {
                int si = dir[k][0], sj = dir[k][1];
                double a = AT(s->F, i - si, j - sj);      /* x - d  */
                double b = AT(s->F, i + si, j + sj);      /* x + d  */
                double c = AT(s->F, i + 3 * si, j + 3 * sj); /* x + 3d */
                AT(s->P[k], i, j) = candidate(a, b, c);
                AT(s->S[k], i, j) = indicator(a, b, c, step, scale);
            }
        }
    }
}

/* combined indicators, nonlinear weights and the blend, eqs. (2DsmoothnessFinal),
 * (alpha), (IzrazOmega2d), (2dKombinacija) for phase 1 and (tezine),
 * (IzrazOmega2dRavno), (2dKombinacijaRavno) for phase 2; the accumulation
 * follows algorithms 1 and 2: u = sum alpha p, then u /= sum alpha. */
static void blend_pass(wo_state* s, int phase, int lo, int hi_i, int hi_j)
{
    const int (*nb)[2] = phase == 1 ? NB1 : NB2;
    #pragma omp parallel for schedule(static)
    for (int i = lo; i < hi_i; ++i) {
        for (int j = lo; j < hi_j; ++j) {
            if (!in_class(phase, i, j)) continue;
            double u = 0.0, asum = 0.0;
            for (int k = 0; k < 4; ++k) {
                double nsum = 0.0;
                for (int q = 0; q < 4; ++q) nsum += AT(s->S[k], i + nb[q][0], j + nb[q][1]);
                double D = AT(s->S[k], i, j) + s->nbw * nsum;
                double t = s->eps + D;
                AT(s->T[k], i, j) = t;
                double alpha = 0.5 / pow(t, s->beta);
                u += alpha * AT(s->P[k], i, j);
                asum += alpha;
            }
            AT(s->F, i, j) = u / asum;
        }
    }
}

/* fine-index ranges (lower bound, and upper bound relative to 2n / 2m):
 * phase 1 stencils on [-9, 2n+9), phase 1 blend on [-7, 2n+7),
 * phase 2 stencils on [-4, 2n+4), phase 2 blend on [-3, 2n+3). */
static void forward_all(wo_state* s)
{
    int n2 = 2 * s->n, m2 = 2 * s->m;
    stencil_pass(s, 1, -9, n2 + 9, m2 + 9);
    blend_pass(s, 1, -7, n2 + 7, m2 + 7);
    stencil_pass(s, 2, -4, n2 + 4, m2 + 4);
    blend_pass(s, 2, -3, n2 + 3, m2 + 3);
}

static int check_args(const double* V, int n, int m, const weno_oracle_params* p, const void* out)
{
    if (!V || !p || !out || n < 1 || m < 1) return WO_EINVAL;
    if (!(p->beta >= 0.0) || !(p->h > 0.0) || !(p->keps >= 0.0)) return WO_EINVAL;
    return WO_OK;
}

/* U: 2n x 2m, row-major.  U[2I][2J] = V[I][J]; U[2I+1][2J+1] = x point;
 * U[2I+1][2J] and U[2I][2J+1] = + points. */
int weno_oracle_zoom2x(const double* V, int n, int m, const weno_oracle_params* p, double* U)
{
    int rc = check_args(V, n, m, p, U);
    if (rc) return rc;
    wo_state s;
    rc = st_init(&s, V, n, m, p);
    if (rc) return rc;
    forward_all(&s);
    for (int i = 0; i < 2 * n; ++i)
        for (int j = 0; j < 2 * m; ++j) U[(size_t)i * (size_t)(2 * m) + (size_t)j] = AT(s.F, i, j);
    st_free(&s);
    return WO_OK;
}

/* Nonlinear weights omega_k at every output point (4 per point, zero at the
 * originals), 2n x 2m x 4 row-major.  For property tests. */
int weno_oracle_weights(const double* V, int n, int m, const weno_oracle_params* p, double* W)
{
    int rc = check_args(V, n, m, p, W);
    if (rc) return rc;
    wo_state s;
    rc = st_init(&s, V, n, m, p);
    if (rc) return rc;
    forward_all(&s);
    for (int i = 0; i < 2 * n; ++i) {
        for (int j = 0; j < 2 * m; ++j) {
            double* w = W + ((size_t)i * (size_t)(2 * m) + (size_t)j) * 4;
            if (!is_odd(i) && !is_odd(j)) {
                w[0] = w[1] = w[2] = w[3] = 0.0;
                continue;
            }
            double a[4], asum = 0.0;
            for (int k = 0; k < 4; ++k) {
                a[k] = 0.5 / pow(AT(s.T[k], i, j), s.beta);
                asum += a[k];
            }
            for (int k = 0; k < 4; ++k) w[k] = a[k] / asum;
        }
    }
    st_free(&s);
    return WO_OK;
}

/* ---------------------------------------------------------------------------
 * Hand adjoint.  Given G = dL/dU (2n x 2m), returns gV = dL/dV (n x m).
 * At a point with candidates p_k and t_k = eps + D_k:
 *   du/dp_k = omega_k,   du/dt_k = -beta omega_k (p_k - u) / t_k,
 * t_k depends on its own SI_k with weight 1 and on the four neighbour SI_k
 * with the neighbour weight; each SI_k and p_k depends on its stencil triple.
 * Phase 2 is reversed first (it feeds gradients into the x points and the
 * originals), then phase 1, then padded reads are folded onto the clamped
 * source pixels.  Plain serial scatter.
 * ------------------------------------------------------------------------- */
static void adjoint_pass(wo_state* s, fgrid* gF, fgrid gS[4], int phase, int lo, int hi_i, int hi_j,
                         int slo, int shi_i, int shi_j)
{
    const int (*dir)[2] = phase == 1 ? DIAG : AXIS;
    const int (*nb)[2] = phase == 1 ? NB1 : NB2;
    double step = phase == 1 ? s->step1 : s->step2;
    double scale = phase == 1 ? s->scale1 : s->scale2;
    for (int k = 0; k < 4; ++k) memset(gS[k].a, 0, sizeof(double) * (size_t)gS[k].rows * (size_t)gS[k].cols);
    fgrid gP[4];
    for (int k = 0; k < 4; ++k) fg_alloc(&gP[k], s->n, s->m);

    /* blend points: seeds for the candidates and the indicators */
    for (int i = lo; i < hi_i; ++i) {
        for (int j = lo; j < hi_j; ++j) {
            if (!in_class(phase, i, j)) continue;
            double g = AT(*gF, i, j);
            if (g == 0.0) continue;
            double a[4], asum = 0.0;
            for (int k = 0; k < 4; ++k) {
                a[k] = 0.5 / pow(AT(s->T[k], i, j), s->beta);
                asum += a[k];
            }
            double u = AT(s->F, i, j);
            for (int k = 0; k < 4; ++k) {
                double w = a[k] / asum;
                double pk = AT(s->P[k], i, j);
                /* with beta = 0 the weights 0.5 / t^0 do not depend on t
                 * (eq. alpha), so the term vanishes, also where t = 0 */
                double gt = s->beta == 0.0 ? 0.0 : -s->beta * g * w * (pk - u) / AT(s->T[k], i, j);
                AT(gP[k], i, j) += g * w;
                AT(gS[k], i, j) += gt;
                for (int q = 0; q < 4; ++q) AT(gS[k], i + nb[q][0], j + nb[q][1]) += s->nbw * gt;
            }
        }
    }
    /* stencil points: candidate and indicator gradients onto the triples */
    for (int i = slo; i < shi_i; ++i) {
        for (int j = slo; j < shi_j; ++j) {
            if (!in_class(phase, i, j)) continue;
            for (int k = 0; k < 4; ++k) {
                double gp = AT(gP[k], i, j), gs = AT(gS[k], i, j);
                if (gp == 0.0 && gs == 0.0) continue;
                int si = dir[k][0], sj = dir[k][1];
                double va = AT(s->F, i - si, j - sj);
                double vb = AT(s->F, i + si, j + sj);
                double vc = AT(s->F, i + 3 * si, j + 3 * sj);
                double cg[3], sg[3];
                candidate_grad(cg);
                indicator_grad(va, vb, vc, step, scale, sg);
                AT(*gF, i - si, j - sj) += gp * cg[0] + gs * sg[0];
                AT(*gF, i + si, j + sj) += gp * cg[1] + gs * sg[1];
                AT(*gF, i + 3 * si, j + 3 * sj) += gp * cg[2] + gs * sg[2];
            }
        }
    }
    for (int k = 0; k < 4; ++k) fg_free(&gP[k]);
}

int weno_oracle_backward(const double* V, int n, int m, const weno_oracle_params* p, const double* G,
                         double* gV)
{
    int rc = check_args(V, n, m, p, gV);
    if (rc) return rc;
    if (!G) return WO_EINVAL;
    wo_state s;
    rc = st_init(&s, V, n, m, p);
    if (rc) return rc;
    int n2 = 2 * n, m2 = 2 * m;
    /* forward, keeping phase-1 fields separately since phase 2 reuses P/S/T */
    stencil_pass(&s, 1, -9, n2 + 9, m2 + 9);
    blend_pass(&s, 1, -7, n2 + 7, m2 + 7);
    fgrid P1[4], T1[4];
    int bad = 0;
    for (int k = 0; k < 4; ++k) {
        bad |= fg_alloc(&P1[k], n, m);
        bad |= fg_alloc(&T1[k], n, m);
    }
    fgrid gF, gS[4];
    bad |= fg_alloc(&gF, n, m);
    for (int k = 0; k < 4; ++k) bad |= fg_alloc(&gS[k], n, m);
    if (bad) {
        for (int k = 0; k < 4; ++k) { fg_free(&P1[k]); fg_free(&T1[k]); fg_free(&gS[k]); }
        fg_free(&gF);
        st_free(&s);
        return WO_ENOMEM;
    }
    size_t bytes = sizeof(double) * (size_t)s.F.rows * (size_t)s.F.cols;
    for (int k = 0; k < 4; ++k) {
        memcpy(P1[k].a, s.P[k].a, bytes);
        memcpy(T1[k].a, s.T[k].a, bytes);
    }
    stencil_pass(&s, 2, -4, n2 + 4, m2 + 4);
    blend_pass(&s, 2, -3, n2 + 3, m2 + 3);

    /* output gradient on the 2n x 2m grid, zero in the margin */
    for (int i = 0; i < n2; ++i)
        for (int j = 0; j < m2; ++j) AT(gF, i, j) = G[(size_t)i * (size_t)m2 + (size_t)j];

    /* reverse phase 2 */
    adjoint_pass(&s, &gF, gS, 2, -3, n2 + 3, m2 + 3, -4, n2 + 4, m2 + 4);
    /* reverse phase 1 with its own candidate / weight fields */
    for (int k = 0; k < 4; ++k) {
        memcpy(s.P[k].a, P1[k].a, bytes);
        memcpy(s.T[k].a, T1[k].a, bytes);
    }
    adjoint_pass(&s, &gF, gS, 1, -7, n2 + 7, m2 + 7, -9, n2 + 9, m2 + 9);

    /* fold the gradients of padded (clamped) reads onto the source pixels */
    memset(gV, 0, sizeof(double) * (size_t)n * (size_t)m);
    for (int i = -FM; i < n2 + FM; ++i) {
        if (is_odd(i)) continue;
        for (int j = -FM; j < m2 + FM; ++j) {
            if (is_odd(j)) continue;
            int I = clampi(i / 2, 0, n - 1);
            int J = clampi(j / 2, 0, m - 1);
            gV[(size_t)I * (size_t)m + (size_t)J] += AT(gF, i, j);
        }
    }
    for (int k = 0; k < 4; ++k) { fg_free(&P1[k]); fg_free(&T1[k]); fg_free(&gS[k]); }
    fg_free(&gF);
    st_free(&s);
    return WO_OK;
}

/* The hand adjoint of `planes` independent planes, one plane per OpenMP
 * thread (V: planes x n x m, G: planes x 2n x 2m, gV: planes x n x m, all
 * row-major).  Each plane is weno_oracle_backward, unchanged. */
int weno_oracle_backward_planes(const double* V, int planes, int n, int m, const weno_oracle_params* p,
                                const double* G, double* gV)
{
    if (planes < 1) return WO_EINVAL;
    int rc = WO_OK;
    #pragma omp parallel for schedule(dynamic, 1)
    for (int c = 0; c < planes; ++c) {
        const size_t in = (size_t)n * (size_t)m;
        int r = weno_oracle_backward(V + (size_t)c * in, n, m, p, G + (size_t)c * 4 * in, gV + (size_t)c * in);
        if (r) {
            #pragma omp critical
            rc = r;
        }
    }
    return rc;
}
