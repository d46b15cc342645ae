/*
 * pwrel oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, single-threaded FP64 CPU implementation of the perceptron
 * point-wise-relative (PW_REL) compressor of Chen & Li, "Significant
 * improvement of lossy compression rate and speed of HPC data using
 * perceptron parallelized compression" (arXiv 2309.09778).  Only the test
 * suite, the package smoke check and the benchmark's CPU-baseline leg may
 * load this library.  It shares no source with the HIP library: every
 * routine here (including the deterministic log2/exp2 and the splitmix64
 * hash) is written independently from its published definition.
 *
 * Build: gcc -O2 -std=c11 -ffp-contract=off -fno-fast-math -fPIC -shared.
 * Contraction must stay off: every a*b+c below is two roundings unless it
 * is written as an explicit fma()/fmaf().
 *
 * Section map (paper):
 *   stats, factors, bound ........ Sec. 3.2, Eq. 8-11 and Algorithm 1 (first three steps)
 *   log-domain transform ......... Sec. 3.2, Eq. 6, 7, 12; Algorithm 1 (transform branch)
 *   inverse + zero/sign rule ..... Sec. 3.2, text after Eq. 12
 *   Lorenzo predictor ............ Sec. 4.1 (one-layer Lorenzo formula)
 *   three-layer perceptron ....... Sec. 4.2 and Fig. 3 (init rule: end of Sec. 4.2)
 *   data selection rule .......... Sec. 4.4.1 and 4.4.2 (predict from actual values)
 *   quantizer / balance points ... Sec. 4.3 (codes 0..2^m-1), Sec. 4.4.1(b), Algorithm 1
 *   decompression ................ Sec. 5 (decompression paragraph)
 *   training ..................... Sec. 4.3 (10% uniform sample, 8:2 split, L2,
 *                                  one round, several lr/lambda sets, pick best)
 *   Huffman stage ................ Sec. 4.1 coding stage, Algorithm 1, Sec. 5
 *   trained codebook ............. Sec. 4.3 (code frequencies of validation blocks)
 *
 * Readings where the paper is silent or inconsistent (each is listed in the
 * design notes of the repository):
 *   - factor_pos is the smallest non-zero |x| (Eq. 9), not |min x|.
 *   - "actual values" on the prediction surface are the neighbours' values
 *     snapped to the 2*b_a quantization grid (integer grid value p); the
 *     decoder reproduces p exactly, so the bound holds on every point.
 *   - log/exp are the deterministic series below (det_log2 / det_exp2).
 *   - eps0 = min(smallest normal of the dtype, abs_min/2); zero decodes iff
 *     p <= p_zero.
 *   - an integer offset delta >= 0 keeps every negative strictly above the
 *     positive ceiling (a constant factor 2^(delta*w) on factor_neg, allowed
 *     by the constant-factor lemma of Sec. 3.1).
 *   - the network predicts the difference to the previous point along the
 *     fastest axis from the other neighbours' differences, Lorenzo at init.
 *   - m = 16: codes 1..65535, code 0 = balance point (raw input value kept).
 *   - the trained codebook gives codes unseen in validation an escape
 *     codeword plus their 16 bits (the paper does not say what happens to
 *     them).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_EINVAL (-1)
#define OR_ERANGE (-2)
#define OR_ENONFINITE (-3)
#define OR_ENOMEM (-7)

#define OR_F32 0
#define OR_F64 1

#define OR_R 32768     /* 2^(m-1), m = 16 */
#define OR_MAXH 32
#define OR_MAXK 6
#define OR_PLIM 1073741824.0 /* |t| must stay below 2^30 */

/* ------------------------------------------------------------------------ */
/* Deterministic log2 / exp2 in FP64 (only +,-,*,/, fma, rint, ldexp, bits). */
/* ------------------------------------------------------------------------ */

/* log2(x), x > 0 finite.  x = m * 2^e with m in (sqrt2/2, sqrt2];
 * ln m = 2 atanh(s), s = (m-1)/(m+1), summed as 2 s sum_k s^(2k)/(2k+1). */
double or_det_log2(double x)
{
    static const double c[11] = {
        1.0, 1.0 / 3.0, 1.0 / 5.0, 1.0 / 7.0, 1.0 / 9.0, 1.0 / 11.0,
        1.0 / 13.0, 1.0 / 15.0, 1.0 / 17.0, 1.0 / 19.0, 1.0 / 21.0};
    int eadj = 0;
    if (x < 0x1p-1022) { /* subnormal input: scale into the normal range */
        x = x * 0x1p54;
        eadj = -54;
    }
    uint64_t bits;
    memcpy(&bits, &x, sizeof bits);
    int e = (int)((bits >> 52) & 0x7ff) - 1023;
    bits = (bits & 0x000fffffffffffffULL) | 0x3ff0000000000000ULL;
    double m;
    memcpy(&m, &bits, sizeof m);
    if (m > 1.4142135623730951) {
        m = m * 0.5;
        e = e + 1;
    }
    double s = (m - 1.0) / (m + 1.0);
    double z = s * s;
    double P = c[10];
    for (int k = 9; k >= 0; --k)
        P = fma(P, z, c[k]);
    return (double)(e + eadj) + ((s + s) * P) * 1.4426950408889634;
}

/* 2^t, t finite with |t| < 2^31.  2^t = 2^k e^a, k = rint(t),
 * a = (t-k) ln 2, e^a by its Taylor series to degree 13. */
double or_det_exp2(double t)
{
    static const double d[14] = {
        1.0, 1.0, 1.0 / 2.0, 1.0 / 6.0, 1.0 / 24.0, 1.0 / 120.0, 1.0 / 720.0,
        1.0 / 5040.0, 1.0 / 40320.0, 1.0 / 362880.0, 1.0 / 3628800.0,
        1.0 / 39916800.0, 1.0 / 479001600.0, 1.0 / 6227020800.0};
    double k = rint(t);
    double f = t - k;
    double a = f * 0.6931471805599453;
    double P = d[13];
    for (int j = 12; j >= 0; --j)
        P = fma(P, a, d[j]);
    return ldexp(P, (int)k);
}

/* ------------------------------------------------------------------------ */
/* splitmix64 (Steele, Lea, Flood 2014; Vigna's reference constants), used as */
/* a counter-based hash: h(i) = splitmix64_next with state seed ^ i.         */
/* ------------------------------------------------------------------------ */
uint64_t or_splitmix64(uint64_t state)
{
    uint64_t z = state + 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* uniform in [0,1) from the top 53 bits */
static double u01(uint64_t h) { return (double)(h >> 11) * 0x1p-53; }

/* ------------------------------------------------------------------------ */
/* Statistics and constants (Sec. 3.2, Eq. 8-12; Algorithm 1 first steps)    */
/* ------------------------------------------------------------------------ */
typedef struct {
    double abs_min;   /* smallest non-zero |x| (1 if none) */
    double abs_max;   /* largest |x| (1 if no non-zero) */
    uint64_t n;
    uint64_t n_zero;
    uint64_t n_neg;
    uint64_t n_nonfinite;
} or_stats;

typedef struct {
    double eps;   /* point-wise relative bound b_r */
    double eps0;  /* zero stand-in */
    double b_a;   /* absolute bound in the log2 domain, Eq. 8 */
    double w;     /* grid step 2 b_a */
    double r;     /* 1 / w */
    double Lp;    /* log2 factor_pos, Eq. 9 */
    double Ln;    /* log2 factor_neg, Eq. 10/11 */
    double d0;    /* log-domain image of zero, Eq. 12 */
    int64_t p_zero; /* grid value of zero; p <= p_zero decodes to 0 */
    int64_t b_sign; /* positive ceiling: largest grid value of a positive */
    int64_t n_lo;   /* grid value of the smallest-magnitude negative (before delta) */
    int64_t delta;  /* integer offset added to every negative's grid value */
} or_consts;

static double load_val(const void *x, int dtype, uint64_t i)
{
    if (dtype == OR_F32)
        return (double)((const float *)x)[i];
    return ((const double *)x)[i];
}

static void store_val(void *x, int dtype, uint64_t i, double v)
{
    if (dtype == OR_F32)
        ((float *)x)[i] = (float)v;
    else
        ((double *)x)[i] = v;
}

static double cast_t(double v, int dtype)
{
    if (dtype == OR_F32)
        return (double)(float)v;
    return v;
}

int or_stats_compute(const void *x, uint64_t n, int dtype, or_stats *st)
{
    if (dtype != OR_F32 && dtype != OR_F64)
        return OR_EINVAL;
    double amin = INFINITY, amax = 0.0;
    uint64_t nz = 0, nn = 0, nf = 0;
    for (uint64_t i = 0; i < n; ++i) {
        double v = load_val(x, dtype, i);
        if (!isfinite(v)) {
            nf++;
            continue;
        }
        double a = fabs(v);
        if (v == 0.0) {
            nz++;
            continue;
        }
        if (v < 0.0)
            nn++;
        if (a < amin)
            amin = a;
        if (a > amax)
            amax = a;
    }
    if (nz + nf == n) { /* no finite non-zero value */
        amin = 1.0;
        amax = 1.0;
    }
    st->abs_min = amin;
    st->abs_max = amax;
    st->n = n;
    st->n_zero = nz;
    st->n_neg = nn;
    st->n_nonfinite = nf;
    return nf ? OR_ENONFINITE : OR_OK;
}

static int fits(double t) { return fabs(t) < OR_PLIM; }

int or_consts_compute(const or_stats *st, int dtype, double eps, or_consts *c)
{
    if (!(eps > 0.0 && eps < 1.0))
        return OR_EINVAL;
    double tau = (dtype == OR_F32) ? 0x1p-126 : 0x1p-1022;
    double eps0 = st->abs_min * 0.5;
    if (tau < eps0)
        eps0 = tau;
    if (!(eps0 > 0.0))
        return OR_ERANGE; /* abs_min is the smallest subnormal: no room below it */
    double one_eps = 1.0 + eps;
    if (!(one_eps > 1.0))
        return OR_EINVAL;
    c->eps = eps;
    c->eps0 = eps0;
    c->b_a = or_det_log2(one_eps);
    c->w = c->b_a + c->b_a;
    c->r = 1.0 / c->w;
    c->Lp = or_det_log2(st->abs_min);
    c->Ln = ((or_det_log2(st->abs_max + eps0) + c->Lp) + c->w) - or_det_log2(st->abs_min - eps0);
    c->d0 = or_det_log2(eps0) + c->Lp;
    double tz = c->d0 * c->r;
    double tb = (or_det_log2(st->abs_max) + c->Lp) * c->r;
    double tn = (or_det_log2(st->abs_min) + c->Ln) * c->r;
    if (!fits(tz) || !fits(tb) || !fits(tn))
        return OR_ERANGE;
    c->p_zero = (int64_t)rint(tz);
    c->b_sign = (int64_t)rint(tb);
    c->n_lo = (int64_t)rint(tn);
    c->delta = c->b_sign + 1 - c->n_lo;
    if (c->delta < 0)
        c->delta = 0;
    return OR_OK;
}

/* Grid value of one input value (Eq. 6, 7, 12 with the clamps that keep the
 * three ranges zero < positive < negative disjoint). */
static int32_t transform_pt(double x, const or_consts *c, int *status)
{
    if (x == 0.0)
        return (int32_t)c->p_zero;
    if (x > 0.0) {
        double t = (or_det_log2(x) + c->Lp) * c->r;
        if (!fits(t)) {
            *status = OR_ERANGE;
            return 0;
        }
        int64_t q = (int64_t)rint(t);
        if (q < c->p_zero + 1)
            q = c->p_zero + 1;
        if (q > c->b_sign)
            q = c->b_sign;
        return (int32_t)q;
    }
    double t = (or_det_log2(-x) + c->Ln) * c->r;
    if (!fits(t)) {
        *status = OR_ERANGE;
        return 0;
    }
    int64_t q = (int64_t)rint(t) + c->delta;
    if (q < c->b_sign + 1)
        q = c->b_sign + 1;
    if (!(fabs((double)q) < OR_PLIM)) {
        *status = OR_ERANGE;
        return 0;
    }
    return (int32_t)q;
}

/* Inverse map of a grid value, rounded to the input dtype. */
static double inverse_pt(int32_t p, const or_consts *c, int dtype)
{
    double v;
    if ((int64_t)p <= c->p_zero)
        v = 0.0;
    else if ((int64_t)p <= c->b_sign)
        v = or_det_exp2((double)p * c->w - c->Lp);
    else
        v = -or_det_exp2((double)((int64_t)p - c->delta) * c->w - c->Ln);
    return cast_t(v, dtype);
}

/* The PW_REL bound with sign and zero preserved, evaluated in FP64. */
static int verify_pt(double x, double xh, double eps)
{
    if (x == 0.0)
        return xh == 0.0;
    if (xh == 0.0)
        return 0;
    if (signbit(x) != signbit(xh))
        return 0;
    return fabs(x - xh) <= eps * fabs(x);
}

int32_t or_transform(double x, const or_consts *c, int *status) { return transform_pt(x, c, status); }
double or_inverse(int32_t p, const or_consts *c, int dtype) { return inverse_pt(p, c, dtype); }
int or_verify(double x, double xh, double eps) { return verify_pt(x, xh, eps); }

int or_transform_field(const void *x, uint64_t n, int dtype, const or_consts *c, int32_t *p)
{
    int status = OR_OK;
    for (uint64_t i = 0; i < n; ++i) {
        p[i] = transform_pt(load_val(x, dtype, i), c, &status);
        if (status != OR_OK)
            return status;
    }
    return OR_OK;
}

int or_inverse_field(const int32_t *p, uint64_t n, int dtype, const or_consts *c, void *xh)
{
    for (uint64_t i = 0; i < n; ++i)
        store_val(xh, dtype, i, inverse_pt(p[i], c, dtype));
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Perceptron (Sec. 4.2).  FP32, explicit fmaf, this exact order.            */
/* ------------------------------------------------------------------------ */
typedef struct {
    int32_t hidden;          /* H */
    int32_t inputs;          /* K = 2^D - 2 */
    float alpha;             /* leaky-ReLU slope */
    float w1[OR_MAXH][OR_MAXK];
    float b1[OR_MAXH];
    float v[OR_MAXH];
    float b2;
    int32_t precision;       /* 0 = FP32 evaluation, 1 = BF16 operands (reference only) */
} or_mlp;

static float lrelu_f(float z, float alpha) { return (z < 0.0f) ? z * alpha : z; }

/* FP32 network value y(u) with u_k = float(n_{k+2} - n_1). */
static float mlp_eval_f32(const or_mlp *m, const float *u)
{
    float h[OR_MAXH];
    for (int j = 0; j < m->hidden; ++j) {
        float z = m->b1[j];
        for (int k = 0; k < m->inputs; ++k)
            z = fmaf(m->w1[j][k], u[k], z);
        h[j] = lrelu_f(z, m->alpha);
    }
    float y = m->b2;
    for (int j = 0; j < m->hidden; ++j)
        y = fmaf(m->v[j], h[j], y);
    return y;
}

/* round-to-nearest-even to bfloat16, returned as float */
static float bf16_rne(float f)
{
    uint32_t u;
    memcpy(&u, &f, 4);
    uint32_t lsb = (u >> 16) & 1u;
    u = (u + 0x7fffu + lsb) & 0xffff0000u;
    float g;
    memcpy(&g, &u, 4);
    return g;
}

/* Reference value of the BF16-operand network, in FP64, with the leaky ReLU
 * written as lrelu(z) = (1 - alpha) relu(z) + alpha z:
 *   z_j  = b1_j + sum_k bf16(w1_jk) bf16(u_k)
 *   y    = b2 + sum_j bf16((1 - alpha) v_j) relu(bf16(z_j)) + bf16(alpha v_j) bf16(z_j)
 * ((1 - alpha) and the products with v_j in FP32 before the bf16 rounding).
 * The matrix-core path accumulates in FP32 in the hardware's order: its z_j
 * lies within d_j = Z_j 2^-19 of the exact one (Z_j = |b1_j| + sum |products|,
 * a generous bound for at most 8 FP32 roundings), so its bf16(z_j) lies
 * between bf16(z_j - d_j) and bf16(z_j + d_j) (rounding is monotone).
 * *slack bounds |y_device - y|: (|a_j| + |c_j|) times the largest such move
 * of bf16(z_j), summed over hidden units, plus 2^-18 times the sum of the
 * magnitudes of layer 2 (its FP32 accumulation). */
static double mlp_eval_bf16_ref(const or_mlp *m, const float *u, double *slack)
{
    const float ar = 1.0f - m->alpha, al = m->alpha;
    double y = (double)m->b2, sl = 0.0, mag = fabs((double)m->b2);
    for (int j = 0; j < m->hidden; ++j) {
        double z = (double)m->b1[j], za = fabs(z);
        for (int k = 0; k < m->inputs; ++k) {
            double t = (double)bf16_rne(m->w1[j][k]) * (double)bf16_rne(u[k]);
            z += t;
            za += fabs(t);
        }
        double zb = (double)bf16_rne((float)z);
        double a = (double)bf16_rne(ar * m->v[j]);
        double c = (double)bf16_rne(al * m->v[j]);
        double t1 = a * (zb > 0.0 ? zb : 0.0), t2 = c * zb;
        y += t1 + t2;
        mag += fabs(t1) + fabs(t2);
        double d = za * 0x1p-19;
        double zlo = (double)bf16_rne((float)(z - d)), zhi = (double)bf16_rne((float)(z + d));
        double dz = fabs(zlo - zb) > fabs(zhi - zb) ? fabs(zlo - zb) : fabs(zhi - zb);
        sl += (fabs(a) + fabs(c)) * dz;
    }
    *slack = sl + mag * 0x1p-18;
    return y;
}

/* The network evaluated in FP64 from its FP32 weights (the value every
 * finite-precision evaluation approximates); u as given (FP32 values). */
static double mlp_eval_f64(const or_mlp *m, const float *u)
{
    const double a = (double)m->alpha;
    double y = (double)m->b2;
    for (int j = 0; j < m->hidden; ++j) {
        double z = (double)m->b1[j];
        for (int k = 0; k < m->inputs; ++k)
            z += (double)m->w1[j][k] * (double)u[k];
        y += (double)m->v[j] * (z < 0.0 ? a * z : z);
    }
    return y;
}

/* Error bound of BF16-operand inference against mlp_eval_f64.  It covers any
 * evaluation in which
 *   (i)  every first-layer weight and every input is rounded once to bfloat16
 *        (8 significant bits: relative error <= U = 2^-8), the products (exact
 *        in FP32) and b1 summed in FP32 in any order;
 *   (ii) every hidden pre-activation is rounded once to bfloat16 before the
 *        leaky ReLU;
 *   (iii) every output weight enters as bfloat16 numbers within relative
 *        U + 2^-22 of (1 - alpha) v and alpha v (the two parts of the leaky
 *        ReLU, v lrelu(z) = (1 - alpha) v relu(z) + alpha v z, possibly after
 *        FP32 scalings) or of v itself, and the 2H (or H) products plus b2 are
 *        summed in FP32 in any order.
 * With S_j = sum_k |w_jk u_k|, Z_j = |z_j|, g_n = n 2^-24 / (1 - n 2^-24):
 *   first layer:  d_j = (2U + U^2) S_j + g_K (|b1_j| + (1 + U)^2 S_j)
 *   rounding z:   D_j = d_j + U (Z_j + d_j)           (|z^_j - z_j| <= D_j)
 *   unit j:       E_j = |v_j| D_j + (U + 2^-22) |v_j| (Z_j + D_j)
 *                 (lrelu is 1-Lipschitz and |lrelu(z)| <= |z|)
 *   second layer: g_{2H} (|b2| + (1 + U + 2^-22) sum_j |v_j| (Z_j + D_j))
 * The bound is the sum of the E_j and the second-layer term, plus 2^-50 of
 * the magnitudes for the FP64 reference's own rounding. */
static double mlp_bf16_bound(const or_mlp *m, const float *u)
{
    const double U = 0x1p-8, Uw = 0x1p-8 + 0x1p-22;
    const int K = m->inputs, H = m->hidden;
    const double gK = K * 0x1p-24 / (1.0 - K * 0x1p-24);
    const double g2H = 2 * H * 0x1p-24 / (1.0 - 2 * H * 0x1p-24);
    double sum_e = 0.0, mag2 = fabs((double)m->b2), magall = fabs((double)m->b2);
    for (int j = 0; j < H; ++j) {
        double z = (double)m->b1[j], S = 0.0;
        for (int k = 0; k < K; ++k) {
            const double t = (double)m->w1[j][k] * (double)u[k];
            z += t;
            S += fabs(t);
        }
        const double Z = fabs(z), av = fabs((double)m->v[j]);
        const double d = (2.0 * U + U * U) * S + gK * (fabs((double)m->b1[j]) + (1.0 + U) * (1.0 + U) * S);
        const double D = d + U * (Z + d);
        sum_e += av * D + Uw * av * (Z + D);
        mag2 += (1.0 + Uw) * av * (Z + D);
        magall += av * Z + fabs((double)m->b1[j]) + S;
    }
    return sum_e + g2H * mag2 + 0x1p-50 * magall;
}

/* ------------------------------------------------------------------------ */
/* Geometry: C-order dims n[0..D-1] (axis D-1 fastest), blocks of edge B     */
/* clipped at the high faces, blocks in raster order, points in local raster */
/* order inside each block.                                                  */
/* ------------------------------------------------------------------------ */
typedef struct {
    int D;
    int64_t n[3];
    int64_t nb[3];
    int64_t B;
    int64_t N;
    int64_t nblocks;
} geom;

static int geom_init(geom *g, const uint64_t *dims, int ndim, int B)
{
    if (ndim < 1 || ndim > 3 || B < 2 || B > 4096)
        return OR_EINVAL;
    int64_t bd = 1;
    for (int d = 0; d < ndim; ++d)
        bd *= B;
    if (bd > (1 << 20))
        return OR_EINVAL;
    g->D = ndim;
    g->B = B;
    g->N = 1;
    g->nblocks = 1;
    for (int d = 0; d < ndim; ++d) {
        if (dims[d] < 1)
            return OR_EINVAL;
        g->n[d] = (int64_t)dims[d];
        g->nb[d] = (g->n[d] + B - 1) / B;
        g->N *= g->n[d];
        g->nblocks *= g->nb[d];
    }
    return OR_OK;
}

static int64_t lin(const geom *g, const int64_t *c)
{
    int64_t i = 0;
    for (int d = 0; d < g->D; ++d)
        i = i * g->n[d] + c[d];
    return i;
}

/* extent of block b along axis d */
static int64_t bext(const geom *g, int d, int64_t b)
{
    int64_t s = g->n[d] - b * g->B;
    return s < g->B ? s : g->B;
}

/* stream position of the first point of block (bc[0..D-1]) */
static int64_t block_start(const geom *g, const int64_t *bc)
{
    int64_t off = 0, scale = 1;
    for (int d = 0; d < g->D; ++d) {
        int64_t rest = 1;
        for (int e = d + 1; e < g->D; ++e)
            rest *= g->n[e];
        off += scale * bc[d] * g->B * rest;
        scale *= bext(g, d, bc[d]);
    }
    return off;
}

/* Neighbour with offset o (bit i of o steps back along axis D-1-i). */
static int neighbour(const geom *g, const int64_t *c, int o, int independent, int64_t *out)
{
    for (int d = 0; d < g->D; ++d) {
        int bit = (o >> (g->D - 1 - d)) & 1;
        int64_t q = c[d] - bit;
        if (q < 0)
            return 0;
        if (independent && (q / g->B) != (c[d] / g->B))
            return 0;
        out[d] = q;
    }
    return 1;
}

/* Lorenzo coefficient (-1)^(|o|+1) of the one-layer Lorenzo predictor */
static int lorenzo_coef(int o)
{
    int pc = __builtin_popcount((unsigned)o);
    return (pc & 1) ? 1 : -1;
}

/* Prediction of point c from grid values P (Sec. 4.1, 4.2, 4.4.1).
 * mode: 0 = Lorenzo only, 1 = network where all neighbours exist (FP32),
 *       2 = BF16 reference value (returns through yref / slack).           */
typedef struct {
    int use_net;
    int64_t pred;
    double yref, slack; /* BF16 reference only */
    int net_used;
} pred_out;

static void predict_pt(const geom *g, const int32_t *P, const int64_t *c, int independent,
                       const or_mlp *m, int use_net, pred_out *po)
{
    int no = (1 << g->D) - 1;
    int64_t nv[8];
    int avail = 0, all = 1;
    for (int o = 1; o <= no; ++o) {
        int64_t q[3];
        if (neighbour(g, c, o, independent, q)) {
            nv[o] = P[lin(g, q)];
            avail |= 1 << o;
        } else {
            nv[o] = 0;
            all = 0;
        }
    }
    po->net_used = 0;
    if (use_net && m && all) {
        float u[OR_MAXK];
        for (int k = 0; k < m->inputs; ++k)
            u[k] = (float)(int32_t)(nv[k + 2] - nv[1]);
        if (m->precision == 1) {
            double sl;
            po->yref = mlp_eval_bf16_ref(m, u, &sl);
            po->slack = sl;
        }
        float y = mlp_eval_f32(m, u);
        if (y > 0x1p30f)
            y = 0x1p30f;
        if (!(y >= -0x1p30f))
            y = -0x1p30f;
        po->pred = nv[1] + (int64_t)rintf(y);
        po->net_used = 1;
        return;
    }
    int64_t s = 0;
    for (int o = 1; o <= no; ++o)
        if (avail & (1 << o))
            s += lorenzo_coef(o) * nv[o];
    po->pred = s;
}

static uint16_t code_of(int64_t pred, int64_t p, int ok)
{
    int64_t e = pred - p; /* prediction minus actual (Algorithm 1) */
    if (ok && e > -OR_R && e < OR_R)
        return (uint16_t)(e + OR_R);
    return 0;
}

/* iterate blocks in raster order, points in local raster order */
typedef struct {
    const geom *g;
    int64_t bc[3], lc[3], ext[3], c[3];
    int64_t block;
    int64_t pos;
    int done;
} iter;

static void it_begin_block(iter *it)
{
    for (int d = 0; d < it->g->D; ++d) {
        it->ext[d] = bext(it->g, d, it->bc[d]);
        it->lc[d] = 0;
        it->c[d] = it->bc[d] * it->g->B;
    }
}

static void it_init(iter *it, const geom *g)
{
    it->g = g;
    for (int d = 0; d < 3; ++d)
        it->bc[d] = it->lc[d] = 0;
    it->block = 0;
    it->pos = 0;
    it->done = (g->N == 0);
    it_begin_block(it);
}

/* returns 1 when a new block starts */
static int it_next(iter *it)
{
    const geom *g = it->g;
    it->pos++;
    for (int d = g->D - 1; d >= 0; --d) {
        if (++it->lc[d] < it->ext[d]) {
            it->c[d] = it->bc[d] * g->B + it->lc[d];
            return 0;
        }
        it->lc[d] = 0;
        it->c[d] = it->bc[d] * g->B;
    }
    it->block++;
    for (int d = g->D - 1; d >= 0; --d) {
        if (++it->bc[d] < g->nb[d]) {
            it_begin_block(it);
            return 1;
        }
        it->bc[d] = 0;
    }
    it->done = 1;
    return 1;
}

/* ------------------------------------------------------------------------ */
/* Per-block judge (learned path): empirical code entropy in fixed point.    */
/* J = sum_s c_s * q(c_s), q(c) = rint(log2(c) * 2^32); H = n q(n) - J.      */
/* ------------------------------------------------------------------------ */
static int64_t qlog(int64_t c) { return (int64_t)rint(or_det_log2((double)c) * 4294967296.0); }

static int cmp_u16(const void *a, const void *b)
{
    uint16_t x = *(const uint16_t *)a, y = *(const uint16_t *)b;
    return (x > y) - (x < y);
}

/* J of a multiset of codes (sorted copy) */
static int64_t entropy_j(uint16_t *tmp, int64_t n)
{
    qsort(tmp, (size_t)n, sizeof(uint16_t), cmp_u16);
    int64_t J = 0;
    int64_t i = 0;
    while (i < n) {
        int64_t j = i;
        while (j < n && tmp[j] == tmp[i])
            j++;
        int64_t cnt = j - i;
        J += cnt * qlog(cnt);
        i = j;
    }
    return J;
}

/* Per-block judge score: J of the block's codes taken as they are, every
 * distinct code (code 0, the balance point, included) one symbol of the
 * multiset, so that n q(n) - J is 2^32 times the block's empirical code
 * entropy in bits (Sec. 4.3 picks the predictor whose codes are cheapest to
 * entropy-code).  The caller's codes are left in their order. */
static int64_t judge_j(const uint16_t *codes, int64_t n)
{
    uint16_t *tmp = (uint16_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(uint16_t));
    if (!tmp)
        return INT64_MIN;
    memcpy(tmp, codes, (size_t)n * sizeof(uint16_t));
    int64_t J = entropy_j(tmp, n);
    free(tmp);
    return J;
}

int64_t or_judge_j(const uint16_t *codes, int64_t n) { return judge_j(codes, n); }

int64_t or_entropy_j(const uint16_t *codes, int64_t n)
{
    uint16_t *tmp = (uint16_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(uint16_t));
    if (!tmp)
        return -1;
    memcpy(tmp, codes, (size_t)n * sizeof(uint16_t));
    int64_t J = entropy_j(tmp, n);
    free(tmp);
    return J;
}

int64_t or_qlog(int64_t c) { return qlog(c); }

/* ------------------------------------------------------------------------ */
/* Compression (Algorithm 1 with the readings above)                         */
/* ------------------------------------------------------------------------ */

/* Codes of a given grid field, every point taken as verified (p-level
 * entry used to pin the predictor in isolation). */
int or_encode_p(const int32_t *P, const uint64_t *dims, int ndim, int B, int independent,
                const or_mlp *m, int use_net, uint16_t *codes)
{
    geom g;
    int st = geom_init(&g, dims, ndim, B);
    if (st)
        return st;
    iter it;
    it_init(&it, &g);
    while (!it.done) {
        pred_out po;
        predict_pt(&g, P, it.c, independent, m, use_net, &po);
        codes[it.pos] = code_of(po.pred, P[lin(&g, it.c)], 1);
        it_next(&it);
    }
    return OR_OK;
}

/* Full compression.  Outputs (caller-allocated):
 *   codes[N] (block-major), counts[nblocks], raw (dtype, capacity N),
 *   n_raw, consts, flags[nblocks] (learned: 1 = network kept, else 0).
 * mode: 0 = Lorenzo only; 1 = plain (network at every eligible point);
 *       2 = learned (per-block judge network vs Lorenzo).
 * p_out (optional, N): the grid field. */
int or_compress(const void *x, const uint64_t *dims, int ndim, int dtype, double eps, int B,
                int independent, const or_mlp *m, int mode, uint16_t *codes, uint32_t *counts,
                void *raw, uint64_t *n_raw, or_consts *consts, uint8_t *flags, int32_t *p_out)
{
    geom g;
    int st = geom_init(&g, dims, ndim, B);
    if (st)
        return st;
    if (dtype != OR_F32 && dtype != OR_F64)
        return OR_EINVAL;
    if (mode != 0 && (!m || m->inputs != (1 << ndim) - 2 || m->hidden < 1 || m->hidden > OR_MAXH))
        return OR_EINVAL;
    or_stats sts;
    st = or_stats_compute(x, (uint64_t)g.N, dtype, &sts);
    if (st)
        return st;
    st = or_consts_compute(&sts, dtype, eps, consts);
    if (st)
        return st;
    int32_t *P = p_out ? p_out : (int32_t *)malloc((size_t)g.N * sizeof(int32_t));
    if (!P)
        return OR_ENOMEM;
    st = or_transform_field(x, (uint64_t)g.N, dtype, consts, P);
    if (st) {
        if (!p_out)
            free(P);
        return st;
    }
    int64_t bsz_max = 1;
    for (int d = 0; d < ndim; ++d)
        bsz_max *= g.B;
    uint16_t *cn = (uint16_t *)malloc((size_t)bsz_max * sizeof(uint16_t));
    uint16_t *cl = (uint16_t *)malloc((size_t)bsz_max * sizeof(uint16_t));
    uint8_t *okb = (uint8_t *)malloc((size_t)bsz_max);
    int64_t *idxb = (int64_t *)malloc((size_t)bsz_max * sizeof(int64_t));
    if (!cn || !cl || !okb || !idxb) {
        free(cn); free(cl); free(okb); free(idxb);
        if (!p_out)
            free(P);
        return OR_ENOMEM;
    }
    uint64_t nr = 0;
    iter it;
    it_init(&it, &g);
    while (!it.done) {
        /* one block: evaluate both predictors, judge, emit */
        int64_t b = it.block, start = it.pos, k = 0;
        do {
            int64_t i = lin(&g, it.c);
            double xv = load_val(x, dtype, (uint64_t)i);
            int ok = verify_pt(xv, inverse_pt(P[i], consts, dtype), eps);
            pred_out pn, pl;
            predict_pt(&g, P, it.c, independent, m, mode != 0, &pn);
            predict_pt(&g, P, it.c, independent, m, 0, &pl);
            cn[k] = code_of(pn.pred, P[i], ok);
            cl[k] = code_of(pl.pred, P[i], ok);
            okb[k] = (uint8_t)ok;
            idxb[k] = i;
            k++;
        } while (!it_next(&it));
        int use_net = (mode == 1);
        if (mode == 2)
            use_net = judge_j(cn, k) > judge_j(cl, k); /* network's entropy strictly lower */
        if (flags)
            flags[b] = (uint8_t)(mode == 2 ? use_net : (mode == 1));
        uint32_t cnt = 0;
        for (int64_t q = 0; q < k; ++q) {
            uint16_t cd = use_net ? cn[q] : cl[q];
            codes[start + q] = cd;
            if (cd == 0) {
                store_val(raw, dtype, nr, load_val(x, dtype, (uint64_t)idxb[q]));
                nr++;
                cnt++;
            }
        }
        counts[b] = cnt;
    }
    free(cn); free(cl); free(okb); free(idxb);
    if (!p_out)
        free(P);
    *n_raw = nr;
    return OR_OK;
}

/* Decompression (Sec. 5): blocks in raster order (a valid dependency order
 * since every neighbour lies at lower coordinates), points in local raster
 * order.  Codes re-create the grid value from the same prediction; code 0
 * takes the next raw value and re-derives its grid value. */
int or_decompress(const uint16_t *codes, const void *raw, uint64_t n_raw, const or_consts *c,
                  const uint64_t *dims, int ndim, int dtype, int B, int independent,
                  const or_mlp *m, int mode, const uint8_t *flags, void *xh, int32_t *p_out)
{
    geom g;
    int st = geom_init(&g, dims, ndim, B);
    if (st)
        return st;
    int32_t *P = p_out ? p_out : (int32_t *)malloc((size_t)g.N * sizeof(int32_t));
    if (!P)
        return OR_ENOMEM;
    uint64_t kr = 0;
    iter it;
    it_init(&it, &g);
    int status = OR_OK;
    while (!it.done) {
        int64_t b = it.block;
        int use_net = (mode == 1) || (mode == 2 && flags && flags[b]);
        do {
            int64_t i = lin(&g, it.c);
            uint16_t cd = codes[it.pos];
            if (cd != 0) {
                pred_out po;
                predict_pt(&g, P, it.c, independent, m, use_net, &po);
                int64_t pv = po.pred - ((int64_t)cd - OR_R);
                if (!(fabs((double)pv) < OR_PLIM)) {
                    status = OR_ERANGE;
                    pv = 0;
                }
                P[i] = (int32_t)pv;
                store_val(xh, dtype, (uint64_t)i, inverse_pt(P[i], c, dtype));
            } else {
                if (kr >= n_raw) {
                    status = OR_EINVAL;
                    break;
                }
                double v = load_val(raw, dtype, kr++);
                store_val(xh, dtype, (uint64_t)i, v);
                P[i] = transform_pt(v, c, &status);
            }
        } while (!it_next(&it));
        if (status == OR_EINVAL)
            break;
    }
    if (!p_out)
        free(P);
    return status;
}

/* Stream position and code of selected points, computed point by point from
 * the field alone (for sampled comparisons on large fields).  mode 0/1 as in
 * or_compress (no judge).  Where the network applies (else NaN): yref/slack
 * (optional) receive the BF16 reference network value (precision 1 only),
 * y64/bound (optional) the FP64 network value and the BF16 error bound. */
int or_codes_at(const void *x, const uint64_t *dims, int ndim, int dtype, const or_consts *c,
                int B, int independent, const or_mlp *m, int mode, const uint64_t *idx,
                uint64_t n_idx, uint16_t *codes_out, uint64_t *pos_out, int32_t *p_out,
                double *yref, double *slack, double *y64, double *bound)
{
    geom g;
    int st = geom_init(&g, dims, ndim, B);
    if (st)
        return st;
    int status = OR_OK;
    for (uint64_t s = 0; s < n_idx; ++s) {
        int64_t i = (int64_t)idx[s];
        if (i < 0 || i >= g.N)
            return OR_EINVAL;
        int64_t cc[3], rem = i;
        for (int d = g.D - 1; d >= 0; --d) {
            cc[d] = rem % g.n[d];
            rem /= g.n[d];
        }
        /* grid values of the point and its neighbours only */
        int64_t nbv[8];
        int no = (1 << g.D) - 1;
        int32_t Pl[8];
        double xv = load_val(x, dtype, (uint64_t)i);
        int32_t pv = transform_pt(xv, c, &status);
        int avail = 0, all = 1;
        for (int o = 1; o <= no; ++o) {
            int64_t q[3];
            if (neighbour(&g, cc, o, independent, q)) {
                Pl[o] = transform_pt(load_val(x, dtype, (uint64_t)lin(&g, q)), c, &status);
                avail |= 1 << o;
            } else {
                Pl[o] = 0;
                all = 0;
            }
            nbv[o] = Pl[o];
        }
        if (status)
            return status;
        int64_t pred = 0;
        double yr = NAN, sl = NAN, ye = NAN, bd = NAN;
        if (mode != 0 && m && all) {
            float u[OR_MAXK];
            for (int k = 0; k < m->inputs; ++k)
                u[k] = (float)(int32_t)(nbv[k + 2] - nbv[1]);
            if (m->precision == 1)
                yr = mlp_eval_bf16_ref(m, u, &sl);
            ye = mlp_eval_f64(m, u);
            bd = mlp_bf16_bound(m, u);
            float y = mlp_eval_f32(m, u);
            if (y > 0x1p30f)
                y = 0x1p30f;
            if (!(y >= -0x1p30f))
                y = -0x1p30f;
            pred = nbv[1] + (int64_t)rintf(y);
        } else {
            for (int o = 1; o <= no; ++o)
                if (avail & (1 << o))
                    pred += lorenzo_coef(o) * nbv[o];
        }
        int ok = verify_pt(xv, inverse_pt(pv, c, dtype), c->eps);
        codes_out[s] = code_of(pred, pv, ok);
        if (yref)
            yref[s] = yr;
        if (y64)
            y64[s] = ye;
        if (bound)
            bound[s] = bd;
        if (slack)
            slack[s] = sl;
        if (p_out)
            p_out[s] = pv;
        if (pos_out) {
            int64_t bc[3], lc[3], ext[3];
            for (int d = 0; d < g.D; ++d) {
                bc[d] = cc[d] / g.B;
                lc[d] = cc[d] % g.B;
                ext[d] = bext(&g, d, bc[d]);
            }
            int64_t loc = 0;
            for (int d = 0; d < g.D; ++d)
                loc = loc * ext[d] + lc[d];
            pos_out[s] = (uint64_t)(block_start(&g, bc) + loc);
        }
    }
    return OR_OK;
}

int64_t or_block_start(const uint64_t *dims, int ndim, int B, const int64_t *bc)
{
    geom g;
    if (geom_init(&g, dims, ndim, B))
        return -1;
    return block_start(&g, bc);
}

/* ------------------------------------------------------------------------ */
/* Network initialisation (end of Sec. 4.2)                                   */
/* ------------------------------------------------------------------------ */
/* hidden 0 = +Lorenzo weights on the differences, hidden 1 = -Lorenzo, biases
 * 0, output weights +1/(1+alpha) and -1/(1+alpha) (two distinct numbers; the
 * skip term n_1 carries the unit sum), hidden j >= 2 small splitmix64
 * weights with zero output weight.  The result equals Lorenzo exactly. */
int or_mlp_init(or_mlp *m, int ndim, int hidden, float alpha, uint64_t seed)
{
    if (ndim < 1 || ndim > 3 || hidden < 2 || hidden > OR_MAXH)
        return OR_EINVAL;
    memset(m, 0, sizeof *m);
    m->hidden = hidden;
    m->inputs = (1 << ndim) - 2;
    m->alpha = alpha;
    for (int k = 0; k < m->inputs; ++k) {
        float cf = (float)lorenzo_coef(k + 2);
        m->w1[0][k] = cf;
        m->w1[1][k] = -cf;
    }
    m->v[0] = (float)(1.0 / (1.0 + (double)alpha));
    m->v[1] = -m->v[0];
    for (int j = 2; j < hidden; ++j)
        for (int k = 0; k < m->inputs; ++k) {
            double U = u01(or_splitmix64(seed ^ (uint64_t)(j * m->inputs + k)));
            m->w1[j][k] = (float)(0.1 * (2.0 * U - 1.0));
        }
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Training (Sec. 4.3), FP64                                                  */
/* ------------------------------------------------------------------------ */

/* Sampling: every network-eligible point i with U(i) = u01(splitmix64(seed ^ i))
 * below rho is drawn; it is a validation sample iff U(i) < 0.2 rho (8:2).
 * Only stencils whose 2^D grid values (point and neighbours) all lie in one
 * sign range -- all in (p_zero, b_sign] or all above b_sign -- are kept: the
 * image of zero and the jump across the sign boundary are stand-ins fixed by
 * the transform, not part of the surface the network should learn.  Pairs
 * with any |u_k| >= R or |t| >= R are dropped.  u = neighbour differences
 * n_{k+2} - n_1, t = p - n_1.  Returns the count (<= cap). */
int64_t or_sample(const int32_t *P, const uint64_t *dims, int ndim, int B, int independent,
                  int64_t p_zero, int64_t b_sign, double rho, uint64_t seed, int64_t cap,
                  int32_t *u_out, int32_t *t_out, uint8_t *is_val, uint64_t *idx_out)
{
    geom g;
    if (geom_init(&g, dims, ndim, B))
        return -1;
    int K = (1 << ndim) - 2, no = (1 << ndim) - 1;
    int64_t cnt = 0;
    for (int64_t i = 0; i < g.N; ++i) {
        double U = u01(or_splitmix64(seed ^ (uint64_t)i));
        if (!(U < rho))
            continue;
        int64_t cc[3], rem = i;
        for (int d = g.D - 1; d >= 0; --d) {
            cc[d] = rem % g.n[d];
            rem /= g.n[d];
        }
        int64_t nv[8];
        int all = 1;
        for (int o = 1; o <= no; ++o) {
            int64_t q[3];
            if (!neighbour(&g, cc, o, independent, q)) {
                all = 0;
                break;
            }
            nv[o] = P[lin(&g, q)];
        }
        if (!all)
            continue;
        int npos = 0, nneg = 0;
        nv[0] = P[i];
        for (int o = 0; o <= no; ++o) {
            npos += (nv[o] > p_zero && nv[o] <= b_sign);
            nneg += (nv[o] > b_sign);
        }
        if (npos != no + 1 && nneg != no + 1)
            continue;
        int64_t t = (int64_t)P[i] - nv[1];
        int keep = (t > -OR_R && t < OR_R);
        for (int k = 0; k < K && keep; ++k) {
            int64_t uk = nv[k + 2] - nv[1];
            keep = (uk > -OR_R && uk < OR_R);
        }
        if (!keep)
            continue;
        if (cnt < cap) {
            for (int k = 0; k < K; ++k)
                u_out[cnt * K + k] = (int32_t)(nv[k + 2] - nv[1]);
            t_out[cnt] = (int32_t)t;
            is_val[cnt] = (uint8_t)(U < 0.2 * rho);
            idx_out[cnt] = (uint64_t)i;
        }
        cnt++;
    }
    return cnt;
}

/* FP64 network parameters: flat layout [W1 (H*K) | b1 (H) | v (H) | b2]. */
static int64_t nparams(int H, int K) { return (int64_t)H * K + 2 * H + 1; }

/* Loss and gradient over samples [0, n): mean of 0.5 (y(u/s) - t/s)^2 plus
 * (lambda/2)(|W1|^2 + |v|^2).  The leaky-ReLU derivative at z = 0 is 1. */
double or_loss_grad(const double *theta, int H, int K, double alpha, const double *u,
                    const double *t, int64_t n, double sigma, double lambda, double *grad)
{
    const double *W = theta, *b1 = theta + H * K, *v = theta + H * K + H;
    double b2 = theta[H * K + 2 * H];
    int64_t np = nparams(H, K);
    if (grad)
        for (int64_t q = 0; q < np; ++q)
            grad[q] = 0.0;
    double loss = 0.0;
    double z[OR_MAXH], h[OR_MAXH], us[OR_MAXK];
    for (int64_t i = 0; i < n; ++i) {
        for (int k = 0; k < K; ++k)
            us[k] = u[i * K + k] / sigma;
        double y = b2;
        for (int j = 0; j < H; ++j) {
            double a = b1[j];
            for (int k = 0; k < K; ++k)
                a += W[j * K + k] * us[k];
            z[j] = a;
            h[j] = (a < 0.0) ? alpha * a : a;
            y += v[j] * h[j];
        }
        double res = y - t[i] / sigma;
        loss += 0.5 * res * res;
        if (grad) {
            double gy = res / (double)n;
            for (int j = 0; j < H; ++j) {
                grad[H * K + H + j] += gy * h[j];
                double gz = gy * v[j] * ((z[j] < 0.0) ? alpha : 1.0);
                grad[H * K + j] += gz;
                for (int k = 0; k < K; ++k)
                    grad[j * K + k] += gz * us[k];
            }
            grad[H * K + 2 * H] += gy;
        }
    }
    loss /= (double)(n > 0 ? n : 1);
    double reg = 0.0;
    for (int q = 0; q < H * K; ++q)
        reg += W[q] * W[q];
    for (int j = 0; j < H; ++j)
        reg += v[j] * v[j];
    loss += 0.5 * lambda * reg;
    if (grad) {
        for (int q = 0; q < H * K; ++q)
            grad[q] += lambda * W[q];
        for (int j = 0; j < H; ++j)
            grad[H * K + H + j] += lambda * v[j];
    }
    return loss;
}

/* Magnitudes behind each gradient component of or_loss_grad, for error
 * bounds of finite-precision evaluations of the same sums:
 *   gabs[q] = sum over samples of |the sample's contribution| / n, plus
 *             |lambda w| (the terms of the sum itself);
 *   gres[q] = sum over samples of F_i |d y_i / d theta_q| / n, with
 *             F_i = |b2| + sum_j |v_j| (|b1_j| + sum_k |w_jk u_ik / s|) + |t_i / s|
 *             the magnitudes the residual y_i - t_i / s is computed from
 *             (its rounding error is a small multiple of F_i).
 * gres may be NULL. */
void or_loss_grad_abs(const double *theta, int H, int K, double alpha, const double *u,
                      const double *t, int64_t n, double sigma, double lambda, double *gabs,
                      double *gres)
{
    const double *W = theta, *b1 = theta + H * K, *v = theta + H * K + H;
    double b2 = theta[H * K + 2 * H];
    int64_t np = nparams(H, K);
    for (int64_t q = 0; q < np; ++q) {
        gabs[q] = 0.0;
        if (gres)
            gres[q] = 0.0;
    }
    double z[OR_MAXH], h[OR_MAXH], us[OR_MAXK];
    for (int64_t i = 0; i < n; ++i) {
        for (int k = 0; k < K; ++k)
            us[k] = u[i * K + k] / sigma;
        double y = b2, F = fabs(b2) + fabs(t[i] / sigma);
        for (int j = 0; j < H; ++j) {
            double a = b1[j], m = fabs(b1[j]);
            for (int k = 0; k < K; ++k) {
                a += W[j * K + k] * us[k];
                m += fabs(W[j * K + k] * us[k]);
            }
            z[j] = a;
            h[j] = (a < 0.0) ? alpha * a : a;
            y += v[j] * h[j];
            F += fabs(v[j]) * m;
        }
        const double gy = fabs(y - t[i] / sigma) / (double)n, fr = F / (double)n;
        for (int j = 0; j < H; ++j) {
            const double dz = fabs(v[j]) * ((z[j] < 0.0) ? alpha : 1.0);
            gabs[H * K + H + j] += gy * fabs(h[j]);
            gabs[H * K + j] += gy * dz;
            for (int k = 0; k < K; ++k)
                gabs[j * K + k] += gy * dz * fabs(us[k]);
            if (gres) {
                gres[H * K + H + j] += fr * fabs(h[j]);
                gres[H * K + j] += fr * dz;
                for (int k = 0; k < K; ++k)
                    gres[j * K + k] += fr * dz * fabs(us[k]);
            }
        }
        gabs[H * K + 2 * H] += gy;
        if (gres)
            gres[H * K + 2 * H] += fr;
    }
    for (int q = 0; q < H * K; ++q)
        gabs[q] += fabs(lambda * W[q]);
    for (int j = 0; j < H; ++j)
        gabs[H * K + H + j] += fabs(lambda * v[j]);
}

/* Network value in the scaled domain of the trainer (FP64): the output for
 * the inputs u / sigma, parameters theta = [w1 | b1 | v | b2]. */
void or_theta_eval_many(const double *theta, int H, int K, double alpha, const double *u,
                        int64_t n, double sigma, double *y)
{
    const double *W = theta, *b1 = theta + H * K, *v = theta + H * K + H;
    for (int64_t i = 0; i < n; ++i) {
        double acc = theta[H * K + 2 * H];
        for (int j = 0; j < H; ++j) {
            double a = b1[j];
            for (int k = 0; k < K; ++k)
                a += W[j * K + k] * (u[i * K + k] / sigma);
            acc += v[j] * ((a < 0.0) ? alpha * a : a);
        }
        y[i] = acc;
    }
}

/* One pass over [0, n) in minibatches of `batch`, in index order.
 * opt 0 = SGD, 1 = Adam (beta1 0.9, beta2 0.999, eps 1e-8).
 * theta is updated in place; adam_m/adam_v/step carry Adam state. */
int or_train_pass(double *theta, int H, int K, double alpha, const double *u, const double *t,
                  int64_t n, double sigma, double lambda, double lr, int batch, int opt,
                  double *adam_m, double *adam_v, int64_t *step)
{
    int64_t np = nparams(H, K);
    double *g = (double *)malloc((size_t)np * sizeof(double));
    if (!g)
        return OR_ENOMEM;
    for (int64_t s = 0; s < n; s += batch) {
        int64_t nb = (n - s < batch) ? (n - s) : batch;
        or_loss_grad(theta, H, K, alpha, u + s * K, t + s, nb, sigma, lambda, g);
        if (opt == 0) {
            for (int64_t q = 0; q < np; ++q)
                theta[q] -= lr * g[q];
        } else {
            (*step)++;
            double b1c = 1.0 - pow(0.9, (double)*step);
            double b2c = 1.0 - pow(0.999, (double)*step);
            for (int64_t q = 0; q < np; ++q) {
                adam_m[q] = 0.9 * adam_m[q] + 0.1 * g[q];
                adam_v[q] = 0.999 * adam_v[q] + 0.001 * g[q] * g[q];
                double mh = adam_m[q] / b1c, vh = adam_v[q] / b2c;
                theta[q] -= lr * mh / (sqrt(vh) + 1e-8);
            }
        }
    }
    free(g);
    return OR_OK;
}

/* FP64 parameters (scaled domain) <-> FP32 network (raw grid domain). */
void or_theta_from_mlp(const or_mlp *m, double *theta)
{
    int H = m->hidden, K = m->inputs;
    for (int j = 0; j < H; ++j) {
        for (int k = 0; k < K; ++k)
            theta[j * K + k] = m->w1[j][k];
        theta[H * K + j] = m->b1[j];
        theta[H * K + H + j] = m->v[j];
    }
    theta[H * K + 2 * H] = m->b2;
}

/* fold sigma: W1/sigma, b1, v*sigma, b2*sigma; round to FP32 */
void or_mlp_from_theta(or_mlp *m, const double *theta, double sigma)
{
    int H = m->hidden, K = m->inputs;
    for (int j = 0; j < H; ++j) {
        for (int k = 0; k < K; ++k)
            m->w1[j][k] = (float)(theta[j * K + k] / sigma);
        m->b1[j] = (float)theta[H * K + j];
        m->v[j] = (float)(theta[H * K + H + j] * sigma);
    }
    m->b2 = (float)(theta[H * K + 2 * H] * sigma);
}

/* Validation score of a network: J of the codes it gives on the samples
 * (code = rint(y(u)) - t + R, or 0 when out of range). Higher J = lower
 * entropy. */
int64_t or_val_score(const or_mlp *m, const int32_t *u, const int32_t *t, int64_t n)
{
    uint16_t *cd = (uint16_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(uint16_t));
    if (!cd)
        return INT64_MIN;
    int K = m->inputs;
    for (int64_t i = 0; i < n; ++i) {
        float uf[OR_MAXK];
        for (int k = 0; k < K; ++k)
            uf[k] = (float)u[i * K + k];
        float y = mlp_eval_f32(m, uf);
        if (y > 0x1p30f)
            y = 0x1p30f;
        if (!(y >= -0x1p30f))
            y = -0x1p30f;
        cd[i] = code_of((int64_t)rintf(y), (int64_t)t[i], 1);
    }
    int64_t J = entropy_j(cd, n);
    free(cd);
    return J;
}

/* The oracle's training rule: sample (rho, seed), sigma = max(1, RMS t) over
 * the training part, candidates = {untrained} + lr x lambda grid, each one
 * SGD pass (batch 256) from the initialisation; keep the candidate with the
 * highest validation J (ties: lower index).  Returns the chosen index. */
int or_train_rule(const int32_t *P, const uint64_t *dims, int ndim, int B, int independent,
                  int64_t p_zero, int64_t b_sign, double rho, uint64_t seed, const or_mlp *init, const double *lrs, int nlr,
                  const double *lambdas, int nlam, int batch, int opt, or_mlp *out,
                  int64_t *n_train_out, int64_t *n_val_out)
{
    geom g;
    if (geom_init(&g, dims, ndim, B))
        return OR_EINVAL;
    int K = (1 << ndim) - 2, H = init->hidden;
    if (init->inputs != K)
        return OR_EINVAL;
    int64_t cap = or_sample(P, dims, ndim, B, independent, p_zero, b_sign, rho, seed, 0, NULL,
                            NULL, NULL, NULL);
    if (cap < 0)
        return OR_EINVAL;
    int32_t *us = (int32_t *)malloc((size_t)(cap * K + 1) * sizeof(int32_t));
    int32_t *ts = (int32_t *)malloc((size_t)(cap + 1) * sizeof(int32_t));
    uint8_t *iv = (uint8_t *)malloc((size_t)(cap + 1));
    uint64_t *ix = (uint64_t *)malloc((size_t)(cap + 1) * sizeof(uint64_t));
    double *ud = (double *)malloc((size_t)(cap * K + 1) * sizeof(double));
    double *td = (double *)malloc((size_t)(cap + 1) * sizeof(double));
    int32_t *uv = (int32_t *)malloc((size_t)(cap * K + 1) * sizeof(int32_t));
    int32_t *tv = (int32_t *)malloc((size_t)(cap + 1) * sizeof(int32_t));
    int64_t np = nparams(H, K);
    double *th = (double *)malloc((size_t)np * sizeof(double));
    double *am = (double *)malloc((size_t)np * sizeof(double));
    double *av = (double *)malloc((size_t)np * sizeof(double));
    int st = OR_OK;
    if (!us || !ts || !iv || !ix || !ud || !td || !uv || !tv || !th || !am || !av) {
        st = OR_ENOMEM;
        goto done;
    }
    or_sample(P, dims, ndim, B, independent, p_zero, b_sign, rho, seed, cap, us, ts, iv, ix);
    int64_t ntr = 0, nva = 0;
    double ss = 0.0;
    for (int64_t i = 0; i < cap; ++i) {
        if (iv[i]) {
            for (int k = 0; k < K; ++k)
                uv[nva * K + k] = us[i * K + k];
            tv[nva++] = ts[i];
        } else {
            for (int k = 0; k < K; ++k)
                ud[ntr * K + k] = (double)us[i * K + k];
            td[ntr] = (double)ts[i];
            ss += td[ntr] * td[ntr];
            ntr++;
        }
    }
    double sigma = ntr ? sqrt(ss / (double)ntr) : 1.0;
    if (sigma < 1.0)
        sigma = 1.0;
    *out = *init;
    int64_t best = or_val_score(init, uv, tv, nva);
    int besti = 0, idx = 0;
    for (int a = 0; a < nlr; ++a)
        for (int b = 0; b < nlam; ++b) {
            idx++;
            or_theta_from_mlp(init, th);
            for (int64_t q = 0; q < np; ++q)
                am[q] = av[q] = 0.0;
            int64_t step = 0;
            st = or_train_pass(th, H, K, (double)init->alpha, ud, td, ntr, sigma, lambdas[b],
                               lrs[a], batch, opt, am, av, &step);
            if (st)
                goto done;
            or_mlp cand = *init;
            or_mlp_from_theta(&cand, th, sigma);
            int64_t sc = or_val_score(&cand, uv, tv, nva);
            if (sc > best) {
                best = sc;
                besti = idx;
                *out = cand;
            }
        }
    *n_train_out = ntr;
    *n_val_out = nva;
    st = besti;
done:
    free(us); free(ts); free(iv); free(ix); free(ud); free(td); free(uv); free(tv);
    free(th); free(am); free(av);
    return st;
}

/* FP32 evaluation of a network on given inputs (diagnostic). */
void or_mlp_eval_many(const or_mlp *m, const float *u, int64_t n, float *y)
{
    for (int64_t i = 0; i < n; ++i)
        y[i] = mlp_eval_f32(m, u + i * m->inputs);
}

void or_mlp_eval_bf16_many(const or_mlp *m, const float *u, int64_t n, double *y, double *slack)
{
    for (int64_t i = 0; i < n; ++i)
        y[i] = mlp_eval_bf16_ref(m, u + i * m->inputs, &slack[i]);
}

float or_bf16_rne(float f) { return bf16_rne(f); }

/* ------------------------------------------------------------------------ */
/* Entropy coding of the codes (Sec. 4.1: the quantised codes go through a   */
/* Huffman coding stage; Algorithm 1's Huffman step; Sec. 5 rebuilds the     */
/* tree to decode).  Code lengths: optimal prefix code with no codeword      */
/* longer than Lmax, by package-merge (Larmore and Hirschberg 1990);         */
/* codewords: canonical assignment (shorter codes first, equal lengths in    */
/* symbol order; the convention of RFC 1951, Sec. 3.2.2).  Bitstream: the    */
/* codewords of the codes in stream order, concatenated; bit i of the stream */
/* is bit 31 - (i mod 32) of 32-bit word i / 32 (most significant first).    */
/* ------------------------------------------------------------------------ */

typedef struct {
    uint64_t w;
    int32_t a, b; /* leaf: a = symbol, b = -1; package: the two item indices (previous row) */
} pm_item;

static int pm_cmp(const void *x, const void *y)
{
    const pm_item *p = (const pm_item *)x, *q = (const pm_item *)y;
    return (p->w > q->w) - (p->w < q->w);
}

/* add 1 to the length of every leaf under item k of row r */
static void pm_count(pm_item **rows, int r, int k, uint8_t *len)
{
    const pm_item *it = &rows[r][k];
    if (it->b < 0) {
        len[it->a]++;
        return;
    }
    pm_count(rows, r - 1, it->a, len);
    pm_count(rows, r - 1, it->b, len);
}

/* Code lengths of the nsym symbols with counts hist (0 = unused, length 0).
 * One used symbol gets length 1.  Returns 0, or -1 if Lmax is too small for
 * the number of used symbols (2^Lmax < n) or memory runs out. */
int or_huff_lengths(const uint64_t *hist, int nsym, int Lmax, uint8_t *len)
{
    int n = 0;
    for (int s = 0; s < nsym; ++s) {
        len[s] = 0;
        n += hist[s] != 0;
    }
    if (n == 0)
        return 0;
    if (n == 1) {
        for (int s = 0; s < nsym; ++s)
            if (hist[s])
                len[s] = 1;
        return 0;
    }
    if (Lmax < 1 || Lmax > 62 || ((uint64_t)1 << Lmax) < (uint64_t)n)
        return -1;
    /* leaves sorted by count (ties: symbol order, by a stable sort of the
     * symbol-ordered list) */
    pm_item *leaves = (pm_item *)malloc((size_t)n * sizeof(pm_item));
    pm_item **rows = (pm_item **)calloc((size_t)Lmax, sizeof(pm_item *));
    int *rn = (int *)calloc((size_t)Lmax, sizeof(int));
    if (!leaves || !rows || !rn) {
        free(leaves); free(rows); free(rn);
        return -1;
    }
    int k = 0;
    for (int s = 0; s < nsym; ++s)
        if (hist[s]) {
            leaves[k].w = hist[s];
            leaves[k].a = s;
            leaves[k].b = -1;
            k++;
        }
    /* insertion sort keeps equal counts in symbol order (stable) */
    for (int i = 1; i < n; ++i) {
        pm_item t = leaves[i];
        int j = i - 1;
        while (j >= 0 && leaves[j].w > t.w) {
            leaves[j + 1] = leaves[j];
            j--;
        }
        leaves[j + 1] = t;
    }
    (void)pm_cmp;
    /* row 0: the leaves; row r: the leaves merged with the packages (pairs)
     * of row r - 1, in weight order (a leaf before a package of equal weight) */
    int st = 0;
    for (int r = 0; r < Lmax && st == 0; ++r) {
        int np = r == 0 ? 0 : rn[r - 1] / 2;
        rows[r] = (pm_item *)malloc((size_t)(n + np) * sizeof(pm_item));
        if (!rows[r]) {
            st = -1;
            break;
        }
        int i = 0, j = 0, o = 0;
        while (i < n || j < np) {
            uint64_t pw = 0;
            if (j < np)
                pw = rows[r - 1][2 * j].w + rows[r - 1][2 * j + 1].w;
            if (j >= np || (i < n && leaves[i].w <= pw)) {
                rows[r][o++] = leaves[i++];
            } else {
                rows[r][o].w = pw;
                rows[r][o].a = 2 * j;
                rows[r][o].b = 2 * j + 1;
                o++;
                j++;
            }
        }
        rn[r] = o;
    }
    if (st == 0 && rn[Lmax - 1] < 2 * n - 2)
        st = -1;
    if (st == 0) {
        /* the 2n - 2 lightest items of the last row; every leaf occurrence
         * inside them adds one to that leaf's length */
        int take = 2 * n - 2;
        for (int q = 0; q < take; ++q)
            pm_count(rows, Lmax - 1, q, len);
    }
    for (int r = 0; r < Lmax; ++r)
        free(rows[r]);
    free(rows); free(rn); free(leaves);
    return st;
}

/* Canonical codewords of the lengths (RFC 1951, Sec. 3.2.2): returns 0, or
 * -1 if the lengths over-subscribe the code space (Kraft sum > 1). */
int or_huff_canonical(const uint8_t *len, int nsym, int Lmax, uint32_t *code)
{
    uint32_t bl_count[64] = {0}, next_code[64] = {0};
    for (int s = 0; s < nsym; ++s) {
        if (len[s] > Lmax)
            return -1;
        if (len[s])
            bl_count[len[s]]++;
    }
    uint64_t c = 0;
    for (int b = 1; b <= Lmax; ++b) {
        c = (c + bl_count[b - 1]) << 1;
        next_code[b] = (uint32_t)c;
        if (c + bl_count[b] > ((uint64_t)1 << b))
            return -1;
    }
    for (int s = 0; s < nsym; ++s)
        code[s] = len[s] ? next_code[len[s]]++ : 0;
    return 0;
}

/* The bitstream of n codes (stream order): word i/32, bit 31 - i%32.
 * words must hold ceil(total bits / 32) zeroed words.  Returns the bit count. */
int64_t or_huff_encode(const uint16_t *codes, int64_t n, const uint8_t *len, const uint32_t *code,
                       uint32_t *words)
{
    int64_t pos = 0;
    for (int64_t i = 0; i < n; ++i) {
        int l = len[codes[i]];
        uint32_t c = code[codes[i]];
        for (int k = l - 1; k >= 0; --k) {
            if ((c >> k) & 1u)
                words[pos >> 5] |= 1u << (31 - (pos & 31));
            pos++;
        }
    }
    return pos;
}

/* Decode n codes from a bitstream starting at bit `start`, bit by bit down
 * the canonical code (a codeword of length l is the l-th bit prefix whose
 * value lies in [first[l], first[l] + count[l]) ).  Returns the bit position
 * after the last code, or -1 if the bits match no codeword. */
int64_t or_huff_decode(const uint32_t *words, int64_t start, int64_t n, const uint8_t *len,
                       int nsym, int Lmax, uint16_t *out)
{
    uint32_t bl_count[64] = {0}, first[64] = {0};
    int32_t index[64] = {0};
    for (int s = 0; s < nsym; ++s)
        if (len[s])
            bl_count[len[s]]++;
    /* symbols in canonical order: by length, then symbol */
    int32_t *sorted = (int32_t *)malloc((size_t)(nsym > 0 ? nsym : 1) * sizeof(int32_t));
    if (!sorted)
        return -1;
    int m = 0;
    uint32_t c = 0;
    for (int b = 1; b <= Lmax; ++b) {
        c = (c + bl_count[b - 1]) << 1;
        first[b] = c;
        index[b] = m;
        for (int s = 0; s < nsym; ++s)
            if (len[s] == b)
                sorted[m++] = s;
    }
    int64_t pos = start;
    for (int64_t i = 0; i < n; ++i) {
        uint32_t v = 0;
        int b = 0, found = 0;
        while (b < Lmax) {
            v = (v << 1) | ((words[pos >> 5] >> (31 - (pos & 31))) & 1u);
            pos++;
            b++;
            if (v - first[b] < bl_count[b]) {
                out[i] = (uint16_t)sorted[index[b] + (int32_t)(v - first[b])];
                found = 1;
                break;
            }
        }
        if (!found) {
            free(sorted);
            return -1;
        }
    }
    free(sorted);
    return pos;
}

/* ------------------------------------------------------------------------ */
/* The codebook of the training phase (Sec. 4.3): one table built once from  */
/* the code frequencies of the validation blocks and reused for every block  */
/* of the compression.  The paper averages the counts per block; an average  */
/* is the total over the validation set divided by the number of blocks, a   */
/* common factor, so the totals give the same lengths.  A code the           */
/* validation never produced has no codeword of its own: the escape symbol   */
/* (alphabet index 65536) stands for every such code and is followed in the  */
/* stream by the code's 16 bits, most significant first.  The escape weighs  */
/* the number of codes seen exactly once, at least 1 (Good-Turing estimate   */
/* of the probability of an unseen code).  With an escape in the alphabet no */
/* codeword is longer than 16 bits, so an escaped code takes at most 32;     */
/* without one (every code seen) the limit is 32.                            */
/* ------------------------------------------------------------------------ */

#define OR_ESC 65536

/* len[0..65536]: the lengths of the 65,536 codes and of the escape (0 when
 * unused).  Returns the escape's length (0: no escape), or -1. */
int or_huff_trained_lengths(const uint64_t *hist, uint8_t *len)
{
    uint64_t *w = (uint64_t *)malloc((OR_ESC + 1) * sizeof(uint64_t));
    if (!w)
        return -1;
    uint64_t ones = 0;
    int unseen = 0;
    for (int s = 0; s < OR_ESC; ++s) {
        w[s] = hist[s];
        ones += hist[s] == 1;
        unseen |= hist[s] == 0;
    }
    w[OR_ESC] = unseen ? (ones > 0 ? ones : 1) : 0;
    int st = or_huff_lengths(w, OR_ESC + 1, unseen ? 16 : 32, len);
    free(w);
    if (st)
        return -1;
    return len[OR_ESC];
}

/* The bitstream of n codes with the escape: a code with a codeword takes
 * it; any other code takes the escape's codeword, then its own 16 bits.
 * len/code have 65,537 entries.  words must hold enough zeroed words.
 * Returns the bit count, or -1 for a code with no codeword and no escape. */
int64_t or_huff_encode_esc(const uint16_t *codes, int64_t n, const uint8_t *len,
                           const uint32_t *code, uint32_t *words)
{
    int64_t pos = 0;
    for (int64_t i = 0; i < n; ++i) {
        const int s = codes[i];
        int nb;
        uint64_t v;
        if (len[s]) {
            nb = len[s];
            v = code[s];
        } else if (len[OR_ESC]) {
            nb = len[OR_ESC] + 16;
            v = ((uint64_t)code[OR_ESC] << 16) | (uint64_t)s;
        } else {
            return -1;
        }
        for (int k = nb - 1; k >= 0; --k) {
            if ((v >> k) & 1u)
                words[pos >> 5] |= 1u << (31 - (pos & 31));
            pos++;
        }
    }
    return pos;
}

/* Decode n codes from bit `start`, bit by bit down the canonical code of the
 * 65,537-symbol alphabet; the escape symbol is followed by the code's 16
 * bits.  Returns the bit position after the last code, or -1 if the bits
 * match no codeword. */
int64_t or_huff_decode_esc(const uint32_t *words, int64_t start, int64_t n, const uint8_t *len,
                           int Lmax, uint16_t *out)
{
    const int nsym = OR_ESC + 1;
    uint32_t bl_count[64] = {0}, first[64] = {0};
    int32_t index[64] = {0};
    for (int s = 0; s < nsym; ++s)
        if (len[s])
            bl_count[len[s]]++;
    int32_t *sorted = (int32_t *)malloc((size_t)nsym * sizeof(int32_t));
    if (!sorted)
        return -1;
    int m = 0;
    uint32_t c = 0;
    for (int b = 1; b <= Lmax; ++b) {
        c = (c + bl_count[b - 1]) << 1;
        first[b] = c;
        index[b] = m;
        for (int s = 0; s < nsym; ++s)
            if (len[s] == b)
                sorted[m++] = s;
    }
    int64_t pos = start;
    for (int64_t i = 0; i < n; ++i) {
        uint32_t v = 0;
        int b = 0, sym = -1;
        while (b < Lmax) {
            v = (v << 1) | ((words[pos >> 5] >> (31 - (pos & 31))) & 1u);
            pos++;
            b++;
            if (v - first[b] < bl_count[b]) {
                sym = sorted[index[b] + (int32_t)(v - first[b])];
                break;
            }
        }
        if (sym < 0) {
            free(sorted);
            return -1;
        }
        if (sym == OR_ESC) {
            uint32_t r = 0;
            for (int k = 0; k < 16; ++k) {
                r = (r << 1) | ((words[pos >> 5] >> (31 - (pos & 31))) & 1u);
                pos++;
            }
            sym = (int)r;
        }
        out[i] = (uint16_t)sym;
    }
    free(sorted);
    return pos;
}

/* The table's validation set (Sec. 4.3: the table comes from the code
 * frequencies of the validation blocks, on which the compression is
 * simulated): block b (stream order) belongs to it iff
 * u01(splitmix64(seed ^ b)) < frac.  hist[65536] receives the counts of
 * their codes, given the codes of the whole field in stream order (blocks in
 * raster order, each block's points contiguous).  The paper averages the
 * counts per block; the totals give the same table.  Returns the number of
 * blocks in the set, or -1 for a bad geometry. */
int64_t or_table_hist(const uint16_t *codes, const uint64_t *dims, int ndim, int B, double frac,
                      uint64_t seed, uint64_t *hist)
{
    geom g;
    if (geom_init(&g, dims, ndim, B))
        return -1;
    memset(hist, 0, 65536 * sizeof(uint64_t));
    int64_t pos = 0, nsel = 0;
    for (int64_t b = 0; b < g.nblocks; ++b) {
        int64_t rem = b, size = 1;
        for (int d = g.D - 1; d >= 0; --d) {
            const int64_t bc = rem % g.nb[d];
            rem /= g.nb[d];
            const int64_t e = g.n[d] - bc * g.B;
            size *= e < g.B ? e : g.B;
        }
        if (u01(or_splitmix64(seed ^ (uint64_t)b)) < frac) {
            nsel++;
            for (int64_t k = 0; k < size; ++k)
                hist[codes[pos + k]]++;
        }
        pos += size;
    }
    return nsel;
}

/* FP64 value of the network and the BF16 error bound of mlp_bf16_bound. */
void or_mlp_eval_f64_many(const or_mlp *m, const float *u, int64_t n, double *y, double *bound)
{
    for (int64_t i = 0; i < n; ++i) {
        y[i] = mlp_eval_f64(m, u + i * m->inputs);
        if (bound)
            bound[i] = mlp_bf16_bound(m, u + i * m->inputs);
    }
}

size_t or_sizeof_mlp(void) { return sizeof(or_mlp); }
size_t or_sizeof_consts(void) { return sizeof(or_consts); }
size_t or_sizeof_stats(void) { return sizeof(or_stats); }

/* ------------------------------------------------------------------------ */
/* Open-loop mode: the paper's literal data selection (Sec. 4.4.1, 4.4.2).  */
/* The compressor predicts every point from its neighbours' raw values in   */
/* the log domain (continuous grid coordinates, before rounding), so all    */
/* points are predicted independently; the decompressor can only predict   */
/* from its own reconstructions, so reconstruction errors can accumulate.   */
/* The controls the paper gives against that drift:                          */
/*   - balance (equilibrium) points, stored raw and exact: codes out of the  */
/*     m-bit range (Sec. 4.3, Sec. 5), the first point of every block (each  */
/*     sub-block starts decompression from a balance point, Sec. 4.4.2), and */
/*     deliberate ones: a point becomes one when `gap` points in a row of    */
/*     its block carried none (Sec. 4.4.1(b); gap 0 = none inserted);        */
/*   - m chosen by coverage, the share of points whose code is in range:    */
/*     closest to 50% below a 1.5% bound, to 80% from 1.5% up (Sec. 4.3);   */
/*   - a model is accepted if the decompressed error stays within 1.5 times */
/*     the bound (Sec. 4.3).                                                 */
/* Independent blocks only.  Codes: e = pred - t, c = rint(e); code c + 2^(m-1) */
/* where |c| < 2^(m-1), else 0 (balance point).                              */
/* ------------------------------------------------------------------------ */

/* continuous grid coordinate of x (the grid value before rounding, Eq. 6, 7) */
static double tcoord(double x, const or_consts *c)
{
    if (x == 0.0)
        return (double)c->p_zero;
    if (x > 0.0)
        return (or_det_log2(x) + c->Lp) * c->r;
    return (or_det_log2(-x) + c->Ln) * c->r + (double)c->delta;
}

/* inverse of a continuous coordinate: zero / positive / negative by its
 * nearest grid value, magnitude from the coordinate itself */
static double tinverse(double t, const or_consts *c, int dtype)
{
    double q = rint(t);
    double v;
    if (q <= (double)c->p_zero)
        v = 0.0;
    else if (q <= (double)c->b_sign)
        v = or_det_exp2(t * c->w - c->Lp);
    else
        v = -or_det_exp2((t - (double)c->delta) * c->w - c->Ln);
    return cast_t(v, dtype);
}

double or_tcoord(double x, const or_consts *c) { return tcoord(x, c); }
double or_tinverse(double t, const or_consts *c, int dtype) { return tinverse(t, c, dtype); }

/* prediction of point c from coordinates T of its block's neighbours:
 * network (FP32 on u_k = float(t_{k+2} - t_1)) where every neighbour exists,
 * else Lorenzo over the available ones, added in offset order */
static double ol_predict(const geom *g, const double *T, const int64_t *c, const or_mlp *m)
{
    int no = (1 << g->D) - 1;
    double nv[8];
    int avail = 0, all = 1;
    for (int o = 1; o <= no; ++o) {
        int64_t q[3];
        if (neighbour(g, c, o, 1, q)) {
            nv[o] = T[lin(g, q)];
            avail |= 1 << o;
        } else {
            nv[o] = 0.0;
            all = 0;
        }
    }
    if (m && all) {
        float u[OR_MAXK];
        for (int k = 0; k < m->inputs; ++k)
            u[k] = (float)(nv[k + 2] - nv[1]);
        return nv[1] + (double)mlp_eval_f32(m, u);
    }
    double s = 0.0;
    for (int o = 1; o <= no; ++o)
        if (avail & (1 << o))
            s = lorenzo_coef(o) > 0 ? s + nv[o] : s - nv[o];
    return s;
}

/* smallest m with |c| < 2^(m-1) (1 for c = 0), 17 when no m <= 16 covers it */
static int m_needed(double c)
{
    double a = fabs(c);
    for (int m = 1; m <= 16; ++m)
        if (a < ldexp(1.0, m - 1))
            return m;
    return 17;
}

/* Open-loop compression.  Outputs (caller-allocated): codes[N] (stream
 * order), counts[nblocks], raw (dtype, capacity N) and n_raw, hist[18]
 * (hist[m] = points whose prediction error first fits m bits, before any
 * balance point is forced), consts.  m: model or NULL (Lorenzo). */
int or_openloop_encode(const void *x, const uint64_t *dims, int ndim, int dtype, double eps,
                       int B, const or_mlp *m, int mbits, int gap, uint16_t *codes,
                       uint32_t *counts, void *raw, uint64_t *n_raw, uint64_t *hist,
                       or_consts *consts)
{
    geom g;
    int st = geom_init(&g, dims, ndim, B);
    if (st)
        return st;
    if ((dtype != OR_F32 && dtype != OR_F64) || mbits < 2 || mbits > 16 || gap < 0)
        return OR_EINVAL;
    if (m && (m->inputs != (1 << ndim) - 2 || m->hidden < 1 || m->hidden > OR_MAXH))
        return OR_EINVAL;
    or_stats sts;
    st = or_stats_compute(x, (uint64_t)g.N, dtype, &sts);
    if (st)
        return st;
    st = or_consts_compute(&sts, dtype, eps, consts);
    if (st)
        return st;
    double *T = (double *)malloc((size_t)g.N * sizeof(double));
    if (!T)
        return OR_ENOMEM;
    for (int64_t i = 0; i < g.N; ++i)
        T[i] = tcoord(load_val(x, dtype, (uint64_t)i), consts);
    for (int j = 0; j < 18; ++j)
        hist[j] = 0;
    const double half = ldexp(1.0, mbits - 1);
    uint64_t nr = 0;
    iter it;
    it_init(&it, &g);
    while (!it.done) {
        int64_t b = it.block, since = 0, k = 0;
        uint32_t cnt = 0;
        do {
            int64_t i = lin(&g, it.c);
            double cq = rint(ol_predict(&g, T, it.c, m) - T[i]);
            hist[m_needed(cq)]++;
            int balance = !(fabs(cq) < half);
            if (k == 0)
                balance = 1; /* the block's starting point */
            else if (!balance && gap > 0 && since + 1 >= gap)
                balance = 1; /* deliberate */
            since = balance ? 0 : since + 1;
            uint16_t cd = balance ? 0 : (uint16_t)(cq + half);
            codes[it.pos] = cd;
            if (cd == 0) {
                store_val(raw, dtype, nr++, load_val(x, dtype, (uint64_t)i));
                cnt++;
            }
            k++;
        } while (!it_next(&it));
        counts[b] = cnt;
    }
    free(T);
    *n_raw = nr;
    return OR_OK;
}

/* Open-loop decompression: blocks and points in stream order, each point
 * predicted from the reconstructed coordinates of its block. */
int or_openloop_decode(const uint16_t *codes, const void *raw, uint64_t n_raw, const or_consts *c,
                       const uint64_t *dims, int ndim, int dtype, int B, const or_mlp *m,
                       int mbits, void *xh, double *t_out)
{
    geom g;
    int st = geom_init(&g, dims, ndim, B);
    if (st)
        return st;
    if (mbits < 2 || mbits > 16)
        return OR_EINVAL;
    double *T = t_out ? t_out : (double *)malloc((size_t)g.N * sizeof(double));
    if (!T)
        return OR_ENOMEM;
    const double half = ldexp(1.0, mbits - 1);
    uint64_t kr = 0;
    iter it;
    it_init(&it, &g);
    int status = OR_OK;
    while (!it.done && status == OR_OK) {
        do {
            int64_t i = lin(&g, it.c);
            uint16_t cd = codes[it.pos];
            if (cd == 0) {
                if (kr >= n_raw) {
                    status = OR_EINVAL;
                    break;
                }
                double v = load_val(raw, dtype, kr++);
                store_val(xh, dtype, (uint64_t)i, v);
                T[i] = tcoord(v, c);
            } else {
                T[i] = ol_predict(&g, T, it.c, m) - ((double)cd - half);
                store_val(xh, dtype, (uint64_t)i, tinverse(T[i], c, dtype));
            }
        } while (!it_next(&it));
    }
    if (!t_out)
        free(T);
    return status;
}

/* m whose coverage (share of points with |c| < 2^(m-1)) is closest to the
 * target: 50% for eps below 1.5%, 80% from 1.5% up; ties to the smaller m */
int or_openloop_choose_m(const uint64_t *hist, double eps)
{
    uint64_t n = 0;
    for (int j = 0; j < 18; ++j)
        n += hist[j];
    double target = eps < 0.015 ? 0.5 : 0.8;
    int best = 2;
    double bestd = INFINITY;
    uint64_t cum = 0;
    for (int mm = 1; mm <= 16; ++mm) {
        cum += hist[mm];
        if (mm < 2)
            continue;
        double cov = n ? (double)cum / (double)n : 1.0;
        double d = fabs(cov - target);
        if (d < bestd) {
            bestd = d;
            best = mm;
        }
    }
    return best;
}
