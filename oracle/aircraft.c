/* Oracle: the discrete abstraction of the sampled aircraft system --
 * TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).
 *
 * Sect. V-B builds the abstraction of a sampled system by covering the
 * state space with a grid of compact hyper-rectangles and over-approximating
 * the attainable set phi(tau, Omega, u) of every cell Omega under every input
 * u by a hyper-rectangle; F'(Omega, u) is the set of cells that meet it.
 * Sect. VI-A applies this to the point-mass aircraft
 *     x1' = x4 cos x3,  x2' = x4 sin x3,
 *     x3' = p_L x4 sin(u2) / m,  x4' = (u1 - p_D x4^2) / m,
 * (positions x1, x2, heading x3, speed x4; thrust u1, bank angle u2).
 *
 * The paper takes its enclosures from a validated integrator it cites; this
 * oracle uses the first-order interval Taylor method (R. E. Moore, Interval
 * Analysis, 1966), written out here:
 *   - every interval operation rounds to nearest and then moves each bound
 *     one unit in the last place outward, which contains the exact result
 *     because +, -, *, / are correctly rounded;
 *   - a step of length h from the box X first finds an a priori enclosure:
 *     a candidate box E with X + [0,h] f(E) contained in E.  Then every
 *     solution starting in X stays in B = X + [0,h] f(E) on [0,h] (Picard
 *     iteration maps E into itself), and x(h) lies in X + h f(B), intersected
 *     with B;
 *   - sin and cos of an interval come from the values at its ends, widened
 *     by a bound on the evaluation error, and from the extrema the interval
 *     contains.
 * Positions enter the dynamics only through their derivatives, so the
 * enclosure of a cell is that of the cell moved to the origin in (x1, x2),
 * shifted back by whole cells.  The table therefore has one entry per
 * (heading cell, speed cell, input): the cells met by the enclosure, as
 * ranges of cell indices (relative offsets on x1 and x2, absolute indices
 * on the heading, unwrapped, and on the speed).
 *
 * Everything is double precision with no contraction of multiply-adds
 * (built with -ffp-contract=off).
 */
#include <math.h>
#include <stdint.h>
#include <string.h>

typedef struct {
    double lo, hi;
} ac_iv;

/* One unit in the last place toward -inf / +inf (finite arguments). */
static double ac_down(double x) {
    uint64_t b;
    memcpy(&b, &x, 8);
    if ((b << 1) == 0) {
        b = 0x8000000000000001ull; /* -0 and +0 -> -smallest subnormal */
    } else if (b >> 63) {
        b += 1;
    } else {
        b -= 1;
    }
    memcpy(&x, &b, 8);
    return x;
}

static double ac_up(double x) { return -ac_down(-x); }

static ac_iv ac_pt(double c) {
    ac_iv r = {c, c};
    return r;
}

static ac_iv ac_add(ac_iv a, ac_iv b) {
    ac_iv r = {ac_down(a.lo + b.lo), ac_up(a.hi + b.hi)};
    return r;
}

static ac_iv ac_sub(ac_iv a, ac_iv b) {
    ac_iv r = {ac_down(a.lo - b.hi), ac_up(a.hi - b.lo)};
    return r;
}

static ac_iv ac_mul(ac_iv a, ac_iv b) {
    double p[4] = {a.lo * b.lo, a.lo * b.hi, a.hi * b.lo, a.hi * b.hi};
    double mn = p[0], mx = p[0];
    for (int i = 1; i < 4; ++i) {
        if (p[i] < mn) mn = p[i];
        if (p[i] > mx) mx = p[i];
    }
    ac_iv r = {ac_down(mn), ac_up(mx)};
    return r;
}

/* a * c and a / c for a positive double c */
static ac_iv ac_scale(ac_iv a, double c) {
    ac_iv r = {ac_down(a.lo * c), ac_up(a.hi * c)};
    return r;
}

static ac_iv ac_div(ac_iv a, double c) {
    ac_iv r = {ac_down(a.lo / c), ac_up(a.hi / c)};
    return r;
}

static ac_iv ac_sqr(ac_iv a) {
    ac_iv r;
    if (a.lo >= 0) {
        r.lo = ac_down(a.lo * a.lo);
        r.hi = ac_up(a.hi * a.hi);
    } else if (a.hi <= 0) {
        r.lo = ac_down(a.hi * a.hi);
        r.hi = ac_up(a.lo * a.lo);
    } else {
        double s = a.lo * a.lo, t = a.hi * a.hi;
        r.lo = 0.0;
        r.hi = ac_up(s > t ? s : t);
    }
    return r;
}

/* [0,h] * a for h > 0 */
static ac_iv ac_span(ac_iv a, double h) {
    double l = ac_down(a.lo * h), u = ac_up(a.hi * h);
    ac_iv r = {l < 0 ? l : 0.0, u > 0 ? u : 0.0};
    return r;
}

/* ---- sin and cos of a double, with an error bound ---------------------
 * Reduction x = k pi/2 + r with |r| <= about pi/4: pi/2 is split into a
 * 33-bit leading part (so that k * PIO2_A is exact for small k) and the
 * double nearest the rest; then the Taylor polynomials of sin and cos in r
 * to degree 17 and 18 (remainders below 1e-19 on |r| <= 0.8), in Horner
 * form.  The reduction and the about twenty roundings stay far below
 * AC_TRIG_ERR for the |x| < 16 that occur here. */
#define AC_PIO2_A 1.5707963267341256      /* 0x3ff921fb54400000 */
#define AC_PIO2_B 6.077100506506192e-11   /* 0x3dd0b4611a626331 */
#define AC_2_OVER_PI 0.6366197723675814
#define AC_PI_DN 3.141592653589793        /* the double just below pi */
#define AC_TRIG_ERR 1e-14

static double ac_sin_poly(double r) {
    double z = r * r;
    double p = 1.0 / 355687428096000.0;   /* 1/17! */
    p = -1.0 / 1307674368000.0 + z * p;   /* 1/15! */
    p = 1.0 / 6227020800.0 + z * p;       /* 1/13! */
    p = -1.0 / 39916800.0 + z * p;        /* 1/11! */
    p = 1.0 / 362880.0 + z * p;           /* 1/9! */
    p = -1.0 / 5040.0 + z * p;            /* 1/7! */
    p = 1.0 / 120.0 + z * p;              /* 1/5! */
    p = -1.0 / 6.0 + z * p;               /* 1/3! */
    return r + r * (z * p);
}

static double ac_cos_poly(double r) {
    double z = r * r;
    double p = 1.0 / 6402373705728000.0;  /* 1/18! */
    p = -1.0 / 20922789888000.0 + z * p;  /* 1/16! */
    p = 1.0 / 87178291200.0 + z * p;      /* 1/14! */
    p = -1.0 / 479001600.0 + z * p;       /* 1/12! */
    p = 1.0 / 3628800.0 + z * p;          /* 1/10! */
    p = -1.0 / 40320.0 + z * p;           /* 1/8! */
    p = 1.0 / 720.0 + z * p;              /* 1/6! */
    p = -1.0 / 24.0 + z * p;              /* 1/4! */
    p = 0.5 + z * p;                      /* 1/2! */
    return 1.0 - z * p;
}

/* q = 0: sin, q = 1: cos (sin(x + pi/2)) */
static double ac_trig(double x, int q) {
    double k = floor(x * AC_2_OVER_PI + 0.5);
    double r = (x - k * AC_PIO2_A) - k * AC_PIO2_B;
    int64_t quad = ((int64_t)k + q) & 3;
    switch (quad) {
        case 0: return ac_sin_poly(r);
        case 1: return ac_cos_poly(r);
        case 2: return -ac_sin_poly(r);
        default: return -ac_cos_poly(r);
    }
}

double oracle_ac_sin(double x) { return ac_trig(x, 0); }
double oracle_ac_cos(double x) { return ac_trig(x, 1); }

/* Does [a, b] contain c + 2 pi j for some integer j?  Checked with a margin
 * of 1e-9, so that a point near an end counts as inside (this only widens
 * the result). */
static int ac_hits(double a, double b, double c) {
    const double two_pi = 2.0 * AC_PI_DN;
    double j0 = floor((a - c) / two_pi) - 1.0;
    for (int t = 0; t < 4; ++t) {
        double p = c + (j0 + t) * two_pi;
        if (p >= a - 1e-9 && p <= b + 1e-9) return 1;
    }
    return 0;
}

/* q = 0: sin, q = 1: cos, of every point of a (width below pi) */
static ac_iv ac_trig_iv(ac_iv a, int q) {
    ac_iv r;
    if (!(a.hi - a.lo < 3.0)) {
        r.lo = -1.0;
        r.hi = 1.0;
        return r;
    }
    double fa = ac_trig(a.lo, q), fb = ac_trig(a.hi, q);
    double mn = fa < fb ? fa : fb, mx = fa < fb ? fb : fa;
    r.lo = ac_down(mn - AC_TRIG_ERR);
    r.hi = ac_up(mx + AC_TRIG_ERR);
    /* maxima of sin at pi/2, of cos at 0; minima half a turn away */
    double cmax = q == 0 ? 0.5 * AC_PI_DN : 0.0;
    if (ac_hits(a.lo, a.hi, cmax)) r.hi = 1.0;
    if (ac_hits(a.lo, a.hi, cmax - AC_PI_DN)) r.lo = -1.0;
    if (r.hi > 1.0) r.hi = 1.0;
    if (r.lo < -1.0) r.lo = -1.0;
    return r;
}

/* ---- the vector field over a box ------------------------------------- */
typedef struct {
    double u1;    /* thrust */
    ac_iv k3;     /* p_L sin(u2) / m */
    double mass;
    double p_D;
} ac_input;

static void ac_field(const ac_iv* x, const ac_input* in, ac_iv* f) {
    ac_iv c = ac_trig_iv(x[2], 1), s = ac_trig_iv(x[2], 0);
    f[0] = ac_mul(x[3], c);
    f[1] = ac_mul(x[3], s);
    f[2] = ac_mul(x[3], in->k3);
    f[3] = ac_div(ac_sub(ac_pt(in->u1), ac_scale(ac_sqr(x[3]), in->p_D)), in->mass);
}

/* One step of length h from X (4 intervals) in place; 0 = ok, -1 = no a
 * priori enclosure found. */
static int ac_step(ac_iv* X, const ac_input* in, double h) {
    ac_iv f[4], E[4], Et[4], B[4];
    ac_field(X, in, f);
    for (int a = 0; a < 4; ++a) E[a] = ac_add(X[a], ac_span(f[a], h));
    for (int it = 0; it < 12; ++it) {
        for (int a = 0; a < 4; ++a) {
            double d = (E[a].hi - E[a].lo) * 0.125 + 1e-10;
            Et[a].lo = E[a].lo - d;
            Et[a].hi = E[a].hi + d;
        }
        ac_field(Et, in, f);
        int inside = 1;
        for (int a = 0; a < 4; ++a) {
            B[a] = ac_add(X[a], ac_span(f[a], h));
            if (B[a].lo < Et[a].lo || B[a].hi > Et[a].hi) inside = 0;
        }
        if (inside) {
            ac_field(B, in, f);
            for (int a = 0; a < 4; ++a) {
                ac_iv y = ac_add(X[a], ac_scale(f[a], h));
                X[a].lo = y.lo > B[a].lo ? y.lo : B[a].lo;
                X[a].hi = y.hi < B[a].hi ? y.hi : B[a].hi;
            }
            return 0;
        }
        for (int a = 0; a < 4; ++a) E[a] = B[a];
    }
    return -1;
}

/* The input of index u: u1 = u / n_bank, u2 = u % n_bank on the vertices of
 * an even subdivision of [0, thrust_max] x [-bank_max, bank_max] (degrees).
 * Bank angle in radians: ((2 b - (n_bank - 1)) * bank_max_deg / (n_bank - 1))
 * * (pi / 180), evaluated in that order. */
static double ac_bank_rad(int b, int n_bank, double bank_max_deg) {
    if (n_bank == 1) return 0.0;
    double t = (double)(2 * b - (n_bank - 1)) * bank_max_deg;
    t = t / (double)(n_bank - 1);
    return t * (AC_PI_DN / 180.0);
}

static double ac_thrust(int a, int n_thrust, double thrust_max) {
    if (n_thrust == 1) return 0.0;
    return (double)a * thrust_max / (double)(n_thrust - 1);
}

double oracle_ac_bank_rad(int b, int n_bank, double bank_max_deg) { return ac_bank_rad(b, n_bank, bank_max_deg); }
double oracle_ac_thrust(int a, int n_thrust, double thrust_max) { return ac_thrust(a, n_thrust, thrust_max); }

/* Enclosure of the attainable set after `steps` steps of tau/steps from the
 * box lo/hi[4] under input (u1, u2), for the pins; 0 = ok. */
int oracle_ac_enclose(const double* lo, const double* hi, double u1, double u2, double mass, double p_D,
                      double p_L, double tau, int steps, double* out_lo, double* out_hi) {
    ac_input in;
    in.u1 = u1;
    in.mass = mass;
    in.p_D = p_D;
    double s2 = ac_trig(u2, 0);
    ac_iv sv = {ac_down(s2 - AC_TRIG_ERR), ac_up(s2 + AC_TRIG_ERR)};
    in.k3 = ac_div(ac_mul(sv, ac_pt(p_L)), mass);
    ac_iv X[4];
    for (int a = 0; a < 4; ++a) {
        X[a].lo = lo[a];
        X[a].hi = hi[a];
    }
    double h = tau / (double)steps;
    for (int s = 0; s < steps; ++s)
        if (ac_step(X, &in, h) != 0) return -1;
    for (int a = 0; a < 4; ++a) {
        out_lo[a] = X[a].lo;
        out_hi[a] = X[a].hi;
    }
    return 0;
}

/* Cells [j eta, (j+1) eta] (relative to the axis origin, eta an interval)
 * that meet [ylo, yhi]: j from ceil(ylo/eta - 1) to floor(yhi/eta), each
 * quotient bounded outward. */
static void ac_cells(double ylo, double yhi, ac_iv eta, int32_t* jlo, int32_t* jhi) {
    double q = ylo >= 0 ? ac_down(ylo / eta.hi) : ac_down(ylo / eta.lo);
    double p = yhi >= 0 ? ac_up(yhi / eta.lo) : ac_up(yhi / eta.hi);
    *jlo = (int32_t)ceil(ac_down(q - 1.0));
    *jhi = (int32_t)floor(p);
}

/* The table.  Grid: dims[0..3] cells on x1 in [0, x1_max], x2 in
 * [0, x2_max], heading in [-pi, pi] (periodic), speed in [v_lo, v_hi].
 * Entry (i3, i4, u), at index (i4 * dims[2] + i3) * K + u with K = n_thrust
 * * n_bank, holds 8 int32: o1lo, o1hi, o2lo, o2hi (cell offsets on x1, x2),
 * j3lo, j3hi (heading cells, unwrapped: reduce mod dims[2]), j4lo, j4hi
 * (speed cells; outside [0, dims[3]) means the set leaves the grid).
 * Returns the number of entries whose a priori enclosure failed (their
 * ranges are set to an empty range, lo > hi). */
int64_t oracle_ac_table(const int32_t* dims, double x1_max, double x2_max, double v_lo, double v_hi, double mass,
                        double p_D, double p_L, double tau, int32_t steps, int32_t n_thrust, int32_t n_bank,
                        double thrust_max, double bank_max_deg, int32_t* table) {
    const int K = n_thrust * n_bank;
    const ac_iv pi = {AC_PI_DN, ac_up(AC_PI_DN)};
    const ac_iv eta1 = ac_div(ac_pt(x1_max), (double)dims[0]);
    const ac_iv eta2 = ac_div(ac_pt(x2_max), (double)dims[1]);
    const ac_iv eta3 = ac_div(ac_scale(pi, 2.0), (double)dims[2]);
    const ac_iv eta4 = ac_div(ac_pt(v_hi - v_lo), (double)dims[3]);
    const ac_iv lo3 = {-pi.hi, -pi.lo};
    const double h = tau / (double)steps;
    int64_t failed = 0;
    for (int u = 0; u < K; ++u) {
        ac_input in;
        in.u1 = ac_thrust(u / n_bank, n_thrust, thrust_max);
        in.mass = mass;
        in.p_D = p_D;
        double s2 = ac_trig(ac_bank_rad(u % n_bank, n_bank, bank_max_deg), 0);
        ac_iv sv = {ac_down(s2 - AC_TRIG_ERR), ac_up(s2 + AC_TRIG_ERR)};
        in.k3 = ac_div(ac_mul(sv, ac_pt(p_L)), mass);
        for (int i4 = 0; i4 < dims[3]; ++i4) {
            for (int i3 = 0; i3 < dims[2]; ++i3) {
                ac_iv X[4];
                X[0].lo = 0.0;
                X[0].hi = eta1.hi;
                X[1].lo = 0.0;
                X[1].hi = eta2.hi;
                X[2].lo = ac_add(lo3, ac_scale(eta3, (double)i3)).lo;
                X[2].hi = ac_add(lo3, ac_scale(eta3, (double)(i3 + 1))).hi;
                X[3].lo = ac_add(ac_pt(v_lo), ac_scale(eta4, (double)i4)).lo;
                X[3].hi = ac_add(ac_pt(v_lo), ac_scale(eta4, (double)(i4 + 1))).hi;
                int32_t* e = table + ((int64_t)(i4 * dims[2] + i3) * K + u) * 8;
                int ok = 1;
                for (int s = 0; s < steps && ok; ++s) ok = ac_step(X, &in, h) == 0;
                if (!ok) {
                    ++failed;
                    for (int t = 0; t < 8; t += 2) {
                        e[t] = 1;
                        e[t + 1] = 0;
                    }
                    continue;
                }
                ac_cells(X[0].lo, X[0].hi, eta1, &e[0], &e[1]);
                ac_cells(X[1].lo, X[1].hi, eta2, &e[2], &e[3]);
                /* heading and speed: distances from the axis origin */
                ac_cells(ac_down(X[2].lo - lo3.hi), ac_up(X[2].hi - lo3.lo), eta3, &e[4], &e[5]);
                ac_cells(ac_down(X[3].lo - v_lo), ac_up(X[3].hi - v_lo), eta4, &e[6], &e[7]);
            }
        }
    }
    return failed;
}
