/*
 * lst_oracle.c -- plain, slow CPU oracle of the Line Segment Tracking object
 * chain (mini-doublets -> line segments -> T3 -> T5, pixel seeds -> pT3/pT5,
 * track-candidate selection), Sec. 1 of the paper.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the benchmark's CPU
 * baseline use it.  It shares no code with the GPU path: it derives its own
 * per-module and per-module-pair window constants from the module table.
 *
 * Structure (each stage is a plain loop nest over all candidates):
 *   MD : every (lower, upper) hit pair of a module               (Sec. 1, MD)
 *   LS : every MD pair whose modules lie on consecutive surfaces, or
 *        with the skip-layer flag also on surfaces two steps apart
 *        (brute force over all module pairs, no connection map)  (Sec. 1, LS)
 *   T3 : every LS pair sharing the middle MD                     (Sec. 1, T3)
 *   T5 : every T3 pair sharing an MD (outer of the first = inner
 *        of the second)                                          (Sec. 1, T5)
 *   pT3, pT5 : every (pixel seed, T3 / T5) pair                  (Sec. 1)
 *   TC : pT5s, pT3s, T5s and pixel seeds not used elsewhere      (Sec. 1 list)
 *   TC duplicate cleaning: every pair of candidates               (reading)
 *
 * The paper gives no cut values (it defers them to its references); the cut
 * catalogue implemented here is this project's own, derived from prompt-helix
 * geometry with a pT threshold (Sec. 1: 0.8 GeV).  Each cut decision is taken
 * in IEEE binary32 with a fixed expression order (the precision of the device
 * kernels); the pixel-seed cuts, which need asin/atan2/sin, decide in
 * binary64.  Window constants are computed in binary64 and rounded once.
 *
 * Borderline bookkeeping: every cut is a test "v <= t".  A candidate whose
 * |t - v| <= flag_margin * |t| on any cut is *flagged*; flagged candidates
 * are kept even when they fail (status bit 1 set, bit 0 = accepted) so that
 * their descendants are known too.  Flags propagate to descendants.
 *
 * Build: gcc -O2 -std=c11 -ffp-contract=off -fno-fast-math -shared -fPIC
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_BARREL 0u
#define OR_ENDCAP 1u
#define OR_PI 3.14159265358979323846

/* ---------------------------------------------------------------- types -- */

typedef struct {
    uint32_t n_mod;
    const uint32_t *kind;   /* 0 barrel, 1 endcap */
    const uint32_t *layer;  /* barrel layer or disk index, ordered outward */
    const int32_t *side;    /* 0 barrel, +1/-1 endcap */
    const double *s_lo, *s_hi;   /* sensor radius (barrel) / signed plane z */
    const double *c_min, *c_max; /* z extent (barrel) / r extent (endcap) */
    const double *phi_min, *phi_max;
} or_geom;

typedef struct {
    double B;           /* field [T] */
    double pt_min;      /* pT threshold [GeV] */
    double L;           /* half-width of the luminous region along z [cm] */
    double sig_rphi;    /* hit resolution along r-phi [cm] */
    double sig_c;       /* coarse resolution: z (barrel) / r (endcap) [cm] */
    double n_sigma;
    double flag_margin; /* relative margin for borderline candidates */
    uint32_t flags;     /* bit 0: line-segment bend-consistency cut;
                           bit 1: skip-layer links (a segment may bridge one surface) */
} or_params;

typedef struct {
    uint32_t n_hits;
    const float *x, *y, *z;
    const uint32_t *module;
    const uint8_t *sensor;
    uint32_t n_pls;
    const float *pls_par; /* 5 per seed: q/pT, phi0, cot(theta), d0, z0 */
    const float *pls_cov; /* 15 per seed: upper triangle, row major */
} or_event;

typedef struct {
    uint32_t n_md;  uint32_t *md;  uint8_t *md_st;  /* hit_lo, hit_up (input indices) */
    uint32_t n_ls;  uint32_t *ls;  uint8_t *ls_st;  /* md_in, md_out */
    uint32_t n_t3;  uint32_t *t3;  uint8_t *t3_st;  /* ls_in, ls_out */
    float *t3_k, *t3_sk;
    uint32_t n_t5;  uint32_t *t5;  uint8_t *t5_st;  /* t3_in, t3_out */
    uint32_t n_pt3; uint32_t *pt3; uint8_t *pt3_st; /* pls, t3 */
    uint32_t n_pt5; uint32_t *pt5; uint8_t *pt5_st; /* pls, t5 */
    uint32_t n_tc;  uint32_t *tc;  uint8_t *tc_st;  /* type, index */
    uint32_t md_cand, ls_cand, t3_cand, t5_cand, pt3_cand, pt5_cand;
    float *t5_k, *t5_sk;    /* curvature through the outer anchors A, C, E of each T5 and its resolution */
    uint8_t *tc_keep;       /* per track candidate: 1 = kept by the duplicate cleaning */
} or_result;

#define ST_ACC 1u
#define ST_FLAG 2u

/* ------------------------------------------------------- growable lists -- */

typedef struct { uint32_t *v; uint8_t *st; float *f0, *f1; size_t n, cap; int has_f; } olist;

static void ol_push(olist *l, uint32_t a, uint32_t b, uint8_t st, float f0, float f1)
{
    if (l->n == l->cap) {
        size_t nc = l->cap ? 2 * l->cap : 1024;
        l->v = (uint32_t *)realloc(l->v, 2 * nc * sizeof(uint32_t));
        l->st = (uint8_t *)realloc(l->st, nc);
        if (l->has_f) {
            l->f0 = (float *)realloc(l->f0, nc * sizeof(float));
            l->f1 = (float *)realloc(l->f1, nc * sizeof(float));
        }
        l->cap = nc;
    }
    l->v[2 * l->n] = a;
    l->v[2 * l->n + 1] = b;
    l->st[l->n] = st;
    if (l->has_f) { l->f0[l->n] = f0; l->f1[l->n] = f1; }
    l->n++;
}

/* --------------------------------------------------- cut bookkeeping ---- */

typedef struct { int hard; int fail; int border; double fm; } verdict;

/* binary32 test v <= t */
static void chk(verdict *s, float v, float t)
{
    int ok = v <= t;
    int b = fabs((double)t - (double)v) <= s->fm * fabs((double)t);
    if (!ok) { s->fail = 1; if (!b) s->hard = 1; }
    if (b) s->border = 1;
}

/* binary64 test v <= t */
static void chkd(verdict *s, double v, double t)
{
    int ok = v <= t;
    int b = fabs(t - v) <= s->fm * fabs(t);
    if (!ok) { s->fail = 1; if (!b) s->hard = 1; }
    if (b) s->border = 1;
}

static uint8_t status_of(const verdict *s)
{
    return (uint8_t)((s->fail ? 0u : ST_ACC) | (s->border ? ST_FLAG : 0u));
}

/* combine a candidate's own verdict with its constituents' status */
static uint8_t combine(uint8_t own, uint8_t c1, uint8_t c2)
{
    uint8_t acc = (uint8_t)(own & c1 & c2 & ST_ACC);
    uint8_t fl = (uint8_t)((own | c1 | c2) & ST_FLAG);
    return (uint8_t)(acc | fl);
}

/* ---------------------------------------------------- window geometry ---- */
/* All in binary64.  kappa_max = 0.299792458e-2 * B / pT_min  [1/cm].       */

typedef struct {
    double kmax;
    /* binary32 copies used by the cuts */
    float L, ec, kmaxf, khalf, ns, srp, sc, Kb;
} derived;

/* A(r): half the turning angle of a kappa_max helix at radius r */
static double turn(double r, double k) { double x = r * k / 2.0; if (x > 1.0) x = 1.0; return asin(x); }
/* f(x) = asin(x)/x, the arc/chord ratio of a circle */
static double arcf(double x) { return x == 0.0 ? 1.0 : asin(x) / x; }

static void derive(const or_geom *g, const or_params *p, derived *d)
{
    double rmax = 0.0;
    for (uint32_t m = 0; m < g->n_mod; m++) {
        double r = g->kind[m] == OR_BARREL ? g->s_lo[m] : g->c_max[m];
        if (r > rmax) rmax = r;
    }
    d->kmax = 0.299792458e-2 * p->B / p->pt_min;
    d->L = (float)p->L;
    d->ec = (float)(p->n_sigma * p->sig_c);
    d->kmaxf = (float)d->kmax;
    d->khalf = (float)(d->kmax / 2.0);
    d->ns = (float)p->n_sigma;
    d->srp = (float)p->sig_rphi;
    d->sc = (float)p->sig_c;
    /* arc-vs-chord bias bound: |f(x1) - f(x2)| <= |x1^2 - x2^2| f'(xm)/(2 xm)
       for chords up to the outermost anchor radius, x = chord * kappa / 2 */
    double xm = rmax * d->kmax / 2.0;
    if (xm > 0.999) xm = 0.999;
    double fp = (xm / sqrt(1.0 - xm * xm) - asin(xm)) / (xm * xm);
    d->Kb = (float)(fp / (2.0 * xm) * d->kmax * d->kmax / 4.0);
}

/* per-module mini-doublet constants */
typedef struct { float S, G, K, D; } mdconst;

static mdconst module_const(const or_geom *g, const or_params *p, const derived *d, uint32_t m)
{
    mdconst c = {0, 0, 0, 0};
    double k = d->kmax, ns = p->n_sigma, rt2 = sqrt(2.0);
    if (g->kind[m] == OR_BARREL) {
        double r1 = g->s_lo[m], r2 = g->s_hi[m];
        double ph = turn(r2, k) - turn(r1, k) + ns * rt2 * p->sig_rphi / r1;
        c.S = (float)sin(fmin(ph, OR_PI / 2));
        c.G = (float)((r2 - r1) / cos(turn(r2, k)));
        c.K = (float)(ns * rt2 * p->sig_c);
    } else {
        double z1 = fabs(g->s_lo[m]), gap = fabs(g->s_hi[m]) - fabs(g->s_lo[m]);
        double rin = g->c_min[m], rout = g->c_max[m];
        double dr = gap * rout / (z1 - p->L);
        double ph = turn(rout + dr, k) - turn(rout, k) + ns * rt2 * p->sig_rphi / rin;
        c.S = (float)sin(fmin(ph, OR_PI / 2));
        c.D = (float)(dr + ns * rt2 * p->sig_c);
    }
    return c;
}

/* per-module-pair line-segment constants */
typedef struct {
    int type;           /* 0 barrel->barrel, 1 endcap->endcap, 2 barrel->endcap */
    float S;
    float rho_lo, rho_hi, lam_lo, lam_hi, tau;  /* BB */
    float lo_fac, hi_fac;                       /* EE */
    float cf, zs, zbpl, zbml;                   /* BE */
} lsconst;

static lsconst pair_const(const or_geom *g, const or_params *p, const derived *d, uint32_t A, uint32_t B)
{
    lsconst c;
    memset(&c, 0, sizeof c);
    double k = d->kmax, ns = p->n_sigma, rt2 = sqrt(2.0);
    int bA = g->kind[A] == OR_BARREL, bB = g->kind[B] == OR_BARREL;
    double a_lo = bA ? g->s_lo[A] : g->c_min[A];
    double b_hi = bB ? g->s_lo[B] : g->c_max[B];
    double ph = turn(b_hi, k) - turn(a_lo, k) + ns * rt2 * p->sig_rphi / a_lo;
    c.S = (float)sin(fmin(ph, OR_PI / 2));
    if (bA && bB) {
        double a = g->s_lo[A], b = g->s_lo[B], gA = g->s_hi[A] - g->s_lo[A];
        c.type = 0;
        c.rho_lo = (float)(b / a);
        c.rho_hi = (float)(turn(b, k) / turn(a, k));
        double llo = (b - a) / gA;
        double lhi = sin(turn(b, k) - turn(a, k)) / sin(turn(g->s_hi[A], k) - turn(a, k));
        c.lam_lo = (float)llo;
        c.lam_hi = (float)lhi;
        c.tau = (float)(ns * rt2 * p->sig_rphi * (1.0 + fmax(llo, lhi)) / a);
    } else if (!bA && !bB) {
        double zA = fabs(g->s_lo[A]), zB = fabs(g->s_lo[B]);
        double tlo = (zB + p->L) / (zA + p->L), thi = (zB - p->L) / (zA - p->L);
        double cf = 1.0 / arcf(b_hi * k / 2.0);
        c.type = 1;
        c.lo_fac = (float)(cf * tlo);
        c.hi_fac = (float)thi;
    } else {
        double zB = fabs(g->s_lo[B]);
        c.type = 2;
        c.cf = (float)(1.0 / arcf(b_hi * k / 2.0));
        c.zs = g->s_lo[B] > 0 ? 1.0f : -1.0f;
        c.zbpl = (float)(zB + p->L);
        c.zbml = (float)(zB - p->L);
    }
    return c;
}

/* ------------------------------------------------------------ surfaces -- */

typedef struct { uint32_t nb, nd; } surfinfo;

static surfinfo surf_info(const or_geom *g)
{
    surfinfo s = {0, 0};
    for (uint32_t m = 0; m < g->n_mod; m++) {
        if (g->kind[m] == OR_BARREL) { if (g->layer[m] + 1 > s.nb) s.nb = g->layer[m] + 1; }
        else if (g->layer[m] + 1 > s.nd) s.nd = g->layer[m] + 1;
    }
    return s;
}

static uint32_t surface_of(const or_geom *g, surfinfo si, uint32_t m)
{
    if (g->kind[m] == OR_BARREL) return g->layer[m];
    return si.nb + (g->side[m] > 0 ? 0 : si.nd) + g->layer[m];
}

/* is surface t the next surface an outgoing prompt track can reach from s */
static int is_next(surfinfo si, uint32_t s, uint32_t t)
{
    if (s < si.nb) {
        if (t == s + 1 && t < si.nb) return 1;
        if (si.nd && (t == si.nb || t == si.nb + si.nd)) return 1;
        return 0;
    }
    uint32_t d = (s - si.nb) % si.nd;
    return d + 1 < si.nd && t == s + 1;
}

/* Surfaces whose modules a segment may join: the next ones, and with skip
   also the next surfaces of those (a track that left no mini-doublet on the
   surface in between is still linked; the paper's connection maps hold the
   module pairs a charged particle can cross in turn, Sec. 1). */
static int is_linked(surfinfo si, uint32_t s, uint32_t t, int skip)
{
    if (is_next(si, s, t)) return 1;
    if (!skip) return 0;
    for (uint32_t u = 0; u < si.nb + 2 * si.nd; u++)
        if (is_next(si, s, u) && is_next(si, u, t)) return 1;
    return 0;
}

/* ---------------------------------------------------------- the cuts ---- */

/* Mini-doublet: lower hit i, upper hit j on module m. */
static verdict md_cut(const or_geom *g, const derived *d, const mdconst *mc, uint32_t m,
                      float xi, float yi, float zi, float ri,
                      float xj, float yj, float zj, float rj, double fm, float *beta)
{
    verdict s = {0, 0, 0, fm};
    float dx = xj - xi, dy = yj - yi;
    float c = xi * dy - yi * dx;
    float dd = xi * xj + yi * yj;
    float rr = ri * rj;
    if (!(dd > 0.0f)) { s.hard = 1; return s; }
    chk(&s, fabsf(c), mc->S * rr);
    if (g->kind[m] == OR_BARREL)
        chk(&s, fabsf(zj - zi) * ri, mc->G * (fabsf(zi) + d->L) + mc->K * ri);
    else
        chk(&s, fabsf(rj - ri), mc->D);
    *beta = c / rr;
    return s;
}

/* Line segment between the anchors (lower hits) of MDs a and b. */
static verdict ls_cut(const derived *d, const lsconst *k, int bend,
                      float xa, float ya, float za, float ra, float beta_a,
                      float xb, float yb, float zb, float rb, double fm)
{
    verdict s = {0, 0, 0, fm};
    float dx = xb - xa, dy = yb - ya;
    float c = xa * dy - ya * dx;
    float dd = xa * xb + ya * yb;
    float rr = ra * rb;
    if (!(dd > 0.0f)) { s.hard = 1; return s; }
    chk(&s, fabsf(c), k->S * rr);
    if (s.hard) return s;
    if (k->type == 0) {
        /* z_b = rho (z_a - v) + v over rho in [rho_lo, rho_hi], v in [-L, L],
           z_a within its resolution: extremes at the corners */
        float rho[2] = {k->rho_lo, k->rho_hi};
        float vv[2] = {-d->L, d->L};
        float zp[2] = {za - d->ec, za + d->ec};
        float lo = 0.0f, hi = 0.0f;
        int first = 1;
        for (int i = 0; i < 2; i++)
            for (int j = 0; j < 2; j++)
                for (int l = 0; l < 2; l++) {
                    float w = rho[i] * (zp[l] - vv[j]) + vv[j];
                    if (first) { lo = w; hi = w; first = 0; }
                    else { lo = fminf(lo, w); hi = fmaxf(hi, w); }
                }
        float mid = 0.5f * (lo + hi), half = 0.5f * (hi - lo) + d->ec;
        chk(&s, fabsf(zb - mid), half);
        if (bend && !s.hard) {
            float sab = c / rr;
            float p1 = k->lam_lo * beta_a, p2 = k->lam_hi * beta_a;
            float blo = fminf(p1, p2) - k->tau, bhi = fmaxf(p1, p2) + k->tau;
            float bmid = 0.5f * (blo + bhi), bhalf = 0.5f * (bhi - blo);
            chk(&s, fabsf(sab - bmid), bhalf);
        }
    } else if (k->type == 1) {
        float lo = k->lo_fac * (ra - d->ec) - d->ec;
        float hi = k->hi_fac * (ra + d->ec) + d->ec;
        float mid = 0.5f * (lo + hi), half = 0.5f * (hi - lo);
        chk(&s, fabsf(rb - mid), half);
    } else {
        float zap = k->zs * za;
        float dhi = (zap + d->ec) + d->L;
        if (!(dhi > 0.0f)) { s.hard = 1; return s; }
        float lo = (k->cf * (k->zbpl / dhi)) * ra - d->ec;
        float dlo = (zap - d->ec) - d->L;
        if (dlo > 0.0f) {
            float hi = (k->zbml / dlo) * ra + d->ec;
            float mid = 0.5f * (lo + hi), half = 0.5f * (hi - lo);
            chk(&s, fabsf(rb - mid), half);
        } else {
            chk(&s, lo, rb);
        }
    }
    return s;
}

/* Curvature of the circle through three transverse points, and its
   resolution.  k* = 1 for an anchor on a disk.  Sign: positive for a
   clockwise turn (positive charge in a field along +z). */
static void kappa3(const derived *d,
                   float xA, float yA, int kA, float xB, float yB, int kB,
                   float xC, float yC, float rC, int kC,
                   float *kap, float *sk, float *d1o, float *d2o)
{
    float dx1 = xB - xA, dy1 = yB - yA;
    float dx2 = xC - xB, dy2 = yC - yB;
    float dx3 = xC - xA, dy3 = yC - yA;
    float cr = dx1 * dy2 - dy1 * dx2;
    float d1 = sqrtf(dx1 * dx1 + dy1 * dy1);
    float d2 = sqrtf(dx2 * dx2 + dy2 * dy2);
    float d3 = sqrtf(dx3 * dx3 + dy3 * dy3);
    *kap = (-2.0f * cr) / ((d1 * d2) * d3);
    float hC = fminf(1.0f, rC * d->khalf);
    float sdisk = d->srp + d->sc * hC;
    float sA = kA ? sdisk : d->srp;
    float sB = kB ? sdisk : d->srp;
    float sC = kC ? sdisk : d->srp;
    *sk = (2.0f * sqrtf((sA * sA + sB * sB) + sC * sC)) / (d1 * d2);
    *d1o = d1;
    *d2o = d2;
}

/* straight-line consistency in (arc length, z) of three anchors */
static void rz3(verdict *s, const derived *d,
                float zA, int kA, float zB, int kB, float zC, int kC, float d1, float d2)
{
    float E = (zB - zA) * d2 - (zC - zB) * d1;
    float szA = kA ? 0.0f : d->sc, szB = kB ? 0.0f : d->sc, szC = kC ? 0.0f : d->sc;
    float stA = kA ? d->sc : d->srp, stB = kB ? d->sc : d->srp, stC = kC ? d->sc : d->srp;
    float res = (((szA * d2 + szB * (d1 + d2)) + szC * d1)
                 + fabsf(zB - zA) * (stB + stC)) + fabsf(zC - zB) * (stA + stB);
    float bias = ((d->Kb * (fabsf(zC - zA) / (d1 + d2))) * (d1 * d2)) * fabsf(d1 * d1 - d2 * d2);
    chk(s, fabsf(E), d->ns * res + bias);
}

typedef struct { float x, y, z, r; int disk; } anchor;

static verdict t3_cut(const derived *d, const anchor *A, const anchor *B, const anchor *C,
                      double fm, float *kap, float *sk)
{
    verdict s = {0, 0, 0, fm};
    float d1, d2;
    kappa3(d, A->x, A->y, A->disk, B->x, B->y, B->disk, C->x, C->y, C->r, C->disk, kap, sk, &d1, &d2);
    chk(&s, fabsf(*kap), d->kmaxf + d->ns * *sk);
    if (s.hard) return s;
    rz3(&s, d, A->z, A->disk, B->z, B->disk, C->z, C->disk, d1, d2);
    return s;
}

static verdict t5_cut(const derived *d, const anchor *A, const anchor *C, const anchor *E,
                      float k1, float sk1, float k2, float sk2, double fm, float *k3o, float *sk3o)
{
    verdict s = {0, 0, 0, fm};
    float k3, sk3, d1, d2;
    kappa3(d, A->x, A->y, A->disk, C->x, C->y, C->disk, E->x, E->y, E->r, E->disk, &k3, &sk3, &d1, &d2);
    *k3o = k3;
    *sk3o = sk3;
    chk(&s, fabsf(k1 - k2), d->ns * (sk1 + sk2));
    chk(&s, fabsf(k1 - k3), d->ns * (sk1 + sk3));
    chk(&s, fabsf(k2 - k3), d->ns * (sk2 + sk3));
    if (s.hard) return s;
    rz3(&s, d, A->z, A->disk, C->z, C->disk, E->z, E->disk, d1, d2);
    return s;
}

/* One anchor of a pixel seed (binary64): the azimuth difference between the
   anchor and the seed's helix at the anchor's radius, its window, and the
   deviation along the coarse coordinate (z at a barrel anchor, r at a disk
   anchor) with its window.  Returns 0 when both tests can be evaluated, 1
   when the helix does not reach the anchor's radius (|r kappa / 2| >= 1), 2
   when the disk prediction is undefined (cot(theta) = 0, plane behind the
   seed, or a turning angle of pi or more). */
static int p_anchor(const or_params *pp, double kp, double skp, const float *par, const float *cov,
                    const anchor *a, double out[4])
{
    double ns = pp->n_sigma;
    double phi0 = par[1], cot = par[2], z0 = par[4];
    double s11 = sqrt((double)cov[5]), s22 = sqrt((double)cov[9]), s44 = sqrt((double)cov[14]);
    double x = a->x, y = a->y, z = a->z;
    double r = sqrt(x * x + y * y);
    double u = r * kp / 2.0;
    if (!(fabs(u) < 1.0)) return 1;
    /* azimuth of the helix at radius r: phi0 minus half the turning angle */
    double dphi = atan2(y, x) - (phi0 - asin(u));
    dphi = fmod(dphi + OR_PI, 2.0 * OR_PI);
    if (dphi < 0.0) dphi += 2.0 * OR_PI;
    dphi -= OR_PI;
    double sr = a->disk ? pp->sig_c : 0.0;
    out[0] = dphi;
    out[1] = ns * (s11 + (r * skp + sr * fabs(kp)) / (2.0 * sqrt(1.0 - u * u)) + pp->sig_rphi / r);
    if (!a->disk) {
        /* z after the transverse arc length s(r) */
        double sa = (u == 0.0) ? r : r * asin(u) / u;
        double zp = z0 + cot * sa;
        out[2] = z - zp;
        out[3] = ns * (s44 + sa * s22 + pp->sig_c);
        return 0;
    }
    /* radius where the helix crosses the anchor's plane */
    if (cot == 0.0) return 2;
    double sa = (z - z0) / cot;
    if (!(sa > 0.0)) return 2;
    double w = fabs(kp) * sa / 2.0;
    if (!(w < OR_PI / 2)) return 2;
    double rp = (w == 0.0) ? sa : sa * sin(w) / w;
    out[2] = r - rp;
    out[3] = ns * ((s44 + sa * s22) / fabs(cot) + pp->sig_c);
    return 0;
}

/* pixel seed p against an object with curvature kobj (+/- skobj) and inner /
   outer anchors; binary64 throughout */
static verdict p_cut(const or_params *pp, const float *par, const float *cov,
                     float kobj, float skobj, const anchor *in, const anchor *out, double fm)
{
    verdict s = {0, 0, 0, fm};
    double kB = 0.299792458e-2 * pp->B, ns = pp->n_sigma;
    double kp = (double)par[0] * kB;
    double skp = kB * sqrt((double)cov[0]);
    chkd(&s, fabs(kp - (double)kobj), ns * (skp + (double)skobj));
    if (s.hard) return s;
    const anchor *an[2] = {in, out};
    for (int i = 0; i < 2; i++) {
        double v[4];
        int code = p_anchor(pp, kp, skp, par, cov, an[i], v);
        if (code == 1) { s.hard = 1; return s; }
        chkd(&s, fabs(v[0]), v[1]);
        if (s.hard) return s;
        if (code == 2) { s.hard = 1; return s; }
        chkd(&s, fabs(v[2]), v[3]);
        if (s.hard) return s;
    }
    return s;
}

/* ------------------------------------------------------------ the run ---- */

static uint32_t *csr_by(const uint32_t *keys, size_t stride, size_t n, uint32_t nkeys, uint32_t **items)
{
    uint32_t *off = (uint32_t *)calloc((size_t)nkeys + 1, sizeof(uint32_t));
    for (size_t i = 0; i < n; i++) off[keys[i * stride] + 1]++;
    for (uint32_t k = 0; k < nkeys; k++) off[k + 1] += off[k];
    uint32_t *pos = (uint32_t *)malloc(((size_t)nkeys + 1) * sizeof(uint32_t));
    memcpy(pos, off, ((size_t)nkeys + 1) * sizeof(uint32_t));
    *items = (uint32_t *)malloc((n ? n : 1) * sizeof(uint32_t));
    for (size_t i = 0; i < n; i++) (*items)[pos[keys[i * stride]]++] = (uint32_t)i;
    free(pos);
    return off;
}

int or_run(const or_geom *g, const or_params *p, const or_event *ev, or_result *out)
{
    memset(out, 0, sizeof *out);
    derived d;
    derive(g, p, &d);
    double fm = p->flag_margin;
    int bend = (int)(p->flags & 1u);
    int skip = (int)((p->flags >> 1) & 1u);
    surfinfo si = surf_info(g);
    uint32_t nsurf = si.nb + 2 * si.nd;
    uint32_t nh = ev->n_hits;

    for (uint32_t h = 0; h < nh; h++) {
        if (ev->module[h] >= g->n_mod || ev->sensor[h] > 1) return -1;
        if (!isfinite(ev->x[h]) || !isfinite(ev->y[h]) || !isfinite(ev->z[h])) return -2;
    }

    float *hr = (float *)malloc((nh ? nh : 1) * sizeof(float));
    for (uint32_t h = 0; h < nh; h++) hr[h] = sqrtf(ev->x[h] * ev->x[h] + ev->y[h] * ev->y[h]);

    /* hits of each (module, sensor), in input order */
    uint32_t *key = (uint32_t *)malloc((nh ? nh : 1) * sizeof(uint32_t));
    for (uint32_t h = 0; h < nh; h++) key[h] = 2 * ev->module[h] + ev->sensor[h];
    uint32_t *hit_items;
    uint32_t *hit_off = csr_by(key, 1, nh, 2 * g->n_mod, &hit_items);

    /* ---- MD ---- */
    olist md = {0};
    olist mdx = {0}; mdx.has_f = 1;   /* anchor x,y */
    olist mdz = {0}; mdz.has_f = 1;   /* anchor z,r */
    olist mdb = {0}; mdb.has_f = 1;   /* beta, unused */
    uint32_t *md_mod_v = NULL; size_t md_mod_cap = 0;
    for (uint32_t m = 0; m < g->n_mod; m++) {
        mdconst mc = module_const(g, p, &d, m);
        for (uint32_t a = hit_off[2 * m]; a < hit_off[2 * m + 1]; a++) {
            uint32_t i = hit_items[a];
            for (uint32_t b = hit_off[2 * m + 1]; b < hit_off[2 * m + 2]; b++) {
                uint32_t j = hit_items[b];
                float beta = 0.0f;
                out->md_cand++;
                verdict s = md_cut(g, &d, &mc, m, ev->x[i], ev->y[i], ev->z[i], hr[i],
                                   ev->x[j], ev->y[j], ev->z[j], hr[j], fm, &beta);
                if (s.hard) continue;
                ol_push(&md, i, j, status_of(&s), 0, 0);
                ol_push(&mdx, 0, 0, 0, ev->x[i], ev->y[i]);
                ol_push(&mdz, 0, 0, 0, ev->z[i], hr[i]);
                ol_push(&mdb, 0, 0, 0, beta, 0);
                if (md.n > md_mod_cap) {
                    md_mod_cap = md.cap;
                    md_mod_v = (uint32_t *)realloc(md_mod_v, md_mod_cap * sizeof(uint32_t));
                }
                md_mod_v[md.n - 1] = m;
            }
        }
    }
    uint32_t nmd = (uint32_t)md.n;
    anchor *anc = (anchor *)malloc((nmd ? nmd : 1) * sizeof(anchor));
    for (uint32_t a = 0; a < nmd; a++) {
        anc[a].x = mdx.f0[a]; anc[a].y = mdx.f1[a];
        anc[a].z = mdz.f0[a]; anc[a].r = mdz.f1[a];
        anc[a].disk = g->kind[md_mod_v[a]] == OR_ENDCAP;
    }

    /* ---- LS: all MD pairs on linked surfaces ---- */
    uint32_t *md_surf = (uint32_t *)malloc((nmd ? nmd : 1) * sizeof(uint32_t));
    for (uint32_t a = 0; a < nmd; a++) md_surf[a] = surface_of(g, si, md_mod_v[a]);
    uint32_t *surf_items;
    uint32_t *surf_off = csr_by(md_surf, 1, nmd, nsurf ? nsurf : 1, &surf_items);
    olist ls = {0};
    for (uint32_t a = 0; a < nmd; a++) {
        uint32_t sa = md_surf[a], A = md_mod_v[a];
        for (uint32_t t = 0; t < nsurf; t++) {
            if (!is_linked(si, sa, t, skip)) continue;
            uint32_t lastB = UINT32_MAX;
            lsconst kc;
            memset(&kc, 0, sizeof kc);
            for (uint32_t q = surf_off[t]; q < surf_off[t + 1]; q++) {
                uint32_t b = surf_items[q], B = md_mod_v[b];
                if (B != lastB) { kc = pair_const(g, p, &d, A, B); lastB = B; }
                out->ls_cand++;
                verdict s = ls_cut(&d, &kc, bend, anc[a].x, anc[a].y, anc[a].z, anc[a].r,
                                   mdb.f0[a], anc[b].x, anc[b].y, anc[b].z, anc[b].r, fm);
                if (s.hard) continue;
                ol_push(&ls, a, b, combine(status_of(&s), md.st[a], md.st[b]), 0, 0);
            }
        }
    }
    uint32_t nls = (uint32_t)ls.n;

    /* ---- T3: LS pairs sharing the middle MD ---- */
    uint32_t *ls_items;
    uint32_t *ls_off = csr_by(ls.v, 2, nls, nmd ? nmd : 1, &ls_items); /* by md_in */
    olist t3 = {0}; t3.has_f = 1;
    olist t3m = {0}; /* (md_a, md_c) of each T3 */
    for (uint32_t l1 = 0; l1 < nls; l1++) {
        uint32_t a = ls.v[2 * l1], b = ls.v[2 * l1 + 1];
        for (uint32_t q = ls_off[b]; q < ls_off[b + 1]; q++) {
            uint32_t l2 = ls_items[q];
            uint32_t c = ls.v[2 * l2 + 1];
            float kap, sk;
            out->t3_cand++;
            verdict s = t3_cut(&d, &anc[a], &anc[b], &anc[c], fm, &kap, &sk);
            if (s.hard) continue;
            ol_push(&t3, l1, l2, combine(status_of(&s), ls.st[l1], ls.st[l2]), kap, sk);
            ol_push(&t3m, a, c, 0, 0, 0);
        }
    }
    uint32_t nt3 = (uint32_t)t3.n;

    /* ---- T5: T3 pairs sharing an MD ---- */
    uint32_t *t3_items;
    uint32_t *t3_off = csr_by(t3m.v, 2, nt3, nmd ? nmd : 1, &t3_items); /* by inner MD */
    olist t5 = {0}; t5.has_f = 1;  /* curvature (and resolution) through A, C, E */
    for (uint32_t u = 0; u < nt3; u++) {
        uint32_t a = t3m.v[2 * u], c = t3m.v[2 * u + 1];
        for (uint32_t q = t3_off[c]; q < t3_off[c + 1]; q++) {
            uint32_t w = t3_items[q];
            uint32_t e = t3m.v[2 * w + 1];
            float k3, sk3;
            out->t5_cand++;
            verdict s = t5_cut(&d, &anc[a], &anc[c], &anc[e], t3.f0[u], t3.f1[u], t3.f0[w], t3.f1[w],
                               fm, &k3, &sk3);
            if (s.hard) continue;
            ol_push(&t5, u, w, combine(status_of(&s), t3.st[u], t3.st[w]), k3, sk3);
        }
    }
    uint32_t nt5 = (uint32_t)t5.n;

    /* ---- pT3 / pT5: every (seed, object) pair ---- */
    olist pt3 = {0}, pt5 = {0};
    for (uint32_t ps = 0; ps < ev->n_pls; ps++) {
        const float *par = ev->pls_par + 5 * (size_t)ps;
        const float *cov = ev->pls_cov + 15 * (size_t)ps;
        for (uint32_t u = 0; u < nt3; u++) {
            out->pt3_cand++;
            verdict s = p_cut(p, par, cov, t3.f0[u], t3.f1[u], &anc[t3m.v[2 * u]], &anc[t3m.v[2 * u + 1]], fm);
            if (s.hard) continue;
            ol_push(&pt3, ps, u, combine(status_of(&s), t3.st[u], ST_ACC), 0, 0);
        }
        for (uint32_t v = 0; v < nt5; v++) {
            uint32_t u = t5.v[2 * v], w = t5.v[2 * v + 1];
            uint32_t a = t3m.v[2 * u], e = t3m.v[2 * w + 1];
            out->pt5_cand++;
            verdict s = p_cut(p, par, cov, t5.f0[v], t5.f1[v], &anc[a], &anc[e], fm);
            if (s.hard) continue;
            ol_push(&pt5, ps, v, combine(status_of(&s), t5.st[v], ST_ACC), 0, 0);
        }
    }

    /* ---- track candidates ---- */
    /* per seed / T5: 2 = used by a certain (accepted, unflagged) object,
       1 = used only by uncertain (flagged) objects, 0 = unused */
    uint32_t np = ev->n_pls;
    uint8_t *pls_pt5 = (uint8_t *)calloc(np ? np : 1, 1);
    uint8_t *pls_pt3 = (uint8_t *)calloc(np ? np : 1, 1);
    uint8_t *t5_pt5 = (uint8_t *)calloc(nt5 ? nt5 : 1, 1);
#define USE(arr, i, st) do { uint8_t u_ = ((st) == ST_ACC) ? 2 : 1; if (u_ > (arr)[i]) (arr)[i] = u_; } while (0)
    for (size_t i = 0; i < pt5.n; i++) { USE(pls_pt5, pt5.v[2 * i], pt5.st[i]); USE(t5_pt5, pt5.v[2 * i + 1], pt5.st[i]); }
    for (size_t i = 0; i < pt3.n; i++) USE(pls_pt3, pt3.v[2 * i], pt3.st[i]);
#undef USE
    olist tc = {0};
    for (size_t i = 0; i < pt5.n; i++) ol_push(&tc, 0, (uint32_t)i, pt5.st[i], 0, 0);
    for (size_t i = 0; i < pt3.n; i++) {
        uint8_t u = pls_pt5[pt3.v[2 * i]];
        if (u == 2) continue;
        ol_push(&tc, 1, (uint32_t)i, (uint8_t)(pt3.st[i] | (u ? ST_FLAG : 0)), 0, 0);
    }
    for (uint32_t i = 0; i < nt5; i++) {
        uint8_t u = t5_pt5[i];
        if (u == 2) continue;
        ol_push(&tc, 2, i, (uint8_t)(t5.st[i] | (u ? ST_FLAG : 0)), 0, 0);
    }
    for (uint32_t i = 0; i < np; i++) {
        uint8_t u = pls_pt5[i] > pls_pt3[i] ? pls_pt5[i] : pls_pt3[i];
        if (u == 2) continue;
        ol_push(&tc, 3, i, (uint8_t)(ST_ACC | (u ? ST_FLAG : 0)), 0, 0);
    }

    /* ---- duplicate cleaning of the track candidates ----
       Reading (the paper lists the candidate types but not how duplicates
       are removed): a candidate with outer-tracker MDs (pT5: the 5 of its
       T5, pT3: the 3 of its T3, T5: its 5) is removed when another such
       candidate shares more than half of the smaller of the two MD sets and
       ranks higher.  Rank: type (pT5, then pT3, then T5), then the smaller
       curvature disagreement -- |kappa_seed - kappa_obj| / (sigma_seed +
       sigma_obj) for pT5 / pT3, |kappa_ABC - kappa_CDE| / (sigma_ABC +
       sigma_CDE) of the two T3s for a T5, in binary64 -- then the smaller
       index in its own list.  Seed-only candidates carry no outer-tracker
       hit and are all kept.  Every pair is compared (no ordering of the
       removals): a candidate is kept unless a higher-ranked duplicate exists. */
    size_t ntc = tc.n;
    uint8_t *keep = (uint8_t *)malloc(ntc ? ntc : 1);
    uint32_t *tmd = (uint32_t *)calloc(5 * (ntc ? ntc : 1), sizeof(uint32_t));
    uint32_t *tnm = (uint32_t *)calloc(ntc ? ntc : 1, sizeof(uint32_t));
    double *tq = (double *)calloc(ntc ? ntc : 1, sizeof(double));
    double kB = 0.299792458e-2 * p->B;
    for (size_t i = 0; i < ntc; i++) {
        uint32_t typ = tc.v[2 * i], idx = tc.v[2 * i + 1];
        keep[i] = 1;
        if (typ == 3 || !(tc.st[i] & ST_ACC)) continue;
        uint32_t u, w = 0, ps = 0;
        if (typ == 0) { ps = pt5.v[2 * idx]; u = t5.v[2 * pt5.v[2 * idx + 1]]; w = t5.v[2 * pt5.v[2 * idx + 1] + 1]; }
        else if (typ == 1) { ps = pt3.v[2 * idx]; u = pt3.v[2 * idx + 1]; }
        else { u = t5.v[2 * idx]; w = t5.v[2 * idx + 1]; }
        uint32_t *m = tmd + 5 * i;
        m[0] = t3m.v[2 * u];
        m[1] = ls.v[2 * t3.v[2 * u] + 1];
        m[2] = t3m.v[2 * u + 1];
        tnm[i] = 3;
        if (typ != 1) {
            m[3] = ls.v[2 * t3.v[2 * w] + 1];
            m[4] = t3m.v[2 * w + 1];
            tnm[i] = 5;
        }
        if (typ == 2) {
            tq[i] = fabs((double)t3.f0[u] - (double)t3.f0[w]) / ((double)t3.f1[u] + (double)t3.f1[w]);
        } else {
            double kp = (double)ev->pls_par[5 * (size_t)ps] * kB;
            double skp = kB * sqrt((double)ev->pls_cov[15 * (size_t)ps]);
            uint32_t o = typ == 0 ? pt5.v[2 * idx + 1] : u;
            double ko = typ == 0 ? (double)t5.f0[o] : (double)t3.f0[o];
            double so = typ == 0 ? (double)t5.f1[o] : (double)t3.f1[o];
            tq[i] = fabs(kp - ko) / (skp + so);
        }
    }
    for (size_t i = 0; i < ntc; i++) {
        if (!tnm[i]) continue;
        for (size_t j = 0; j < ntc && keep[i]; j++) {
            if (j == i || !tnm[j]) continue;
            uint32_t ti = tc.v[2 * i], tj = tc.v[2 * j];
            int better = tj < ti || (tj == ti && (tq[j] < tq[i] || (tq[j] == tq[i] && tc.v[2 * j + 1] < tc.v[2 * i + 1])));
            if (!better) continue;
            uint32_t shared = 0;
            for (uint32_t x = 0; x < tnm[i]; x++)
                for (uint32_t y = 0; y < tnm[j]; y++)
                    if (tmd[5 * i + x] == tmd[5 * j + y]) shared++;
            uint32_t small = tnm[i] < tnm[j] ? tnm[i] : tnm[j];
            if (2 * shared > small) keep[i] = 0;
        }
    }
    free(tmd); free(tnm); free(tq);

    out->n_md = nmd; out->md = md.v; out->md_st = md.st;
    out->n_ls = nls; out->ls = ls.v; out->ls_st = ls.st;
    out->n_t3 = nt3; out->t3 = t3.v; out->t3_st = t3.st; out->t3_k = t3.f0; out->t3_sk = t3.f1;
    out->n_t5 = nt5; out->t5 = t5.v; out->t5_st = t5.st; out->t5_k = t5.f0; out->t5_sk = t5.f1;
    out->tc_keep = keep;
    out->n_pt3 = (uint32_t)pt3.n; out->pt3 = pt3.v; out->pt3_st = pt3.st;
    out->n_pt5 = (uint32_t)pt5.n; out->pt5 = pt5.v; out->pt5_st = pt5.st;
    out->n_tc = (uint32_t)tc.n; out->tc = tc.v; out->tc_st = tc.st;

    free(hr); free(key); free(hit_items); free(hit_off);
    free(mdx.v); free(mdx.st); free(mdx.f0); free(mdx.f1);
    free(mdz.v); free(mdz.st); free(mdz.f0); free(mdz.f1);
    free(mdb.v); free(mdb.st); free(mdb.f0); free(mdb.f1);
    free(md_mod_v); free(anc); free(md_surf); free(surf_items); free(surf_off);
    free(ls_items); free(ls_off); free(t3m.v); free(t3m.st);
    free(t3_items); free(t3_off);
    free(pls_pt5); free(pls_pt3); free(t5_pt5);
    return 0;
}

void or_free(or_result *r)
{
    free(r->md); free(r->md_st); free(r->ls); free(r->ls_st);
    free(r->t3); free(r->t3_st); free(r->t3_k); free(r->t3_sk);
    free(r->t5); free(r->t5_st); free(r->pt3); free(r->pt3_st);
    free(r->pt5); free(r->pt5_st); free(r->tc); free(r->tc_st);
    free(r->t5_k); free(r->t5_sk); free(r->tc_keep);
    memset(r, 0, sizeof *r);
}

/* ------------------------------------------------ single-cut accessors --
 * Small entry points so the tests can pin individual windows. */

void or_module_const(const or_geom *g, const or_params *p, uint32_t m, float out[4])
{
    derived d; derive(g, p, &d);
    mdconst c = module_const(g, p, &d, m);
    out[0] = c.S; out[1] = c.G; out[2] = c.K; out[3] = c.D;
}

void or_pair_const(const or_geom *g, const or_params *p, uint32_t A, uint32_t B, float out[12])
{
    derived d; derive(g, p, &d);
    lsconst c = pair_const(g, p, &d, A, B);
    out[0] = (float)c.type; out[1] = c.S; out[2] = c.rho_lo; out[3] = c.rho_hi;
    out[4] = c.lam_lo; out[5] = c.lam_hi; out[6] = c.tau; out[7] = c.lo_fac;
    out[8] = c.hi_fac; out[9] = c.cf; out[10] = c.zbpl; out[11] = c.zbml;
}

float or_kappa3(const or_geom *g, const or_params *p, const float xy[6])
{
    derived d; derive(g, p, &d);
    float k, sk, d1, d2;
    kappa3(&d, xy[0], xy[1], 0, xy[2], xy[3], 0, xy[4], xy[5], 0.0f, 0, &k, &sk, &d1, &d2);
    return k;
}

/* derived binary32 constants: L, ec, kmax, khalf, ns, srp, sc, Kb */
void or_derived(const or_geom *g, const or_params *p, float out[8])
{
    derived d; derive(g, p, &d);
    out[0] = d.L; out[1] = d.ec; out[2] = d.kmaxf; out[3] = d.khalf;
    out[4] = d.ns; out[5] = d.srp; out[6] = d.sc; out[7] = d.Kb;
}

/* curvature and resolution of three anchors; disk[i] = 1 for an anchor on a
   disk, rC the radius of the third anchor */
void or_kappa3_res(const or_geom *g, const or_params *p, const float xy[6], const int disk[3], float rC,
                   float out[2])
{
    derived d; derive(g, p, &d);
    float k, sk, d1, d2;
    kappa3(&d, xy[0], xy[1], disk[0], xy[2], xy[3], disk[1], xy[4], xy[5], rC, disk[2], &k, &sk, &d1, &d2);
    out[0] = k; out[1] = sk;
}

/* one pixel-seed anchor test (see p_anchor): out = (azimuth difference, its
   window, coarse deviation, its window); returns p_anchor's code */
int or_pls_anchor(const or_params *p, const float par[5], const float cov[15],
                  float x, float y, float z, int disk, double out[4])
{
    double kB = 0.299792458e-2 * p->B;
    double kp = (double)par[0] * kB;
    double skp = kB * sqrt((double)cov[0]);
    anchor a = {x, y, z, sqrtf(x * x + y * y), disk};
    out[0] = out[1] = out[2] = out[3] = 0.0;
    return p_anchor(p, kp, skp, par, cov, &a, out);
}
