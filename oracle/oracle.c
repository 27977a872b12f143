/*
 * Plain FP64 CPU oracle of per-column multi-level accelerated
 * Lambda-iteration (MALI).  TEST INFRASTRUCTURE ONLY: only the tests, the
 * smoke check and the CPU-baseline leg of the benchmark load it.  It shares
 * no code with the GPU library; parity between the two is the point.
 *
 * What it follows.  The paper (Sec. 2.1) names the method: MALI in the
 * Rybicki & Hummer (1992) formalism with a local (diagonal) approximate
 * Psi operator, preconditioned rate equations and overlapping transitions;
 * it writes none of the equations.  The steps below are the standard
 * published forms of those methods, in this order per iteration:
 *   1. opacity and emissivity of every ray from the current populations;
 *   2. formal solution along every (wavelength, angle, direction) ray with
 *      linear short characteristics (Olson & Kunasz 1987), giving I, the
 *      diagonal Lambda* and Psi* = Lambda* over chi, and the effective intensity
 *      I_eff = I - Psi* eta_atom (Sec. 2.1: local approximate Psi operator);
 *   3. accumulation of the preconditioned radiative rates (Sec. 2.1:
 *      preconditioning of the rate equations, overlapping transitions);
 *   4. statistical equilibrium per depth, linear in the new populations,
 *      with particle conservation replacing one equation;
 *   5. maximum relative population change (Sec. 2.3, the convergence
 *      measure of Fig. 1) and Ng extrapolation (Sec. 2.3, Ng 1974 / Auer).
 * Start solutions: LTE, zero radiation and escape-probability iterations
 * (Sec. 2.3, "Different starting solutions").  Collisional-radiative switching (Sec. 2.3; Hummer &
 * Voels 1988): a constant collision multiplier, and a factor on the
 * collision rates that starts at f0 and falls tenfold per iteration to 1
 * (see orc_crs_factor; this schedule is a reading, the paper gives none).
 * Partial frequency redistribution (Sec. 2.1: MALI extended to PRD after
 * Uitenbroek 2001, angle-averaged option; Sec. 2.3: PRD switching, Eq. 1):
 * lines flagged PRD emit with psi = rho phi, rho updated after every
 * iteration from the angle-averaged redistribution function R_II (see
 * orc_rII and prd_update).
 * Output: emergent vertical intensity
 * (Sec. 2.2: only vertical emergent spectra) and per-transition Psi*.
 *
 * Everything is SI.  Depth index k = 0 is the top (largest z).
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <ctype.h>

/* CODATA 2018 */
#define PH 6.62607015e-34
#define PC 2.99792458e8
#define PKB 1.380649e-23
#define PME 9.1093837015e-31
#define PQE 1.602176634e-19
#define PEPS0 8.8541878128e-12
#define PAMU 1.66053906660e-27
#define PPI 3.14159265358979323846
/* electron-impact rate constant of the Omega collision model, m^3 s^-1 K^1/2 */
#define COLL_C0 8.629e-12
/* reference wavelength of the background opacity law */
#define BG_LAMBDA_REF 500.0e-9
#define BG_THETA 8750.0
/* below this optical step the short-characteristic weights use their series */
#define SC_SERIES_X 1.0e-2

static __thread char orc_err[256];
const char *orc_last_error(void) { return orc_err; }
#define FAIL(code, ...) do { snprintf(orc_err, sizeof orc_err, __VA_ARGS__); return (code); } while (0)

typedef struct {
    int kind;           /* 0 bound-bound line, 1 bound-free continuum */
    int l, u;
    double f;           /* line absorption oscillator strength */
    int voigt;          /* line: 1 Voigt profile, 0 Gaussian */
    int coll_kind;      /* 0: Omega model, 1: fixed destruction probability eps */
    double coll_val;
    double alpha0;      /* continuum cross-section at the edge, m^2 */
    double c_el;        /* line: elastic-collision rate per hydrogen atom, m^3 s^-1
                           (Q_E = c_el n_H; broadens the line and sets its coherence) */
    int prd;            /* line: partial frequency redistribution (angle-averaged R_II) */
    /* line: Zeeman pattern (both levels carry J and a Lande factor), else n_zc = 0 */
    int n_zc;
    int *zq;            /* q = M_l - M_u of each component: -1, 0, +1 */
    double *zshift;     /* g_u M_u - g_l M_l: the component's shift in Larmor frequencies */
    double *zstr;       /* relative strength; the strengths of each q sum to 1 */
    int n_own;
    double *lam_own;    /* the transition's own wavelengths, m */
    /* derived */
    double nu0, Aul, Bul, Blu, gamma_rad;
    double lam_min, lam_max;
    int n_act;
    int *act;           /* indices into the union grid, increasing wavelength */
    double *wnu;        /* trapezoid weights in frequency over the active points */
} orc_trans;

typedef struct orc_atom {
    double mass, abund;
    int L;
    double *E, *g;
    int *stage;
    int *twoJ;                /* 2 J of each level, -1 if the atom gives none */
    double *gL;               /* Lande factor of each level */
    int n_lines, n_cont, T;   /* transitions: lines first, then continua */
    orc_trans *tr;
    int bg_kind;              /* 0 none, 1 H-minus-like law */
    double c_bg;
    int NL;
    double *lam, *nu;         /* union grid, increasing wavelength */
} orc_atom;

typedef struct {
    int n_mu;
    double tol;
    int max_iter;
    int ng_order, ng_delay, ng_period;
    int start;           /* 0 LTE, 1 zero radiation, 2 provided */
    double coll_scale;   /* collision multiplier (1 = physical) */
    double crs_f0;       /* collisional-radiative switching: initial factor (<= 1: off) */
    double tol_fp;       /* > 0: also require the estimated distance to the fixed point
                            below tol_fp (see converged_at); 0: off */
    int esc_iter;        /* escape-probability start: number of iterations */
    int prd;             /* 1: lines flagged PRD in the atom use PRD; 0: every line CRD */
    double prd_eps0;     /* PRD switching (Eq. 1): eps of the update after iteration n is
                            min(1, prd_eps0 n^2); <= 0: off (eps = 1) */
} orc_opts;

/* ------------------------------------------------------------------ */
/* atom file                                                            */
/* ------------------------------------------------------------------ */
typedef struct { char *buf; char *p; } tokstream;

static const char *next_tok(tokstream *ts) {
    for (;;) {
        while (*ts->p && isspace((unsigned char)*ts->p)) ts->p++;
        if (*ts->p == '#') { while (*ts->p && *ts->p != '\n') ts->p++; continue; }
        break;
    }
    if (!*ts->p) return NULL;
    char *s = ts->p;
    while (*ts->p && !isspace((unsigned char)*ts->p)) ts->p++;
    if (*ts->p) { *ts->p = 0; ts->p++; }
    return s;
}

static int tok_double(tokstream *ts, double *v) {
    const char *t = next_tok(ts);
    if (!t) return -1;
    char *e; *v = strtod(t, &e);
    return (*e == 0) ? 0 : -1;
}
static int tok_int(tokstream *ts, int *v) {
    const char *t = next_tok(ts);
    if (!t) return -1;
    char *e; long x = strtol(t, &e, 10);
    *v = (int)x;
    return (*e == 0) ? 0 : -1;
}
static int tok_expect(tokstream *ts, const char *kw) {
    const char *t = next_tok(ts);
    return (t && strcmp(t, kw) == 0) ? 0 : -1;
}

static int cmp_double(const void *a, const void *b) {
    double x = *(const double *)a, y = *(const double *)b;
    return (x > y) - (x < y);
}

void orc_atom_free(orc_atom *a) {
    if (!a) return;
    for (int t = 0; t < a->T; t++) {
        free(a->tr[t].lam_own); free(a->tr[t].act); free(a->tr[t].wnu);
        free(a->tr[t].zq); free(a->tr[t].zshift); free(a->tr[t].zstr);
    }
    free(a->tr); free(a->E); free(a->g); free(a->stage); free(a->lam); free(a->nu); free(a->twoJ); free(a->gL);
    free(a);
}

static int parse_transition(tokstream *ts, orc_trans *t, int kind, int L) {
    t->kind = kind;
    if (tok_int(ts, &t->l) || tok_int(ts, &t->u)) return -1;
    if (t->l < 0 || t->u >= L || t->l >= t->u) return -1;
    if (kind == 0) {
        if (tok_double(ts, &t->f)) return -1;
        const char *p = next_tok(ts);
        if (!p) return -1;
        if (!strcmp(p, "VOIGT")) t->voigt = 1; else if (!strcmp(p, "GAUSS")) t->voigt = 0; else return -1;
    } else {
        if (tok_double(ts, &t->alpha0)) return -1;
    }
    const char *c = next_tok(ts);
    if (!c) return -1;
    if (!strcmp(c, "OMEGA")) t->coll_kind = 0; else if (!strcmp(c, "EPS")) t->coll_kind = 1; else return -1;
    if (tok_double(ts, &t->coll_val) || tok_int(ts, &t->n_own) || t->n_own < 2) return -1;
    t->lam_own = malloc(sizeof(double) * t->n_own);
    for (int i = 0; i < t->n_own; i++) {
        if (tok_double(ts, &t->lam_own[i])) return -1;
        t->lam_own[i] *= 1e-9;
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* Zeeman patterns                                                      */
/* ------------------------------------------------------------------ */
static double fact(int n) {
    double f = 1.0;
    for (int i = 2; i <= n; i++) f *= i;
    return f;
}

/* Wigner 3j symbol (j1 j2 j3; m1 m2 m3) from Racah's single-sum formula;
 * arguments are twice the angular momenta and projections. */
double orc_wigner3j(int tj1, int tj2, int tj3, int tm1, int tm2, int tm3) {
    if (tm1 + tm2 + tm3 != 0) return 0.0;
    if (tj3 < abs(tj1 - tj2) || tj3 > tj1 + tj2 || ((tj1 + tj2 + tj3) & 1)) return 0.0;
    if (abs(tm1) > tj1 || abs(tm2) > tj2 || abs(tm3) > tj3) return 0.0;
    if (((tj1 + tm1) & 1) || ((tj2 + tm2) & 1) || ((tj3 + tm3) & 1)) return 0.0;
    /* integer combinations (halves of sums of the doubled arguments) */
    int a1 = (tj1 + tj2 - tj3) / 2, a2 = (tj1 - tj2 + tj3) / 2, a3 = (-tj1 + tj2 + tj3) / 2;
    int a4 = (tj1 + tj2 + tj3) / 2 + 1;
    double tri = fact(a1) * fact(a2) * fact(a3) / fact(a4);
    double pre = fact((tj1 + tm1) / 2) * fact((tj1 - tm1) / 2) * fact((tj2 + tm2) / 2) * fact((tj2 - tm2) / 2) *
                 fact((tj3 + tm3) / 2) * fact((tj3 - tm3) / 2);
    int b1 = (tj3 - tj2 + tm1) / 2, b2 = (tj3 - tj1 - tm2) / 2;   /* k + b1 >= 0, k + b2 >= 0 */
    int c1 = (tj1 + tj2 - tj3) / 2, c2 = (tj1 - tm1) / 2, c3 = (tj2 + tm2) / 2;  /* k <= c */
    int kmin = 0;
    if (-b1 > kmin) kmin = -b1;
    if (-b2 > kmin) kmin = -b2;
    int kmax = c1;
    if (c2 < kmax) kmax = c2;
    if (c3 < kmax) kmax = c3;
    double sum = 0.0;
    for (int k = kmin; k <= kmax; k++) {
        double d = fact(k) * fact(k + b1) * fact(k + b2) * fact(c1 - k) * fact(c2 - k) * fact(c3 - k);
        sum += ((k & 1) ? -1.0 : 1.0) / d;
    }
    int ph = (tj1 - tj2 - tm3) / 2;
    return ((ph & 1) ? -1.0 : 1.0) * sqrt(tri * pre) * sum;
}

/* Anomalous Zeeman pattern of a dipole line between a lower level (J_l,
 * g_l) and an upper level (J_u, g_u) (Sec. 2.1: Zeeman splitting of
 * bound-bound transitions).  Components are the pairs (M_u, M_l) with
 * q = M_l - M_u in {-1, 0, 1}; each is shifted by (g_u M_u - g_l M_l)
 * Larmor frequencies e B / (4 pi m_e) and has the strength
 * 3 (J_u J_l 1; -M_u M_l -q)^2, which sums to 1 over the components of each
 * q.  Components of zero strength are left out.  Arguments are 2J; returns
 * the number of components (at most max), or -1. */
int orc_zeeman_pattern(int twoJl, double gl, int twoJu, double gu, int max, int *q, double *shift, double *strength) {
    int n = 0;
    for (int tmu = -twoJu; tmu <= twoJu; tmu += 2)
        for (int tml = -twoJl; tml <= twoJl; tml += 2) {
            int tq = tml - tmu;
            if (tq < -2 || tq > 2) continue;
            double w = orc_wigner3j(twoJu, twoJl, 2, -tmu, tml, -tq);
            if (w == 0.0) continue;
            if (n >= max) return -1;
            q[n] = tq / 2;
            shift[n] = gu * 0.5 * tmu - gl * 0.5 * tml;
            strength[n] = 3.0 * w * w;
            n++;
        }
    return n;
}

int orc_atom_load(const char *path, orc_atom **out) {
    *out = NULL;
    FILE *fp = fopen(path, "rb");
    if (!fp) FAIL(-1, "cannot open %s", path);
    fseek(fp, 0, SEEK_END); long n = ftell(fp); fseek(fp, 0, SEEK_SET);
    tokstream ts; ts.buf = malloc(n + 1);
    if (fread(ts.buf, 1, n, fp) != (size_t)n) { fclose(fp); free(ts.buf); FAIL(-1, "read error"); }
    ts.buf[n] = 0; ts.p = ts.buf; fclose(fp);
    orc_atom *a = calloc(1, sizeof *a);
    int ver, rc = -1;
    const char *tk;
    if (tok_expect(&ts, "RH15D-ATOM") || tok_int(&ts, &ver)) goto bad;
    if (tok_expect(&ts, "NAME") || !next_tok(&ts)) goto bad;
    if (tok_expect(&ts, "MASS_AMU") || tok_double(&ts, &a->mass)) goto bad;
    a->mass *= PAMU;
    if (tok_expect(&ts, "ABUNDANCE") || tok_double(&ts, &a->abund)) goto bad;
    if (tok_expect(&ts, "LEVELS") || tok_int(&ts, &a->L) || a->L < 2) goto bad;
    a->E = malloc(sizeof(double) * a->L); a->g = malloc(sizeof(double) * a->L); a->stage = malloc(sizeof(int) * a->L);
    for (int i = 0; i < a->L; i++) {
        if (tok_double(&ts, &a->E[i]) || tok_double(&ts, &a->g[i]) || tok_int(&ts, &a->stage[i])) goto bad;
        a->E[i] *= PQE;
    }
    if (tok_expect(&ts, "LINES") || tok_int(&ts, &a->n_lines) || a->n_lines < 0) goto bad;
    orc_trans *lines = calloc(a->n_lines ? a->n_lines : 1, sizeof(orc_trans));
    for (int i = 0; i < a->n_lines; i++) if (parse_transition(&ts, &lines[i], 0, a->L)) { free(lines); goto bad; }
    if (tok_expect(&ts, "CONTINUA") || tok_int(&ts, &a->n_cont) || a->n_cont < 0) { free(lines); goto bad; }
    a->T = a->n_lines + a->n_cont;
    a->tr = calloc(a->T ? a->T : 1, sizeof(orc_trans));
    memcpy(a->tr, lines, sizeof(orc_trans) * a->n_lines);
    free(lines);
    for (int i = 0; i < a->n_cont; i++) if (parse_transition(&ts, &a->tr[a->n_lines + i], 1, a->L)) goto bad;
    /* optional: elastic collisions and the redistribution of lines */
    if (!(tk = next_tok(&ts))) goto bad;
    if (!strcmp(tk, "ELASTIC")) {
        int ne;
        if (tok_int(&ts, &ne) || ne < 0) goto bad;
        for (int i = 0; i < ne; i++) {
            int li;
            double c;
            const char *kind;
            if (tok_int(&ts, &li) || li < 0 || li >= a->n_lines || tok_double(&ts, &c) || !(c >= 0.0)) goto bad;
            if (!(kind = next_tok(&ts))) goto bad;
            a->tr[li].c_el = c;
            if (!strcmp(kind, "PRD")) a->tr[li].prd = 1; else if (!strcmp(kind, "CRD")) a->tr[li].prd = 0; else goto bad;
        }
        if (!(tk = next_tok(&ts))) goto bad;
    }
    a->twoJ = malloc(sizeof(int) * a->L);
    a->gL = calloc(a->L, sizeof(double));
    for (int i = 0; i < a->L; i++) a->twoJ[i] = -1;
    if (!strcmp(tk, "ZEEMAN")) {
        int nz;
        if (tok_int(&ts, &nz) || nz < 0) goto bad;
        for (int i = 0; i < nz; i++) {
            int li, tj;
            double gl;
            if (tok_int(&ts, &li) || li < 0 || li >= a->L || tok_int(&ts, &tj) || tj < 0 || tj > 40 ||
                tok_double(&ts, &gl))
                goto bad;
            a->twoJ[li] = tj;
            a->gL[li] = gl;
        }
        if (!(tk = next_tok(&ts))) goto bad;
    }
    if (strcmp(tk, "BACKGROUND") || !(tk = next_tok(&ts))) goto bad;
    if (!strcmp(tk, "NONE")) a->bg_kind = 0;
    else if (!strcmp(tk, "HMINUS")) { a->bg_kind = 1; if (tok_double(&ts, &a->c_bg)) goto bad; }
    else goto bad;
    if (tok_expect(&ts, "END")) goto bad;
    rc = 0;
bad:
    free(ts.buf);
    if (rc) { orc_atom_free(a); FAIL(-2, "malformed atom file %s", path); }

    /* atomic data of each transition */
    for (int t = 0; t < a->T; t++) {
        orc_trans *tr = &a->tr[t];
        double dE = a->E[tr->u] - a->E[tr->l];
        if (!(dE > 0)) { orc_atom_free(a); FAIL(-2, "transition %d has no positive energy gap", t); }
        tr->nu0 = dE / PH;
        if (tr->kind == 0) {
            tr->Aul = 2.0 * PPI * PQE * PQE * tr->nu0 * tr->nu0 / (PEPS0 * PME * PC * PC * PC)
                      * (a->g[tr->l] / a->g[tr->u]) * tr->f;
            tr->Bul = tr->Aul * PC * PC / (2.0 * PH * tr->nu0 * tr->nu0 * tr->nu0);
            tr->Blu = a->g[tr->u] / a->g[tr->l] * tr->Bul;
        }
        tr->lam_min = tr->lam_max = tr->lam_own[0];
        for (int i = 1; i < tr->n_own; i++) {
            if (tr->lam_own[i] < tr->lam_min) tr->lam_min = tr->lam_own[i];
            if (tr->lam_own[i] > tr->lam_max) tr->lam_max = tr->lam_own[i];
        }
    }
    /* radiative damping: spontaneous rates out of both levels of each line */
    for (int t = 0; t < a->n_lines; t++) {
        orc_trans *tr = &a->tr[t];
        double gam = 0.0;
        for (int s = 0; s < a->n_lines; s++) {
            if (a->tr[s].u == tr->u) gam += a->tr[s].Aul;
            if (a->tr[s].u == tr->l) gam += a->tr[s].Aul;
        }
        tr->gamma_rad = gam;
    }
    /* Zeeman patterns of the lines whose two levels carry J and g */
    for (int t = 0; t < a->n_lines; t++) {
        orc_trans *tr = &a->tr[t];
        int jl = a->twoJ[tr->l], ju = a->twoJ[tr->u];
        if (jl < 0 || ju < 0) continue;
        int mx = (jl + 1) * (ju + 1);
        tr->zq = malloc(sizeof(int) * mx); tr->zshift = malloc(sizeof(double) * mx); tr->zstr = malloc(sizeof(double) * mx);
        tr->n_zc = orc_zeeman_pattern(jl, a->gL[tr->l], ju, a->gL[tr->u], mx, tr->zq, tr->zshift, tr->zstr);
        if (tr->n_zc <= 0) { orc_atom_free(a); FAIL(-2, "line %d: J values allow no dipole transition", t); }
    }
    /* union wavelength grid: all own points, sorted, exact duplicates merged */
    int tot = 0;
    for (int t = 0; t < a->T; t++) tot += a->tr[t].n_own;
    double *all = malloc(sizeof(double) * tot);
    int q = 0;
    for (int t = 0; t < a->T; t++) for (int i = 0; i < a->tr[t].n_own; i++) all[q++] = a->tr[t].lam_own[i];
    qsort(all, tot, sizeof(double), cmp_double);
    a->lam = malloc(sizeof(double) * tot);
    a->NL = 0;
    for (int i = 0; i < tot; i++) if (a->NL == 0 || all[i] != a->lam[a->NL - 1]) a->lam[a->NL++] = all[i];
    free(all);
    a->nu = malloc(sizeof(double) * a->NL);
    for (int j = 0; j < a->NL; j++) a->nu[j] = PC / a->lam[j];
    /* active points of each transition and their trapezoid weights in frequency */
    for (int t = 0; t < a->T; t++) {
        orc_trans *tr = &a->tr[t];
        tr->act = malloc(sizeof(int) * a->NL);
        tr->n_act = 0;
        for (int j = 0; j < a->NL; j++)
            if (a->lam[j] >= tr->lam_min && a->lam[j] <= tr->lam_max) tr->act[tr->n_act++] = j;
        tr->wnu = malloc(sizeof(double) * tr->n_act);
        for (int i = 0; i < tr->n_act; i++) {
            double nl = a->nu[tr->act[i > 0 ? i - 1 : i]];
            double nr = a->nu[tr->act[i < tr->n_act - 1 ? i + 1 : i]];
            tr->wnu[i] = 0.5 * (nl - nr);
        }
    }
    *out = a;
    return 0;
}

int orc_atom_info(const orc_atom *a, int *L, int *n_lines, int *n_cont, int *NL) {
    *L = a->L; *n_lines = a->n_lines; *n_cont = a->n_cont; *NL = a->NL;
    return 0;
}
double orc_atom_abundance(const orc_atom *a) { return a->abund; }
int orc_atom_lambda(const orc_atom *a, double *lam) { memcpy(lam, a->lam, sizeof(double) * a->NL); return 0; }
/* per transition: l, u, kind, n_active; weights copied if w != NULL (size n_active) */
int orc_atom_transition(const orc_atom *a, int t, int *l, int *u, int *kind, int *n_act, int *act, double *w) {
    if (t < 0 || t >= a->T) return -1;
    const orc_trans *tr = &a->tr[t];
    *l = tr->l; *u = tr->u; *kind = tr->kind; *n_act = tr->n_act;
    if (act) memcpy(act, tr->act, sizeof(int) * tr->n_act);
    if (w) memcpy(w, tr->wnu, sizeof(double) * tr->n_act);
    return 0;
}
double orc_atom_einstein_A(const orc_atom *a, int t) { return a->tr[t].Aul; }

/* ------------------------------------------------------------------ */
/* small numerical pieces                                               */
/* ------------------------------------------------------------------ */

/* Gauss-Legendre nodes and weights on (0, 1), ascending; weights sum to 1. */
int orc_gauss_legendre(int n, double *x, double *w) {
    if (n < 1 || n > 64) return -1;
    for (int i = 0; i < n; i++) {
        double z = cos(PPI * (i + 0.75) / (n + 0.5)), dp = 1.0;
        for (int it = 0; it < 100; it++) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; k++) { double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k; p0 = p1; p1 = p2; }
            if (n == 1) { p1 = z; p0 = 1.0; }
            dp = n * (z * p1 - p0) / (z * z - 1.0);
            double dz = p1 / dp;
            z -= dz;
            if (fabs(dz) < 1e-16) break;
        }
        double p0 = 1.0, p1 = z;
        for (int k = 2; k <= n; k++) { double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k; p0 = p1; p1 = p2; }
        if (n == 1) { p1 = z; p0 = 1.0; }
        dp = n * (z * p1 - p0) / (z * z - 1.0);
        /* root z of P_n descends with i, so 0.5 (1 - z) ascends on (0, 1) */
        x[i] = 0.5 * (1.0 - z);
        w[i] = 1.0 / ((1.0 - z * z) * dp * dp);
    }
    return 0;
}

/* Faddeeva function w(v + i a) = H(a, v) + i L(a, v) by Humlicek (1982)
 * rational approximation W4 (four regions in s = |v| + a): H is the Voigt
 * function, L the (odd) dispersion function, so that the absorption and
 * magneto-optical profiles per unit v are H / sqrt(pi) and L / sqrt(pi). */
void orc_voigt_w(double a, double v, double *H, double *L) {
    double x = v, y = a;
    double s = fabs(x) + y;
    /* t = y - i x */
    double tr = y, ti = -x;
    double wr, wi;
    if (s >= 15.0) {
        /* t * 0.5641896 / (0.5 + t^2) */
        double ur = tr * tr - ti * ti + 0.5, ui = 2.0 * tr * ti;
        double nr = 0.5641896 * tr, ni = 0.5641896 * ti;
        double d = ur * ur + ui * ui;
        wr = (nr * ur + ni * ui) / d; wi = (ni * ur - nr * ui) / d;
    } else if (s >= 5.5) {
        /* t (1.410474 + u 0.5641896) / (0.75 + u (3 + u)), u = t^2 */
        double ur = tr * tr - ti * ti, ui = 2.0 * tr * ti;
        double pr = 1.410474 + 0.5641896 * ur, pi = 0.5641896 * ui;
        double nr = tr * pr - ti * pi, ni = tr * pi + ti * pr;
        double qr = 3.0 + ur, qi = ui;
        double dr = 0.75 + (ur * qr - ui * qi), di = (ur * qi + ui * qr);
        double d = dr * dr + di * di;
        wr = (nr * dr + ni * di) / d; wi = (ni * dr - nr * di) / d;
    } else if (y >= 0.195 * fabs(x) - 0.176) {
        static const double pa[5] = {16.4955, 20.20933, 11.96482, 3.778987, 0.5642236};
        static const double qa[6] = {16.4955, 38.82363, 39.27121, 21.69274, 6.699398, 1.0};
        double nr = pa[4], ni = 0.0;
        for (int i = 3; i >= 0; i--) { double r = nr * tr - ni * ti + pa[i], im = nr * ti + ni * tr; nr = r; ni = im; }
        double dr = qa[5], di = 0.0;
        for (int i = 4; i >= 0; i--) { double r = dr * tr - di * ti + qa[i], im = dr * ti + di * tr; dr = r; di = im; }
        double d = dr * dr + di * di;
        wr = (nr * dr + ni * di) / d; wi = (ni * dr - nr * di) / d;
    } else {
        /* exp(u) - t P(u) / Q(u), u = t^2 */
        static const double pb[7] = {36183.31, -3321.9905, 1540.787, -219.0313, 35.76683, -1.320522, 0.56419};
        static const double qb[8] = {32066.6, -24322.84, 9022.228, -2186.181, 364.2191, -61.57037, 1.841439, -1.0};
        double ur = tr * tr - ti * ti, ui = 2.0 * tr * ti;
        double pr = pb[6], pim = 0.0;
        for (int i = 5; i >= 0; i--) { double r = pr * ur - pim * ui + pb[i], im = pr * ui + pim * ur; pr = r; pim = im; }
        double qr = qb[7], qi = 0.0;
        for (int i = 6; i >= 0; i--) { double r = qr * ur - qi * ui + qb[i], im = qr * ui + qi * ur; qr = r; qi = im; }
        double nr = tr * pr - ti * pim, ni = tr * pim + ti * pr;
        double d = qr * qr + qi * qi;
        double fr = (nr * qr + ni * qi) / d, fi = (ni * qr - nr * qi) / d;
        double eu = exp(ur);
        wr = eu * cos(ui) - fr; wi = eu * sin(ui) - fi;
    }
    *H = wr;
    *L = wi;
}

/* Voigt function H(a, v) = Re w(v + i a). */
double orc_voigt_H(double a, double v) {
    double H, L;
    orc_voigt_w(a, v, &H, &L);
    return H;
}

/* Angle-averaged redistribution function R_II (Hummer 1962) in Doppler
 * units, for damping parameter a > 0 and frequencies x, x2 (normalised so
 * that its integral over x2 is H(a, x) / sqrt(pi)).  Written as the
 * Lorentzian average, over the frequency xi of the scattering in the atom's
 * frame, of the angle-averaged Doppler kernel of coherent scattering,
 * (1/2) erfc(max(|x - xi|, |x2 - xi|)) = (1/2) erfc(|xi - m| + d) with
 * m = (x + x2)/2 and d = |x - x2|/2:
 *   R_II(x, x2) = 1/2 integral (a/pi) / (a^2 + xi^2) erfc(|xi - m| + d) dxi,
 * which equals Hummer's integral over u of exp(-u^2) times a difference of
 * arctangents.  Quadrature (a reading; the paper prints no formula):
 * 0 where d >= 6 (erfc(6) = 2.2e-17); otherwise xi runs over
 * [m - w, m + w], w = 6 - d, cut at xi = m (the kink) and at xi = +-0.5
 * where inside; pieces within |xi| <= 0.5 (the Lorentzian core) are mapped
 * to t = asinh(xi / a), where the Lorentzian measure is dt / (pi cosh t),
 * and integrated by 4-point Gauss-Legendre on 8 panels uniform in t; the
 * other pieces by 4-point Gauss-Legendre on ceil(length) panels uniform in
 * xi.  Accuracy: within 1e-4 of the larger of R_II(x, x) and
 * R_II(x2, x2) for 1e-4 <= a <= 0.5. */
#define RII_CORE 0.5
#define RII_CORE_PANELS 8
double orc_rII(double a, double x, double x2) {
    static const double gx[4] = {-0.8611363115940526, -0.3399810435848563, 0.3399810435848563, 0.8611363115940526};
    static const double gw[4] = {0.3478548451374538, 0.6521451548625461, 0.6521451548625461, 0.3478548451374538};
    double m = 0.5 * (x + x2), d = 0.5 * fabs(x - x2);
    if (d >= 6.0) return 0.0;
    double w = 6.0 - d;
    /* cut points in increasing order */
    double e[5];
    int ne = 0;
    e[ne++] = m - w;
    if (-RII_CORE > m - w && -RII_CORE < m) e[ne++] = -RII_CORE;
    if (RII_CORE > m - w && RII_CORE < m) e[ne++] = RII_CORE;
    e[ne++] = m;
    double e2[2];
    int ne2 = 0;
    if (-RII_CORE > m && -RII_CORE < m + w) e2[ne2++] = -RII_CORE;
    if (RII_CORE > m && RII_CORE < m + w) e2[ne2++] = RII_CORE;
    for (int i = 0; i < ne2; i++) e[ne++] = e2[i];
    e[ne++] = m + w;
    double sum = 0.0;
    for (int i = 0; i + 1 < ne; i++) {
        double lo = e[i], hi = e[i + 1];
        if (!(hi > lo)) continue;
        if (lo >= -RII_CORE && hi <= RII_CORE) {
            double t0 = asinh(lo / a), h = (asinh(hi / a) - t0) / RII_CORE_PANELS;
            for (int p = 0; p < RII_CORE_PANELS; p++) {
                double c = t0 + (p + 0.5) * h;
                for (int q = 0; q < 4; q++) {
                    double sh = sinh(c + 0.5 * h * gx[q]);
                    sum += 0.5 * h * gw[q] * erfc(fabs(a * sh - m) + d) / (PPI * sqrt(1.0 + sh * sh));
                }
            }
        } else {
            int np = (int)ceil(hi - lo);
            if (np < 1) np = 1;
            double h = (hi - lo) / np;
            for (int p = 0; p < np; p++) {
                double c = lo + (p + 0.5) * h;
                for (int q = 0; q < 4; q++) {
                    double xi = c + 0.5 * h * gx[q];
                    sum += 0.5 * h * gw[q] * (a / PPI) / (a * a + xi * xi) * erfc(fabs(xi - m) + d);
                }
            }
        }
    }
    return 0.5 * sum;
}

/* Linear short-characteristic weights for an optical step x along a ray:
 * I_b = I_a e + wa S_a + wb S_b. */
void orc_sc_coefficients(double x, double *e, double *wa, double *wb) {
    if (x < SC_SERIES_X) {
        double x2 = x * x, x3 = x2 * x, x4 = x3 * x, x5 = x4 * x, x6 = x5 * x;
        *wb = x / 2.0 - x2 / 6.0 + x3 / 24.0 - x4 / 120.0 + x5 / 720.0 - x6 / 5040.0;
        *wa = x / 2.0 - x2 / 3.0 + x3 / 8.0 - x4 / 30.0 + x5 / 144.0 - x6 / 840.0;
        *e = exp(-x);
    } else {
        double em = -expm1(-x);
        double q = em / x;
        *e = 1.0 - em;
        *wb = 1.0 - q;
        *wa = q - *e;
    }
}

/* Formal solution along one ray of n points given the optical steps
 * dtau[i] between points i-1 and i (dtau[0] unused), the source function
 * S and the incoming intensity I0 at point 0.  Returns I and the diagonal
 * Lambda* (0 at the boundary point). */
int orc_formal_ray(int n, const double *dtau, const double *S, double I0, double *I, double *lstar) {
    I[0] = I0; lstar[0] = 0.0;
    for (int i = 1; i < n; i++) {
        double e, wa, wb;
        orc_sc_coefficients(dtau[i], &e, &wa, &wb);
        I[i] = I[i - 1] * e + wa * S[i - 1] + wb * S[i];
        lstar[i] = wb;
    }
    return 0;
}

/* LTE (Saha-Boltzmann) populations of one depth point, summing to ntot. */
static void lte_log_ratios(const orc_atom *a, double T, double ne, double *lnr) {
    double kT = PKB * T;
    double saha = log(2.0 / ne) + 1.5 * log(2.0 * PPI * PME * kT / (PH * PH));
    for (int i = 0; i < a->L; i++)
        lnr[i] = log(a->g[i] / a->g[0]) - (a->E[i] - a->E[0]) / kT + (a->stage[i] - a->stage[0]) * saha;
}
static void lte_from_log_ratios(int L, const double *lnr, double ntot, double *n) {
    double mx = lnr[0];
    for (int i = 1; i < L; i++) if (lnr[i] > mx) mx = lnr[i];
    double s = 0.0;
    for (int i = 0; i < L; i++) s += exp(lnr[i] - mx);
    for (int i = 0; i < L; i++) n[i] = ntot * exp(lnr[i] - mx) / s;
}
int orc_lte_populations(const orc_atom *a, double T, double ne, double ntot, double *n) {
    double lnr[64];
    if (a->L > 64) return -1;
    lte_log_ratios(a, T, ne, lnr);
    lte_from_log_ratios(a->L, lnr, ntot, n);
    return 0;
}

/* Planck function B_nu(T) */
static double planck(double nu, double T) {
    double x = PH * nu / (PKB * T);
    return 2.0 * PH * nu * nu * nu / (PC * PC) * exp(-x) / (-expm1(-x));
}

/* Dense Gaussian elimination with partial pivoting: solves A x = b (n x n). */
static int gauss_solve(int n, double *A, double *b) {
    for (int c = 0; c < n; c++) {
        int p = c;
        for (int r = c + 1; r < n; r++) if (fabs(A[r * n + c]) > fabs(A[p * n + c])) p = r;
        if (A[p * n + c] == 0.0) return -1;
        if (p != c) {
            for (int k = 0; k < n; k++) { double t = A[c * n + k]; A[c * n + k] = A[p * n + k]; A[p * n + k] = t; }
            double t = b[c]; b[c] = b[p]; b[p] = t;
        }
        for (int r = c + 1; r < n; r++) {
            double f = A[r * n + c] / A[c * n + c];
            for (int k = c; k < n; k++) A[r * n + k] -= f * A[c * n + k];
            b[r] -= f * b[c];
        }
    }
    for (int r = n - 1; r >= 0; r--) {
        double s = b[r];
        for (int k = r + 1; k < n; k++) s -= A[r * n + k] * b[k];
        b[r] = s / A[r * n + r];
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* one column                                                           */
/* ------------------------------------------------------------------ */
typedef struct {
    const orc_atom *a;
    int N, nmu;
    const double *z, *T, *ne, *nH, *vz, *vt;
    double *mu, *wmu;
    double *ntot;        /* [N] */
    double *lnr;         /* [N][L] Saha-Boltzmann log ratios to level 0 */
    double *nstar;       /* [N][L] */
    double *C;           /* [N][L][L]  C[i][j]: rate i -> j */
    double *kbg;         /* [N] background opacity at 500 nm */
    double *dnuD;        /* [n_lines][N] */
    double *adamp;       /* [n_lines][N] */
    double *norm;        /* [n_lines][N] profile normalisation sum */
    double **phi;        /* per line: [N][n_act][nmu][2] normalised profile */
    /* PRD (lines with prd set, when the solve enables PRD; NULL otherwise) */
    double **gII;        /* per line: [N][n_act][n_act] redistribution weights g(j', j) */
    double **rho;        /* per line: [N][n_act] emission / absorption profile ratio */
    double *Iall;        /* [NL][nmu][2][N] intensity of every ray of the last sweep */
} colstate;

static double line_profile(const orc_atom *a, int t, const colstate *cs, int k, double nu, double mus) {
    const orc_trans *tr = &a->tr[t];
    double dnd = cs->dnuD[t * cs->N + k];
    double v = (nu - tr->nu0 * (1.0 + mus * cs->vz[k] / PC)) / dnd;
    double H = tr->voigt ? orc_voigt_H(cs->adamp[t * cs->N + k], v) : exp(-v * v);
    return H / (sqrt(PPI) * dnd);
}

static void column_prepare(colstate *cs, double coll_scale) {
    const orc_atom *a = cs->a;
    int N = cs->N, L = a->L, nmu = cs->nmu;
    cs->ntot = malloc(sizeof(double) * N);
    cs->lnr = malloc(sizeof(double) * N * L);
    cs->nstar = malloc(sizeof(double) * N * L);
    cs->C = calloc((size_t)N * L * L, sizeof(double));
    cs->kbg = malloc(sizeof(double) * N);
    int nl = a->n_lines ? a->n_lines : 1;
    cs->dnuD = malloc(sizeof(double) * nl * N);
    cs->adamp = malloc(sizeof(double) * nl * N);
    cs->norm = malloc(sizeof(double) * nl * N);
    cs->phi = calloc(nl, sizeof(double *));
    for (int k = 0; k < N; k++) {
        cs->ntot[k] = a->abund * cs->nH[k];
        lte_log_ratios(a, cs->T[k], cs->ne[k], &cs->lnr[k * L]);
        lte_from_log_ratios(L, &cs->lnr[k * L], cs->ntot[k], &cs->nstar[k * L]);
        cs->kbg[k] = (a->bg_kind == 1)
            ? a->c_bg * cs->nH[k] * cs->ne[k] * pow(cs->T[k], -1.5) * exp(BG_THETA / cs->T[k]) : 0.0;
        /* collisions */
        for (int t = 0; t < a->T; t++) {
            const orc_trans *tr = &a->tr[t];
            double Cul;
            if (tr->coll_kind == 0) {
                Cul = cs->ne[k] * COLL_C0 * tr->coll_val / (a->g[tr->u] * sqrt(cs->T[k]));
            } else {
                double x = PH * tr->nu0 / (PKB * cs->T[k]);
                Cul = tr->coll_val / (1.0 - tr->coll_val) * tr->Aul / (-expm1(-x));
            }
            Cul *= coll_scale;
            double Clu = Cul * exp(cs->lnr[k * L + tr->u] - cs->lnr[k * L + tr->l]);
            cs->C[(k * L + tr->u) * L + tr->l] += Cul;
            cs->C[(k * L + tr->l) * L + tr->u] += Clu;
        }
    }
    /* line profiles on every ray of the quadrature, normalised per depth */
    for (int t = 0; t < a->n_lines; t++) {
        const orc_trans *tr = &a->tr[t];
        for (int k = 0; k < N; k++) {
            double vth2 = 2.0 * PKB * cs->T[k] / a->mass + cs->vt[k] * cs->vt[k];
            double dnd = tr->nu0 / PC * sqrt(vth2);
            cs->dnuD[t * N + k] = dnd;
            cs->adamp[t * N + k] = (tr->gamma_rad + tr->c_el * cs->nH[k]) / (4.0 * PPI * dnd);
        }
        int na = tr->n_act;
        double *ph = malloc(sizeof(double) * (size_t)N * na * nmu * 2);
        for (int k = 0; k < N; k++) {
            double sum = 0.0;
            for (int ja = 0; ja < na; ja++) {
                double nu = a->nu[tr->act[ja]];
                for (int m = 0; m < nmu; m++) for (int s = 0; s < 2; s++) {
                    double mus = s ? cs->mu[m] : -cs->mu[m];     /* s = 1: upward */
                    double p = line_profile(a, t, cs, k, nu, mus);
                    ph[(((size_t)k * na + ja) * nmu + m) * 2 + s] = p;
                    sum += tr->wnu[ja] * 0.5 * cs->wmu[m] * p;
                }
            }
            cs->norm[t * N + k] = sum;
            for (int i = 0; i < na * nmu * 2; i++) ph[(size_t)k * na * nmu * 2 + i] /= sum;
        }
        cs->phi[t] = ph;
    }
}

static void prd_tables(colstate *cs, int t);

static void column_release(colstate *cs) {
    free(cs->ntot); free(cs->lnr); free(cs->nstar); free(cs->C); free(cs->kbg);
    for (int t = 0; t < cs->a->n_lines; t++) free(cs->phi[t]);
    free(cs->phi); free(cs->dnuD); free(cs->adamp); free(cs->norm);
    if (cs->rho) {
        for (int t = 0; t < cs->a->n_lines; t++) { free(cs->rho[t]); free(cs->gII[t]); }
        free(cs->rho); free(cs->gII);
    }
    free(cs->Iall);
}

/* PRD state of a prepared column: rho = 1 (CRD) and the redistribution
 * weights of every PRD line; returns 1 if any line uses PRD. */
static int prd_prepare(colstate *cs) {
    const orc_atom *a = cs->a;
    int any = 0;
    for (int t = 0; t < a->n_lines; t++) any |= a->tr[t].prd;
    if (!any) return 0;
    int nl = a->n_lines;
    cs->rho = calloc(nl, sizeof(double *));
    cs->gII = calloc(nl, sizeof(double *));
    for (int t = 0; t < nl; t++) {
        if (!a->tr[t].prd) continue;
        size_t n = (size_t)cs->N * a->tr[t].n_act;
        cs->rho[t] = malloc(sizeof(double) * n);
        for (size_t i = 0; i < n; i++) cs->rho[t][i] = 1.0;
        prd_tables(cs, t);
    }
    cs->Iall = malloc(sizeof(double) * (size_t)a->NL * cs->nmu * 2 * cs->N);
    return 1;
}

/* Accumulators of the preconditioned rates. */
typedef struct { double *P, *Q, *X; } rates;   /* P,Q: [T][N]; X: [T][T][N] */

/* Opacity terms of active transition t at ray (j, m, s), depth k:
 * V_lu, V_ul, U and the rate weight kappa = 4 pi W / (h nu_t). */
static void transition_terms(const colstate *cs, const double *n, int t, int ja, int j, int m, int s, int k,
                             double *Vlu, double *Vul, double *U, double *kap) {
    const orc_atom *a = cs->a;
    const orc_trans *tr = &a->tr[t];
    int L = a->L;
    double W = tr->wnu[ja] * 0.5 * cs->wmu[m];
    (void)n;
    if (tr->kind == 0) {
        double p = cs->phi[t][(((size_t)k * tr->n_act + ja) * cs->nmu + m) * 2 + s];
        /* emission (spontaneous and stimulated) with psi = rho phi for PRD lines */
        double ps = cs->rho && cs->rho[t] ? p * cs->rho[t][(size_t)k * tr->n_act + ja] : p;
        double c = PH * tr->nu0 / (4.0 * PPI);
        *Vlu = c * tr->Blu * p; *Vul = c * tr->Bul * ps; *U = c * tr->Aul * ps;
        *kap = 4.0 * PPI * W / (PH * tr->nu0);
    } else {
        double nu = a->nu[j];
        double alpha = tr->alpha0 * pow(tr->nu0 / nu, 3.0);
        double G = exp(cs->lnr[k * L + tr->l] - cs->lnr[k * L + tr->u]) * exp(-PH * nu / (PKB * cs->T[k]));
        *Vlu = alpha; *Vul = G * alpha; *U = 2.0 * PH * nu * nu * nu / (PC * PC) * G * alpha;
        *kap = 4.0 * PPI * W / (PH * nu);
    }
}

/* One formal-solution sweep over all rays with populations n.
 * mode 0: preconditioned rates; mode 1: zero-radiation rates (I_eff = 0,
 * Psi* = 0); mode 2: Psi* averaged per transition into psi_out[T][N]. */
static void sweep(const colstate *cs, const double *n, int mode, rates *R, double *psi_out, double *psi_ray) {
    const orc_atom *a = cs->a;
    int N = cs->N, L = a->L, T = a->T;
    double *chi = malloc(sizeof(double) * N), *eta = malloc(sizeof(double) * N), *S = malloc(sizeof(double) * N);
    double *etabg = malloc(sizeof(double) * N), *B = malloc(sizeof(double) * N);
    double *Ieff = malloc(sizeof(double) * N), *psi = malloc(sizeof(double) * N);
    double *Vlu = malloc(sizeof(double) * T * N), *Vul = malloc(sizeof(double) * T * N);
    double *U = malloc(sizeof(double) * T * N), *kap = malloc(sizeof(double) * T * N), *chit = malloc(sizeof(double) * T * N);
    int *act = malloc(sizeof(int) * (T ? T : 1)), *jact = malloc(sizeof(int) * (T ? T : 1));
    if (R) {
        memset(R->P, 0, sizeof(double) * T * N);
        memset(R->Q, 0, sizeof(double) * T * N);
        memset(R->X, 0, sizeof(double) * T * T * N);
    }
    if (psi_out) memset(psi_out, 0, sizeof(double) * T * N);
    for (int j = 0; j < a->NL; j++) {
        double nu = a->nu[j];
        int na = 0;
        for (int t = 0; t < T; t++) {
            const orc_trans *tr = &a->tr[t];
            for (int q = 0; q < tr->n_act; q++) if (tr->act[q] == j) { act[na] = t; jact[na] = q; na++; break; }
        }
        if (na == 0) continue;
        for (int k = 0; k < N; k++) {
            double chibg = cs->kbg[k] * (a->lam[j] / BG_LAMBDA_REF);
            B[k] = planck(nu, cs->T[k]);
            etabg[k] = chibg * B[k];
            chi[k] = chibg;
        }
        for (int m = 0; m < cs->nmu; m++) {
            double mu = cs->mu[m];
            for (int s = 0; s < 2; s++) {
                /* opacities of this ray */
                for (int k = 0; k < N; k++) {
                    double c = cs->kbg[k] * (a->lam[j] / BG_LAMBDA_REF), e = etabg[k];
                    for (int q = 0; q < na; q++) {
                        int t = act[q];
                        const orc_trans *tr = &a->tr[t];
                        size_t o = (size_t)q * N + k;
                        transition_terms(cs, n, t, jact[q], j, m, s, k, &Vlu[o], &Vul[o], &U[o], &kap[o]);
                        chit[o] = n[k * L + tr->l] * Vlu[o] - n[k * L + tr->u] * Vul[o];
                        c += chit[o];
                        e += n[k * L + tr->u] * U[o];
                    }
                    chi[k] = c; eta[k] = e; S[k] = e / c;
                }
                /* formal solution */
                if (mode == 1) {
                    for (int k = 0; k < N; k++) { Ieff[k] = 0.0; psi[k] = 0.0; }
                } else if (s == 0) {               /* downward: top to bottom */
                    double I = 0.0;
                    double *Is = (mode == 0 && cs->Iall) ? cs->Iall + (((size_t)j * cs->nmu + m) * 2 + s) * N : NULL;
                    Ieff[0] = 0.0; psi[0] = 0.0;
                    if (Is) Is[0] = I;
                    for (int k = 1; k < N; k++) {
                        double x = 0.5 * (chi[k - 1] + chi[k]) * (cs->z[k - 1] - cs->z[k]) / mu;
                        double e, wa, wb;
                        orc_sc_coefficients(x, &e, &wa, &wb);
                        Ieff[k] = I * e + wa * S[k - 1] + wb * etabg[k] / chi[k];
                        psi[k] = wb / chi[k];
                        I = I * e + wa * S[k - 1] + wb * S[k];
                        if (Is) Is[k] = I;
                    }
                } else {                           /* upward: bottom to top */
                    double dtv = 0.5 * (chi[N - 1] + chi[N - 2]) * (cs->z[N - 2] - cs->z[N - 1]);
                    double I = (dtv > 0.0) ? B[N - 1] + mu * (B[N - 1] - B[N - 2]) / dtv : B[N - 1];
                    double *Is = (mode == 0 && cs->Iall) ? cs->Iall + (((size_t)j * cs->nmu + m) * 2 + s) * N : NULL;
                    Ieff[N - 1] = I; psi[N - 1] = 0.0;
                    if (Is) Is[N - 1] = I;
                    for (int k = N - 2; k >= 0; k--) {
                        double x = 0.5 * (chi[k + 1] + chi[k]) * (cs->z[k] - cs->z[k + 1]) / mu;
                        double e, wa, wb;
                        orc_sc_coefficients(x, &e, &wa, &wb);
                        Ieff[k] = I * e + wa * S[k + 1] + wb * etabg[k] / chi[k];
                        psi[k] = wb / chi[k];
                        I = I * e + wa * S[k + 1] + wb * S[k];
                        if (Is) Is[k] = I;
                    }
                }
                if (psi_ray)
                    for (int k = 0; k < N; k++) psi_ray[(((size_t)k * a->NL + j) * cs->nmu + m) * 2 + s] = psi[k];
                /* accumulation */
                for (int q = 0; q < na; q++) {
                    int t = act[q];
                    for (int k = 0; k < N; k++) {
                        size_t o = (size_t)q * N + k;
                        if (mode == 2) {
                            const orc_trans *tr = &a->tr[t];
                            double W = tr->wnu[jact[q]] * 0.5 * cs->wmu[m];
                            double om;
                            if (tr->kind == 0) om = W * cs->phi[t][(((size_t)k * tr->n_act + jact[q]) * cs->nmu + m) * 2 + s];
                            else { double ws = 0.0; for (int i = 0; i < tr->n_act; i++) ws += tr->wnu[i]; om = W / ws; }
                            psi_out[t * N + k] += om * psi[k];
                            continue;
                        }
                        R->P[t * N + k] += kap[o] * Vlu[o] * Ieff[k];
                        R->Q[t * N + k] += kap[o] * (U[o] * (1.0 - chit[o] * psi[k]) + Vul[o] * Ieff[k]);
                        for (int q2 = 0; q2 < na; q2++) {
                            if (q2 == q) continue;
                            int t2 = act[q2];
                            R->X[((size_t)t * T + t2) * N + k] += kap[o] * chit[o] * psi[k] * U[(size_t)q2 * N + k];
                        }
                    }
                }
            }
        }
    }
    free(chi); free(eta); free(S); free(etabg); free(B); free(Ieff); free(psi);
    free(Vlu); free(Vul); free(U); free(kap); free(chit); free(act); free(jact);
}

/* ------------------------------------------------------------------ */
/* partial frequency redistribution                                     */
/* ------------------------------------------------------------------ */
static int prd_on(const colstate *cs, int t) { return cs->rho && cs->rho[t]; }

/* Redistribution weights of PRD line t at every depth point:
 * g(j', j) = w_j' R_II(x_j', x_j) / sum_j'' w_j'' R_II(x_j'', x_j), x the
 * rest-frame frequency offset in Doppler widths of the point, w the
 * line's trapezoid frequency weights.  With these weights a constant
 * mean intensity is redistributed into itself exactly. */
static void prd_tables(colstate *cs, int t) {
    const orc_atom *a = cs->a;
    const orc_trans *tr = &a->tr[t];
    int N = cs->N, na = tr->n_act;
    double *g = malloc(sizeof(double) * (size_t)N * na * na);
    double *x = malloc(sizeof(double) * na), *R = malloc(sizeof(double) * na * na);
    for (int k = 0; k < N; k++) {
        double dnd = cs->dnuD[t * N + k], ad = cs->adamp[t * N + k];
        for (int j = 0; j < na; j++) x[j] = (a->nu[tr->act[j]] - tr->nu0) / dnd;
        for (int j = 0; j < na; j++)
            for (int j2 = 0; j2 <= j; j2++) R[j * na + j2] = R[j2 * na + j] = orc_rII(ad, x[j], x[j2]);
        for (int j = 0; j < na; j++) {
            double sum = 0.0;
            for (int j2 = 0; j2 < na; j2++) sum += tr->wnu[j2] * R[j2 * na + j];
            for (int j2 = 0; j2 < na; j2++) g[((size_t)k * na + j) * na + j2] = tr->wnu[j2] * R[j2 * na + j] / sum;
        }
    }
    free(x); free(R);
    cs->gII[t] = g;
}

/* Actual radiative rate coefficients of transition t at depth k with the
 * intensities of the last sweep: upward (per particle in l) and downward
 * (per particle in u), emission with the current rho. */
static void actual_rates(const colstate *cs, int t, int k, double *up, double *down) {
    const orc_atom *a = cs->a;
    const orc_trans *tr = &a->tr[t];
    int N = cs->N;
    double ru = 0.0, rd = 0.0;
    for (int ja = 0; ja < tr->n_act; ja++) {
        int j = tr->act[ja];
        for (int m = 0; m < cs->nmu; m++) for (int s = 0; s < 2; s++) {
            double Vlu, Vul, U, kap;
            transition_terms(cs, NULL, t, ja, j, m, s, k, &Vlu, &Vul, &U, &kap);
            double I = cs->Iall[(((size_t)j * cs->nmu + m) * 2 + s) * N + k];
            ru += kap * Vlu * I;
            rd += kap * (U + Vul * I);
        }
    }
    *up = ru; *down = rd;
}

/* rho update of every PRD line after iteration `it` (Uitenbroek 2001,
 * angle-averaged PRD; the emission profile of a line whose upper level u
 * is populated partly by coherent scattering), from the intensities of the
 * iteration's formal solution and the new populations n:
 *   rho(j) = 1 + gamma n_l B_lu / (n_u P_u) [sum_j' g(j', j) J(j') - Jbar],
 * J(j') = sum over angles and directions of (w_mu / 2) I, Jbar the
 * profile-weighted mean intensity sum_rays W phi I, P_u the total rate out
 * of u (radiative with the sweep's intensities and the current rho, plus
 * collisional with factor cf), gamma = P_u / (P_u + Q_E) the coherent
 * fraction, Q_E = c_el n_H.  Then PRD switching (Sec. 2.3, Eq. 1):
 * rho' = rho eps + (1 - eps), eps = min(1, eps0 it^2) (eps0 <= 0: 1);
 * negative rho' count as 0; and rho' is normalised so that
 * sum_rays W phi rho' = 1 (the emission profile integrates to 1, as the
 * absorption profile does); where that sum is not positive (every rho'
 * clamped), rho = 1 (CRD) at that point. */
static void prd_update(colstate *cs, const double *n, int it, double eps0, double cf) {
    const orc_atom *a = cs->a;
    int N = cs->N, L = a->L, T = a->T;
    double eps = 1.0;
    if (eps0 > 0.0) { eps = eps0 * (double)it * (double)it; if (eps > 1.0) eps = 1.0; }
    double **newrho = calloc(a->n_lines ? a->n_lines : 1, sizeof(double *));
    for (int t = 0; t < a->n_lines; t++) {
        if (!prd_on(cs, t)) continue;
        const orc_trans *tr = &a->tr[t];
        int na = tr->n_act, u = tr->u, l = tr->l;
        double *nr = malloc(sizeof(double) * (size_t)N * na), *J = malloc(sizeof(double) * na);
        for (int k = 0; k < N; k++) {
            /* total rate out of the upper level */
            double Pu = 0.0;
            for (int t2 = 0; t2 < T; t2++) {
                if (a->tr[t2].u != u && a->tr[t2].l != u) continue;
                double up, down;
                actual_rates(cs, t2, k, &up, &down);
                Pu += (a->tr[t2].u == u) ? down : up;
            }
            for (int i = 0; i < L; i++) if (i != u) Pu += cs->C[(k * L + u) * L + i] * cf;
            double gam = Pu / (Pu + tr->c_el * cs->nH[k]);
            double nl = n[k * L + l], nu = n[k * L + u];
            double fac = gam * nl * tr->Blu / (nu * Pu);
            /* angle-averaged and profile-weighted mean intensities */
            double Jbar = 0.0;
            for (int ja = 0; ja < na; ja++) {
                int j = tr->act[ja];
                J[ja] = 0.0;
                for (int m = 0; m < cs->nmu; m++) for (int s = 0; s < 2; s++) {
                    double I = cs->Iall[(((size_t)j * cs->nmu + m) * 2 + s) * N + k];
                    J[ja] += 0.5 * cs->wmu[m] * I;
                    Jbar += tr->wnu[ja] * 0.5 * cs->wmu[m] * cs->phi[t][(((size_t)k * na + ja) * cs->nmu + m) * 2 + s] * I;
                }
            }
            double norm = 0.0;
            for (int ja = 0; ja < na; ja++) {
                double sJ = 0.0;
                for (int j2 = 0; j2 < na; j2++) sJ += cs->gII[t][((size_t)k * na + ja) * na + j2] * J[j2];
                double r = isfinite(fac) ? 1.0 + fac * (sJ - Jbar) : 1.0;
                r = r * eps + (1.0 - eps);
                if (!(r > 0.0)) r = 0.0;
                nr[(size_t)k * na + ja] = r;
                for (int m = 0; m < cs->nmu; m++) for (int s = 0; s < 2; s++)
                    norm += tr->wnu[ja] * 0.5 * cs->wmu[m] * cs->phi[t][(((size_t)k * na + ja) * cs->nmu + m) * 2 + s] * r;
            }
            /* no positive emission left (every rho' clamped to 0): CRD at this point */
            for (int ja = 0; ja < na; ja++)
                nr[(size_t)k * na + ja] = (norm > 0.0 && isfinite(norm)) ? nr[(size_t)k * na + ja] / norm : 1.0;
        }
        free(J);
        newrho[t] = nr;
    }
    /* every line's rates above used the previous rho: replace them only now */
    for (int t = 0; t < a->n_lines; t++)
        if (newrho[t]) { free(cs->rho[t]); cs->rho[t] = newrho[t]; }
    free(newrho);
}

/* Statistical equilibrium at every depth; returns 0 or -1 on a singular system. */
/* Collisional-radiative switching (Sec. 2.3; Hummer & Voels 1988): the
 * collision rates of iteration it (1, 2, ...) are multiplied by
 * f0 / 10^(it-1) while that exceeds 1, by 1 afterwards.  The factor is
 * formed by repeated division by 10 (the same IEEE operations in any
 * implementation). */
double orc_crs_factor(double f0, int it) {
    double f = f0;
    for (int i = 1; i < it && f > 1.0; i++) f /= 10.0;
    return f > 1.0 ? f : 1.0;
}

/* SE at every depth point with the collision rates times cf. */
static int solve_se(const colstate *cs, const rates *R, const double *nold, double *nnew, double cf) {
    const orc_atom *a = cs->a;
    int N = cs->N, L = a->L, T = a->T;
    double *G = malloc(sizeof(double) * L * L), *b = malloc(sizeof(double) * L);
    int rc = 0;
    for (int k = 0; k < N; k++) {
        memset(G, 0, sizeof(double) * L * L);
        for (int t = 0; t < T; t++) {
            int l = a->tr[t].l, u = a->tr[t].u;
            double P = R->P[t * N + k], Q = R->Q[t * N + k];
            G[u * L + l] += P; G[l * L + l] -= P;
            G[l * L + u] += Q; G[u * L + u] -= Q;
            for (int t2 = 0; t2 < T; t2++) {
                if (t2 == t) continue;
                double X = R->X[((size_t)t * T + t2) * N + k];
                if (X == 0.0) continue;
                int u2 = a->tr[t2].u;
                G[u * L + u2] += X; G[l * L + u2] -= X;
            }
        }
        for (int i = 0; i < L; i++) for (int j = 0; j < L; j++) {
            if (i == j) continue;
            double c = cs->C[(k * L + i) * L + j] * cf;
            G[j * L + i] += c; G[i * L + i] -= c;
        }
        int istar = 0;
        for (int i = 1; i < L; i++) if (nold[k * L + i] > nold[k * L + istar]) istar = i;
        for (int j = 0; j < L; j++) { G[istar * L + j] = 1.0; b[j] = 0.0; }
        b[istar] = cs->ntot[k];
        if (gauss_solve(L, G, b)) { rc = -1; }
        for (int i = 0; i < L; i++) nnew[k * L + i] = b[i];
    }
    free(G); free(b);
    return rc;
}

/* Emergent intensity at mu = 1 (vertical, upward) for every wavelength. */
static void emergent(const colstate *cs, const double *n, double *spec) {
    const orc_atom *a = cs->a;
    int N = cs->N, L = a->L;
    double *chi = malloc(sizeof(double) * N), *S = malloc(sizeof(double) * N), *B = malloc(sizeof(double) * N);
    for (int j = 0; j < a->NL; j++) {
        double nu = a->nu[j];
        for (int k = 0; k < N; k++) {
            double c = cs->kbg[k] * (a->lam[j] / BG_LAMBDA_REF);
            B[k] = planck(nu, cs->T[k]);
            double e = c * B[k];
            for (int t = 0; t < a->T; t++) {
                const orc_trans *tr = &a->tr[t];
                if (!(a->lam[j] >= tr->lam_min && a->lam[j] <= tr->lam_max)) continue;
                double Vlu, Vul, U;
                if (tr->kind == 0) {
                    double p = line_profile(a, t, cs, k, nu, 1.0) / cs->norm[t * N + k];
                    double ps = p;
                    if (cs->rho && cs->rho[t]) {
                        int ja = 0;
                        while (tr->act[ja] != j) ja++;
                        ps = p * cs->rho[t][(size_t)k * tr->n_act + ja];
                    }
                    double cc = PH * tr->nu0 / (4.0 * PPI);
                    Vlu = cc * tr->Blu * p; Vul = cc * tr->Bul * ps; U = cc * tr->Aul * ps;
                } else {
                    double alpha = tr->alpha0 * pow(tr->nu0 / nu, 3.0);
                    double G = exp(cs->lnr[k * L + tr->l] - cs->lnr[k * L + tr->u]) * exp(-PH * nu / (PKB * cs->T[k]));
                    Vlu = alpha; Vul = G * alpha; U = 2.0 * PH * nu * nu * nu / (PC * PC) * G * alpha;
                }
                c += n[k * L + tr->l] * Vlu - n[k * L + tr->u] * Vul;
                e += n[k * L + tr->u] * U;
            }
            chi[k] = c; S[k] = e / c;
        }
        double dtv = 0.5 * (chi[N - 1] + chi[N - 2]) * (cs->z[N - 2] - cs->z[N - 1]);
        double I = (dtv > 0.0) ? B[N - 1] + (B[N - 1] - B[N - 2]) / dtv : B[N - 1];
        for (int k = N - 2; k >= 0; k--) {
            double x = 0.5 * (chi[k + 1] + chi[k]) * (cs->z[k] - cs->z[k + 1]);
            double e, wa, wb;
            orc_sc_coefficients(x, &e, &wa, &wb);
            I = I * e + wa * S[k + 1] + wb * S[k];
        }
        spec[j] = I;
    }
    free(chi); free(S); free(B);
}

/* Ng extrapolation of order M from the ring of the last M+2 iterates
 * (x[0] newest).  Returns 1 and writes out if applied, 0 if skipped. */
int orc_ng_step(int M, int n, double *const *x, double *out) {
    if (M != 2) return 0;
    double A11 = 0, A12 = 0, A22 = 0, b1 = 0, b2 = 0;
    for (int i = 0; i < n; i++) {
        double w = 1.0 / (x[0][i] * x[0][i]);
        double d0 = x[0][i] - x[1][i], d1 = x[1][i] - x[2][i], d2 = x[2][i] - x[3][i];
        double e1 = d0 - d1, e2 = d0 - d2;
        A11 += w * e1 * e1; A12 += w * e1 * e2; A22 += w * e2 * e2;
        b1 += w * d0 * e1; b2 += w * d0 * e2;
    }
    double det = A11 * A22 - A12 * A12;
    if (!(fabs(det) > 1e-14 * A11 * A22)) return 0;
    double a1 = (b1 * A22 - b2 * A12) / det, a2 = (b2 * A11 - b1 * A12) / det;
    for (int i = 0; i < n; i++) {
        double v = (1.0 - a1 - a2) * x[0][i] + a1 * x[1][i] + a2 * x[2][i];
        if (!(v > 0.0)) return 0;
    }
    for (int i = 0; i < n; i++) out[i] = (1.0 - a1 - a2) * x[0][i] + a1 * x[1][i] + a2 * x[2][i];
    return 1;
}

/* Stopping rule.  Sec. 2.3 measures convergence by the maximum relative
 * population change Delta_k of iteration k; the column has converged when
 * Delta_k < tol.  With tol_fp > 0 the distance to the fixed point that the
 * last two changes imply is bounded as well: for a linear iteration with
 * contraction factor r = Delta_k / Delta_{k-1} the remaining distance is
 * Delta_k r / (1 - r), which must fall below tol_fp; it needs
 * Delta_k < Delta_{k-1} and is tested as Delta_k^2 < tol_fp (Delta_{k-1} -
 * Delta_k), with no division.  The ratio is that of two plain iterations:
 * when the previous iteration ended with an Ng extrapolation, or at the
 * first iteration, there is no ratio and only Delta_k = 0 passes.  (This
 * bound is a reading: the paper states the threshold on Delta only.) */
static int converged_at(double d, double dprev, double tol, double tol_fp) {
    if (!(d < tol)) return 0;
    if (!(tol_fp > 0.0)) return 1;
    if (dprev < 0.0) return d == 0.0;
    return d < dprev && d * d < tol_fp * (dprev - d);
}

/* Column data the method can use: finite positive T, n_e, n_H, finite
 * velocities, non-negative microturbulence and strictly decreasing z. */
static int column_valid(int N, const double *z, const double *T, const double *ne, const double *nH,
                        const double *vz, const double *vt) {
    for (int k = 0; k < N; k++) {
        if (!(isfinite(T[k]) && T[k] > 0.0 && isfinite(ne[k]) && ne[k] > 0.0 && isfinite(nH[k]) && nH[k] > 0.0))
            return 0;
        if (!(isfinite(vz[k]) && isfinite(vt[k]) && vt[k] >= 0.0 && isfinite(z[k]))) return 0;
        if (k > 0 && !(z[k] < z[k - 1])) return 0;
    }
    return 1;
}

/* Escape probability of the escape-probability start: (1 - e^-tau)/tau,
 * the fraction of photons created at vertical optical depth tau that
 * leave a uniform layer of that thickness (1 at tau = 0). */
static double escape_probability(double tau) { return tau > 0.0 ? -expm1(-tau) / tau : 1.0; }

/* Escape-probability start (Sec. 2.3, "Different starting solutions":
 * populations from a few statistical-equilibrium iterations with an
 * assumed probability of photon escape).  Starting from LTE, each of the
 * esc_iter iterations
 *   1. takes, for every transition, the vertical optical depth from the top
 *      at its reference frequency with the current populations: for a line
 *      chi = (h nu0 / 4 pi)(n_l B_lu - n_u B_ul) phi(nu0), phi(nu0) the
 *      rest-frame line-centre profile H(a, 0) / (sqrt(pi) Delta nu_D), for a
 *      continuum chi = (n_l - n_u G(nu_edge)) alpha(nu_edge); negative
 *      opacities count as 0; tau by the trapezoid rule in z from tau = 0
 *      at the top point;
 *   2. solves the rate equations with the spontaneous rate of every
 *      transition times its escape probability beta(tau) and no other
 *      radiative rate (net radiative bracket), plus collisions.
 * beta = 1 everywhere is the zero-radiation start.  zr holds the
 * zero-radiation rates (P = 0, Q' the spontaneous rates); n is updated in
 * place. */
static int escape_start(const colstate *cs, const rates *zr, int n_it, double *n) {
    const orc_atom *a = cs->a;
    int N = cs->N, L = a->L, T = a->T;
    rates R;
    R.P = calloc((size_t)T * N, sizeof(double));
    R.Q = malloc(sizeof(double) * T * N);
    R.X = calloc((size_t)T * T * N, sizeof(double));
    double *chi = malloc(sizeof(double) * N), *nn = malloc(sizeof(double) * N * L);
    int rc = 0;
    for (int s = 0; s < n_it && rc == 0; s++) {
        for (int t = 0; t < T; t++) {
            const orc_trans *tr = &a->tr[t];
            for (int k = 0; k < N; k++) {
                double nl = n[k * L + tr->l], nu = n[k * L + tr->u], c;
                if (tr->kind == 0) {
                    double dnd = cs->dnuD[t * N + k];
                    double H0 = tr->voigt ? orc_voigt_H(cs->adamp[t * N + k], 0.0) : 1.0;
                    c = PH * tr->nu0 / (4.0 * PPI) * (nl * tr->Blu - nu * tr->Bul) * H0 / (sqrt(PPI) * dnd);
                } else {
                    double G = exp(cs->lnr[k * L + tr->l] - cs->lnr[k * L + tr->u]) * exp(-PH * tr->nu0 / (PKB * cs->T[k]));
                    c = (nl - nu * G) * tr->alpha0;
                }
                chi[k] = c > 0.0 ? c : 0.0;
            }
            double tau = 0.0;
            for (int k = 0; k < N; k++) {
                if (k > 0) tau += 0.5 * (chi[k - 1] + chi[k]) * (cs->z[k - 1] - cs->z[k]);
                R.Q[t * N + k] = zr->Q[t * N + k] * escape_probability(tau);
            }
        }
        if (solve_se(cs, &R, n, nn, 1.0)) rc = -1;
        memcpy(n, nn, sizeof(double) * N * L);
    }
    free(R.P); free(R.Q); free(R.X); free(chi); free(nn);
    return rc;
}

/* Solve one column.  Arrays of the column: N points, top first.
 * Outputs (any may be NULL except pops): pops[N][L], history[max_iter],
 * spectrum[NL], psi_star[T][N], prd_rho (the final rho of every PRD line,
 * in line order, [N][n_act] each); n_iter and status scalars.
 * status: 0 converged, 1 iteration limit, 2 non-finite or non-positive
 * populations, 3 singular rate matrix, 4 invalid column data (outputs
 * NaN, no iteration). */
int orc_solve_column(const orc_atom *a, int N, const double *z, const double *T, const double *ne,
                     const double *nH, const double *vz, const double *vt, const double *init_pops,
                     const orc_opts *o, double *pops, double *history, int *n_iter, int *status,
                     double *spectrum, double *psi_star, double *prd_rho) {
    if (N < 2) FAIL(-3, "need at least 2 depth points");
    if (o->n_mu < 1 || o->n_mu > 16) FAIL(-3, "n_mu out of range");
    if (o->ng_order != 0 && o->ng_order != 2) FAIL(-3, "only Ng order 2 (or 0 = off) is implemented");
    if (!column_valid(N, z, T, ne, nH, vz, vt)) {
        for (int i = 0; i < N * a->L; i++) pops[i] = NAN;
        if (history) for (int i = 0; i < o->max_iter; i++) history[i] = NAN;
        if (spectrum) for (int j = 0; j < a->NL; j++) spectrum[j] = NAN;
        if (psi_star) for (int i = 0; i < a->T * N; i++) psi_star[i] = NAN;
        *n_iter = 0;
        *status = 4;
        return 0;
    }
    colstate cs = {0};
    cs.a = a; cs.N = N; cs.nmu = o->n_mu; cs.z = z; cs.T = T; cs.ne = ne; cs.nH = nH; cs.vz = vz; cs.vt = vt;
    cs.mu = malloc(sizeof(double) * o->n_mu); cs.wmu = malloc(sizeof(double) * o->n_mu);
    orc_gauss_legendre(o->n_mu, cs.mu, cs.wmu);
    column_prepare(&cs, o->coll_scale > 0 ? o->coll_scale : 1.0);
    const int prd = o->prd ? prd_prepare(&cs) : 0;
    int L = a->L, Tn = a->T, NV = N * L;
    rates R;
    R.P = malloc(sizeof(double) * (Tn ? Tn : 1) * N); R.Q = malloc(sizeof(double) * (Tn ? Tn : 1) * N);
    R.X = malloc(sizeof(double) * (Tn ? Tn * Tn : 1) * N);
    double *n = malloc(sizeof(double) * NV), *nse = malloc(sizeof(double) * NV);
    int M = o->ng_order, ring_n = M + 2;
    double *ring[8] = {0};
    if (M > 0) for (int i = 0; i < ring_n; i++) ring[i] = malloc(sizeof(double) * NV);
    int ng_count = 0;

    memcpy(n, cs.nstar, sizeof(double) * NV);
    if (o->start == 1) {
        sweep(&cs, n, 1, &R, NULL, NULL);
        solve_se(&cs, &R, cs.nstar, n, 1.0);
    } else if (o->start == 2 && init_pops) {
        memcpy(n, init_pops, sizeof(double) * NV);
    } else if (o->start == 3) {
        sweep(&cs, n, 1, &R, NULL, NULL);
        escape_start(&cs, &R, o->esc_iter, n);
    }
    if (history) for (int i = 0; i < o->max_iter; i++) history[i] = NAN;
    int st = 1, it;
    double dprev = -1.0;   /* change of the previous iteration (none yet) */
    for (it = 1; it <= o->max_iter; it++) {
        sweep(&cs, n, 0, &R, NULL, NULL);
        /* while collisions are switched (cf > 1) the iterate solves another
         * problem: it may not end the iteration or enter Ng's history */
        const double cf = orc_crs_factor(o->crs_f0, it);
        int bad = solve_se(&cs, &R, n, nse, cf);
        double dmax = 0.0;
        int finite = 1;
        for (int i = 0; i < NV; i++) {
            if (!isfinite(nse[i]) || !(nse[i] > 0.0)) { finite = 0; break; }
            double d = fabs(nse[i] - n[i]) / nse[i];
            if (d > dmax) dmax = d;
        }
        if (history) history[it - 1] = finite ? dmax : NAN;
        if (bad) { st = 3; break; }
        if (!finite) { st = 2; break; }
        memcpy(n, nse, sizeof(double) * NV);
        if (cf == 1.0 && converged_at(dmax, dprev, o->tol, o->tol_fp)) { st = 0; break; }
        dprev = dmax;
        if (M > 0 && it >= o->ng_delay && cf == 1.0) {
            /* push newest iterate */
            double *last = ring[ring_n - 1];
            for (int i = ring_n - 1; i > 0; i--) ring[i] = ring[i - 1];
            ring[0] = last;
            memcpy(ring[0], nse, sizeof(double) * NV);
            ng_count++;
            /* an attempt every max(period, M+2) collected iterates; the
             * history restarts after each attempt, applied or skipped */
            int need = o->ng_period > ring_n ? o->ng_period : ring_n;
            if (ng_count >= need) {
                /* an applied extrapolation leaves no contraction ratio for
                 * the next iteration's stopping test */
                if (orc_ng_step(M, NV, ring, n)) dprev = -1.0;
                ng_count = 0;
            }
        }
        /* PRD: rho from this iteration's radiation field and the new
         * populations, for the next formal solution (none after the last
         * iteration: the emergent spectrum keeps the rho of the last one) */
        if (prd && it < o->max_iter) prd_update(&cs, n, it, o->prd_eps0, cf);
    }
    if (it > o->max_iter) it = o->max_iter;
    *n_iter = it;
    *status = st;
    memcpy(pops, n, sizeof(double) * NV);
    if (spectrum) emergent(&cs, n, spectrum);
    if (psi_star) sweep(&cs, n, 2, NULL, psi_star, NULL);
    if (prd_rho && prd)
        for (int t = 0; t < a->n_lines; t++)
            if (cs.rho[t]) {
                size_t m = (size_t)N * a->tr[t].n_act;
                memcpy(prd_rho, cs.rho[t], sizeof(double) * m);
                prd_rho += m;
            }
    for (int i = 0; i < 8; i++) free(ring[i]);
    free(n); free(nse); free(R.P); free(R.Q); free(R.X);
    column_release(&cs);
    free(cs.mu); free(cs.wmu);
    return 0;
}

/* Thin helpers for tests: prepared-column quantities. */
int orc_column_profile_norm(const orc_atom *a, int N, const double *z, const double *T, const double *ne,
                            const double *nH, const double *vz, const double *vt, int n_mu, double *nstar,
                            double *norm) {
    colstate cs = {0};
    cs.a = a; cs.N = N; cs.nmu = n_mu; cs.z = z; cs.T = T; cs.ne = ne; cs.nH = nH; cs.vz = vz; cs.vt = vt;
    cs.mu = malloc(sizeof(double) * n_mu); cs.wmu = malloc(sizeof(double) * n_mu);
    orc_gauss_legendre(n_mu, cs.mu, cs.wmu);
    column_prepare(&cs, 1.0);
    if (nstar) memcpy(nstar, cs.nstar, sizeof(double) * N * a->L);
    if (norm) memcpy(norm, cs.norm, sizeof(double) * N * a->n_lines);
    column_release(&cs);
    free(cs.mu); free(cs.wmu);
    return 0;
}

/* Doppler widths (Hz) and Voigt damping parameters of every line at every
 * depth point of a column, [n_lines][N] each, as the column preparation
 * computes them (tests only). */
int orc_column_damping(const orc_atom *a, int N, const double *z, const double *T, const double *ne,
                       const double *nH, const double *vz, const double *vt, double *dnuD, double *adamp) {
    colstate cs = {0};
    cs.a = a; cs.N = N; cs.nmu = 1; cs.z = z; cs.T = T; cs.ne = ne; cs.nH = nH; cs.vz = vz; cs.vt = vt;
    cs.mu = malloc(sizeof(double)); cs.wmu = malloc(sizeof(double));
    orc_gauss_legendre(1, cs.mu, cs.wmu);
    column_prepare(&cs, 1.0);
    if (dnuD) memcpy(dnuD, cs.dnuD, sizeof(double) * N * a->n_lines);
    if (adamp) memcpy(adamp, cs.adamp, sizeof(double) * N * a->n_lines);
    column_release(&cs);
    free(cs.mu); free(cs.wmu);
    return 0;
}

/* One rho update of a prepared column with every ray's intensity set to
 * I_const, populations pops and switching (eps0, it); rho of the PRD lines
 * out as in orc_solve_column (tests only). */
int orc_column_prd_rho(const orc_atom *a, int N, const double *z, const double *T, const double *ne,
                       const double *nH, const double *vz, const double *vt, int n_mu, const double *pops,
                       double I_const, double eps0, int it, double *rho_out) {
    colstate cs = {0};
    cs.a = a; cs.N = N; cs.nmu = n_mu; cs.z = z; cs.T = T; cs.ne = ne; cs.nH = nH; cs.vz = vz; cs.vt = vt;
    cs.mu = malloc(sizeof(double) * n_mu); cs.wmu = malloc(sizeof(double) * n_mu);
    orc_gauss_legendre(n_mu, cs.mu, cs.wmu);
    column_prepare(&cs, 1.0);
    if (!prd_prepare(&cs)) { column_release(&cs); free(cs.mu); free(cs.wmu); FAIL(-3, "no PRD line"); }
    size_t nI = (size_t)a->NL * n_mu * 2 * N;
    for (size_t i = 0; i < nI; i++) cs.Iall[i] = I_const;
    prd_update(&cs, pops, it, eps0, 1.0);
    for (int t = 0; t < a->n_lines; t++)
        if (cs.rho[t]) {
            size_t m = (size_t)N * a->tr[t].n_act;
            memcpy(rho_out, cs.rho[t], sizeof(double) * m);
            rho_out += m;
        }
    column_release(&cs);
    free(cs.mu); free(cs.wmu);
    return 0;
}

/* ------------------------------------------------------------------ */
/* grid optimisation                                                    */
/* ------------------------------------------------------------------ */
/* Re-gridding of one column (Sec. 2.3, "Grid optimisation": more points
 * where temperature, velocity or optical depth change fast).  Reading (the
 * paper gives no formula): each interval i between points i-1 and i gets the
 * length
 *   d_i = sqrt((w_z dz_i / H)^2 + (w_T d ln T_i)^2 + (w_v dv_i)^2
 *              + (w_tau d ln(tau_i + tau_min))^2),
 * H the column's height range, tau the optical depth from the top at the
 * reference wavelength of the background law (trapezoid rule in z; 0 without
 * a background), tau_min = 1e-5; the n_out new points divide the summed
 * length into equal parts (first and last point kept), and every variable
 * is interpolated linearly in that length within its interval: z, v_z and
 * v_turb as they are, T, n_e and n_H in their logarithms.  The weights are
 * w[0..3] = (w_z, w_T, w_v [s/m], w_tau), each >= 0; the input must have z
 * strictly decreasing and T, n_e, n_H > 0, and the summed length must be
 * positive (error -3 otherwise). */
#define GRID_TAU_MIN 1.0e-5
int orc_optimize_grid(const orc_atom *a, int N, const double *z, const double *T, const double *ne,
                      const double *nH, const double *vz, const double *vt, int n_out, const double *w,
                      double *zo, double *To, double *neo, double *nHo, double *vzo, double *vto) {
    if (N < 2 || n_out < 2) FAIL(-3, "need at least 2 points in and out");
    for (int i = 0; i < 4; i++)
        if (!(w[i] >= 0.0 && isfinite(w[i]))) FAIL(-3, "grid weights must be finite and >= 0");
    for (int k = 0; k < N; k++) {
        if (!(T[k] > 0.0 && ne[k] > 0.0 && nH[k] > 0.0) || !isfinite(T[k] + ne[k] + nH[k] + vz[k] + vt[k] + z[k]))
            FAIL(-3, "depth point %d: T, n_e, n_H must be finite and > 0", k);
        if (k > 0 && !(z[k] < z[k - 1])) FAIL(-3, "z must decrease strictly (point %d)", k);
    }
    double *M = malloc(sizeof(double) * N);
    double H = z[0] - z[N - 1], tau = 0.0, kp = 0.0;
    M[0] = 0.0;
    for (int k = 0; k < N; k++) {
        double kap = a->bg_kind == 1 ? a->c_bg * nH[k] * ne[k] * pow(T[k], -1.5) * exp(BG_THETA / T[k]) : 0.0;
        if (k > 0) {
            double tprev = tau;
            tau += 0.5 * (kp + kap) * (z[k - 1] - z[k]);
            double dz = w[0] * (z[k - 1] - z[k]) / H;
            double dT = w[1] * (log(T[k]) - log(T[k - 1]));
            double dv = w[2] * (vz[k] - vz[k - 1]);
            double dt = w[3] * (log(tau + GRID_TAU_MIN) - log(tprev + GRID_TAU_MIN));
            M[k] = M[k - 1] + sqrt(dz * dz + dT * dT + dv * dv + dt * dt);
        }
        kp = kap;
    }
    if (!(M[N - 1] > 0.0 && isfinite(M[N - 1]))) {
        free(M);
        FAIL(-3, "the column's grid length is zero or not finite (all weights zero?)");
    }
    int k = 1;
    for (int j = 0; j < n_out; j++) {
        double target = M[N - 1] * (double)j / (double)(n_out - 1);
        if (j == n_out - 1) target = M[N - 1];
        while (k < N - 1 && M[k] < target) k++;
        double f = (target - M[k - 1]) / (M[k] - M[k - 1]);
        zo[j] = z[k - 1] + f * (z[k] - z[k - 1]);
        To[j] = exp(log(T[k - 1]) + f * (log(T[k]) - log(T[k - 1])));
        neo[j] = exp(log(ne[k - 1]) + f * (log(ne[k]) - log(ne[k - 1])));
        nHo[j] = exp(log(nH[k - 1]) + f * (log(nH[k]) - log(nH[k - 1])));
        vzo[j] = vz[k - 1] + f * (vz[k] - vz[k - 1]);
        vto[j] = vt[k - 1] + f * (vt[k] - vt[k - 1]);
    }
    /* the end points exactly */
    zo[0] = z[0]; To[0] = T[0]; neo[0] = ne[0]; nHo[0] = nH[0]; vzo[0] = vz[0]; vto[0] = vt[0];
    zo[n_out - 1] = z[N - 1]; To[n_out - 1] = T[N - 1]; neo[n_out - 1] = ne[N - 1]; nHo[n_out - 1] = nH[N - 1];
    vzo[n_out - 1] = vz[N - 1]; vto[n_out - 1] = vt[N - 1];
    free(M);
    return 0;
}

/* ------------------------------------------------------------------ */
/* polarised emergent spectrum                                          */
/* ------------------------------------------------------------------ */
/* Vertical, upward formal solution of the Stokes vector (I, Q, U, V) at one
 * wavelength (Sec. 2.1: the full Stokes vector from Zeeman splitting; the
 * paper names no polarised solver).  Reading: DELO with a linear effective
 * source function (Rees, Durrant & Murphy 1989).  With chi_I the total
 * opacity, K' = K / chi_I - 1 (zero diagonal) and S' = eps / chi_I, the
 * transfer equation along the optical depth reads dI/dtau = I - (S' - K' I);
 * taking the bracket linear in tau over each interval gives, from the
 * deeper point k+1 to point k with the short-characteristic weights of the
 * unpolarised solver (step x, e = exp(-x), w_a, w_b),
 *   (1 + w_b K'_k) I_k = (e - w_a K'_{k+1}) I_{k+1} + w_a S'_{k+1} + w_b S'_k,
 * a 4 x 4 system solved at every point.  The propagation matrix is
 *   K = [[eI, eQ, eU, eV], [eQ, eI, rV, -rU], [eU, -rV, eI, rQ], [eV, rU, -rQ, eI]].
 * Inputs per point: z, chi_I, K6 = (eQ, eU, eV, rQ, rU, rV) and
 * eps = (eps_I, eps_Q, eps_U, eps_V); Ibot enters at the bottom point. */
static void kprime(const double *K6, double chiI, double *Kp) {
    double eQ = K6[0] / chiI, eU = K6[1] / chiI, eV = K6[2] / chiI;
    double rQ = K6[3] / chiI, rU = K6[4] / chiI, rV = K6[5] / chiI;
    double M[16] = {0.0, eQ, eU, eV,
                    eQ, 0.0, rV, -rU,
                    eU, -rV, 0.0, rQ,
                    eV, rU, -rQ, 0.0};
    memcpy(Kp, M, sizeof M);
}

int orc_stokes_formal(int N, const double *z, const double *chiI, const double *K6, const double *eps,
                      const double *Ibot, double *Itop) {
    double I[4] = {Ibot[0], Ibot[1], Ibot[2], Ibot[3]};
    for (int k = N - 2; k >= 0; k--) {
        double x = 0.5 * (chiI[k + 1] + chiI[k]) * (z[k] - z[k + 1]);
        double e, wa, wb;
        orc_sc_coefficients(x, &e, &wa, &wb);
        double Kd[16], Kc[16];
        kprime(&K6[(k + 1) * 6], chiI[k + 1], Kd);
        kprime(&K6[k * 6], chiI[k], Kc);
        double rhs[4], M[16];
        for (int i = 0; i < 4; i++) {
            double s = e * I[i];
            for (int c = 0; c < 4; c++) s -= wa * Kd[i * 4 + c] * I[c];
            rhs[i] = s + wa * eps[(k + 1) * 4 + i] / chiI[k + 1] + wb * eps[k * 4 + i] / chiI[k];
            for (int c = 0; c < 4; c++) M[i * 4 + c] = (i == c ? 1.0 : 0.0) + wb * Kc[i * 4 + c];
        }
        if (gauss_solve(4, M, rhs)) FAIL(-3, "singular DELO system at point %d", k);
        for (int i = 0; i < 4; i++) I[i] = rhs[i];
    }
    for (int i = 0; i < 4; i++) Itop[i] = I[i];
    return 0;
}

/* Stokes vector of the vertical emergent spectrum of a column whose
 * populations n are given (the unpolarised emergent spectrum's opacities
 * and emissivities, the same profile normalisation and PRD ratio rho),
 * with a magnetic field of strength B [T], inclination incl to the
 * vertical (the line of sight) and azimuth azim [rad] at every depth.  A
 * line whose Zeeman pattern the atom gives contributes, per absorption
 * and emission coefficient (the scalar coefficients of the unpolarised
 * solve), the Zeeman profiles phi_q = sum of strength * H(a, v - shift v_L)
 * / (sqrt(pi) dnu_D) and psi_q (the same with the dispersion function L),
 * v_L the Larmor frequency in Doppler widths, combined as
 *   eta_I = [phi_0 sin^2(theta) + (phi_{+1} + phi_{-1})(1 + cos^2(theta))/2] / 2,
 *   eta_Q = [phi_0 - (phi_{+1} + phi_{-1})/2] sin^2(theta) cos(2 chi) / 2,
 *   eta_U = the same with sin(2 chi),  eta_V = (phi_{+1} - phi_{-1}) cos(theta) / 2,
 * and rho_Q, rho_U, rho_V likewise from psi_q; eps = emission coefficient
 * times (eta_I, eta_Q, eta_U, eta_V).  Other transitions and the background
 * are unpolarised.  Bottom: (B_nu + dB/dtau, 0, 0, 0), as the unpolarised
 * spectrum.  out: [NL][4]. */
/* Opacity chi_I, K6 and eps of one point k at wavelength j (see above). */
static void stokes_point(const colstate *cs, const double *n, const double *Bf, const double *incl,
                         const double *azim, int j, int k, double *chi, double *kk, double *ee, double *Bnu) {
    const orc_atom *a = cs->a;
    int N = cs->N, L = a->L;
    double nu = a->nu[j];
    double c = cs->kbg[k] * (a->lam[j] / BG_LAMBDA_REF);
    *Bnu = planck(nu, cs->T[k]);
    for (int i = 0; i < 6; i++) kk[i] = 0.0;
    ee[0] = c * *Bnu; ee[1] = ee[2] = ee[3] = 0.0;
    for (int t = 0; t < a->T; t++) {
        const orc_trans *tr = &a->tr[t];
        if (!(a->lam[j] >= tr->lam_min && a->lam[j] <= tr->lam_max)) continue;
        if (tr->kind == 0) {
            double rho = 1.0;
            if (cs->rho && cs->rho[t]) {
                int ja = 0;
                while (tr->act[ja] != j) ja++;
                rho = cs->rho[t][(size_t)k * tr->n_act + ja];
            }
            double cc = PH * tr->nu0 / (4.0 * PPI) / cs->norm[t * N + k];
            double cabs = cc * (n[k * L + tr->l] * tr->Blu - n[k * L + tr->u] * tr->Bul * rho);
            double cem = cc * n[k * L + tr->u] * tr->Aul * rho;
            if (tr->n_zc == 0) {
                double p = line_profile(a, t, cs, k, nu, 1.0);
                c += cabs * p;
                ee[0] += cem * p;
                continue;
            }
            double dnd = cs->dnuD[t * N + k], ad = cs->adamp[t * N + k];
            double v = (nu - tr->nu0 * (1.0 + cs->vz[k] / PC)) / dnd;
            double vL = PQE * Bf[k] / (4.0 * PPI * PME) / dnd;
            double ph[3] = {0, 0, 0}, ps[3] = {0, 0, 0};
            for (int i = 0; i < tr->n_zc; i++) {
                double vc = v - tr->zshift[i] * vL, H, Lf;
                orc_voigt_w(tr->voigt ? ad : 0.0, vc, &H, &Lf);
                if (!tr->voigt) H = exp(-vc * vc);
                ph[tr->zq[i] + 1] += tr->zstr[i] * H;
                ps[tr->zq[i] + 1] += tr->zstr[i] * Lf;
            }
            for (int q = 0; q < 3; q++) { ph[q] /= sqrt(PPI) * dnd; ps[q] /= sqrt(PPI) * dnd; }
            double ct = cos(incl[k]), st = sin(incl[k]), s2 = st * st;
            double c2 = cos(2.0 * azim[k]), sn2 = sin(2.0 * azim[k]);
            /* q = +1 is ph[2], q = -1 is ph[0] */
            double pI = 0.5 * (ph[1] * s2 + 0.5 * (ph[2] + ph[0]) * (1.0 + ct * ct));
            double pl = 0.5 * (ph[1] - 0.5 * (ph[2] + ph[0])) * s2;
            double pV = 0.5 * (ph[2] - ph[0]) * ct;
            double rl = 0.5 * (ps[1] - 0.5 * (ps[2] + ps[0])) * s2;
            double rV = 0.5 * (ps[2] - ps[0]) * ct;
            c += cabs * pI;
            kk[0] += cabs * pl * c2; kk[1] += cabs * pl * sn2; kk[2] += cabs * pV;
            kk[3] += cabs * rl * c2; kk[4] += cabs * rl * sn2; kk[5] += cabs * rV;
            ee[0] += cem * pI; ee[1] += cem * pl * c2; ee[2] += cem * pl * sn2; ee[3] += cem * pV;
        } else {
            double alpha = tr->alpha0 * pow(tr->nu0 / nu, 3.0);
            double G = exp(cs->lnr[k * L + tr->l] - cs->lnr[k * L + tr->u]) * exp(-PH * nu / (PKB * cs->T[k]));
            c += n[k * L + tr->l] * alpha - n[k * L + tr->u] * G * alpha;
            ee[0] += n[k * L + tr->u] * 2.0 * PH * nu * nu * nu / (PC * PC) * G * alpha;
        }
    }
    *chi = c;
}

static int stokes_emergent(const colstate *cs, const double *n, const double *Bf, const double *incl,
                           const double *azim, double *out) {
    const orc_atom *a = cs->a;
    int N = cs->N;
    double *chi = malloc(sizeof(double) * N), *K6 = malloc(sizeof(double) * N * 6);
    double *eps = malloc(sizeof(double) * N * 4), *B = malloc(sizeof(double) * N);
    int rc = 0;
    for (int j = 0; j < a->NL && !rc; j++) {
        for (int k = 0; k < N; k++) stokes_point(cs, n, Bf, incl, azim, j, k, &chi[k], &K6[k * 6], &eps[k * 4], &B[k]);
        double dtv = 0.5 * (chi[N - 1] + chi[N - 2]) * (cs->z[N - 2] - cs->z[N - 1]);
        double Ib[4] = {(dtv > 0.0) ? B[N - 1] + (B[N - 1] - B[N - 2]) / dtv : B[N - 1], 0.0, 0.0, 0.0};
        rc = orc_stokes_formal(N, cs->z, chi, K6, eps, Ib, &out[(size_t)j * 4]);
    }
    free(chi); free(K6); free(eps); free(B);
    return rc;
}

/* The Stokes spectrum of one column from given populations pops [N][L]
 * (and, for the lines the atom marks PRD, their final rho as
 * orc_solve_column returns it, or NULL for rho = 1), with the profile
 * normalisation of an n_mu-angle quadrature; stokes: [NL][4] (tests and
 * the benchmark's CPU leg only). */
int orc_stokes_column(const orc_atom *a, int N, const double *z, const double *T, const double *ne, const double *nH,
                      const double *vz, const double *vt, int n_mu, const double *Bf, const double *incl,
                      const double *azim, const double *pops, const double *prd_rho, double *stokes) {
    if (!column_valid(N, z, T, ne, nH, vz, vt)) FAIL(-3, "column data cannot be used");
    colstate cs = {0};
    cs.a = a; cs.N = N; cs.nmu = n_mu; cs.z = z; cs.T = T; cs.ne = ne; cs.nH = nH; cs.vz = vz; cs.vt = vt;
    cs.mu = malloc(sizeof(double) * n_mu); cs.wmu = malloc(sizeof(double) * n_mu);
    orc_gauss_legendre(n_mu, cs.mu, cs.wmu);
    column_prepare(&cs, 1.0);
    if (prd_rho) {
        cs.rho = calloc(a->n_lines ? a->n_lines : 1, sizeof(double *));
        cs.gII = calloc(a->n_lines ? a->n_lines : 1, sizeof(double *));
        for (int t = 0; t < a->n_lines; t++)
            if (a->tr[t].prd) {
                size_t m = (size_t)N * a->tr[t].n_act;
                cs.rho[t] = malloc(sizeof(double) * m);
                memcpy(cs.rho[t], prd_rho, sizeof(double) * m);
                prd_rho += m;
            }
    }
    int rc = stokes_emergent(&cs, pops, Bf, incl, azim, stokes);
    column_release(&cs);
    free(cs.mu); free(cs.wmu);
    return rc;
}

/* chi_I, K6 and eps (11 values) of point k at wavelength j of a column
 * with populations pops and rho = 1 (tests only). */
int orc_stokes_coefficients(const orc_atom *a, int N, const double *z, const double *T, const double *ne,
                            const double *nH, const double *vz, const double *vt, int n_mu, const double *Bf,
                            const double *incl, const double *azim, const double *pops, int j, int k, double *out) {
    if (j < 0 || j >= a->NL || k < 0 || k >= N) FAIL(-3, "point out of range");
    colstate cs = {0};
    cs.a = a; cs.N = N; cs.nmu = n_mu; cs.z = z; cs.T = T; cs.ne = ne; cs.nH = nH; cs.vz = vz; cs.vt = vt;
    cs.mu = malloc(sizeof(double) * n_mu); cs.wmu = malloc(sizeof(double) * n_mu);
    orc_gauss_legendre(n_mu, cs.mu, cs.wmu);
    column_prepare(&cs, 1.0);
    double Bnu;
    stokes_point(&cs, pops, Bf, incl, azim, j, k, &out[0], &out[1], &out[7], &Bnu);
    column_release(&cs);
    free(cs.mu); free(cs.wmu);
    return 0;
}

/* Psi* of every ray (Lambda* over chi, 0 at the ray's boundary point) of a
 * column with populations pops [N][L] (and the final rho of its PRD lines
 * as orc_solve_column returns it, or NULL), the diagonal that the
 * per-transition Psi* of orc_solve_column averages; out: [N][NL][n_mu][2]
 * (direction 0 down, 1 up) (tests only). */
int orc_column_psi_ray(const orc_atom *a, int N, const double *z, const double *T, const double *ne, const double *nH,
                       const double *vz, const double *vt, int n_mu, const double *pops, const double *prd_rho,
                       double *out) {
    if (!column_valid(N, z, T, ne, nH, vz, vt)) FAIL(-3, "column data cannot be used");
    colstate cs = {0};
    cs.a = a; cs.N = N; cs.nmu = n_mu; cs.z = z; cs.T = T; cs.ne = ne; cs.nH = nH; cs.vz = vz; cs.vt = vt;
    cs.mu = malloc(sizeof(double) * n_mu); cs.wmu = malloc(sizeof(double) * n_mu);
    orc_gauss_legendre(n_mu, cs.mu, cs.wmu);
    column_prepare(&cs, 1.0);
    if (prd_rho) {
        cs.rho = calloc(a->n_lines ? a->n_lines : 1, sizeof(double *));
        cs.gII = calloc(a->n_lines ? a->n_lines : 1, sizeof(double *));
        for (int t = 0; t < a->n_lines; t++)
            if (a->tr[t].prd) {
                size_t m = (size_t)N * a->tr[t].n_act;
                cs.rho[t] = malloc(sizeof(double) * m);
                memcpy(cs.rho[t], prd_rho, sizeof(double) * m);
                prd_rho += m;
            }
    }
    double *tmp = malloc(sizeof(double) * (size_t)a->T * N);
    sweep(&cs, pops, 2, NULL, tmp, out);
    free(tmp);
    column_release(&cs);
    free(cs.mu); free(cs.wmu);
    return 0;
}
