/*
 * oracle.c -- plain, slow, double-precision reference for the recursive
 * multibaryon correlator method of Guenther, Toth and Varnhorst,
 * "A recursive approach to determine correlation functions in multibaryon
 * systems" (arXiv:1301.4895).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the package smoke check and
 * the CPU-baseline leg of the benchmark may load this library.  It shares no
 * code, header, table or constant generator with the HIP library; it builds
 * every object it needs (Dirac matrices, the G tensors, blocks, the tensor L,
 * the required-component sets and the operation lists) from the definitions in
 * the paper, by exhaustive enumeration.
 *
 * Index conventions (all 0-based; the paper leaves them open, Sec. 2, 6):
 *   quark spin-colour      kappa = 3*spin + colour            (0..11)
 *   with N_s sources       xi    = N_s*kappa + s              (0..12 N_s - 1)
 *   baryon spin (+source)  chi / psi = N_s*alpha + s           (0..4 N_s - 1)
 *   propagator             S[x][s][row][kappa], row = 3*spin + colour of the
 *                          sink quark, kappa the source spin-colour of source s.
 *   sink weights           w[s'][x] for sink function s'; NULL means w = 1.
 * Complex numbers are C99 `double complex` (layout re, im).
 */
#include <complex.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

/* Threads used by the parallel loops (over independent outputs only). */
void orc_set_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }
int orc_max_threads(void) { return omp_get_max_threads(); }

/* ------------------------------------------------------------------------ */
/* Dirac algebra in the Dirac representation (Sec. 7: the nonrelativistic
 * projector keeps the upper two spinor components in this representation).  */

static void mm4(const cplx *a, const cplx *b, cplx *c)
{
    cplx t[16];
    for (int i = 0; i < 4; i++)
        for (int j = 0; j < 4; j++) {
            cplx s = 0;
            for (int k = 0; k < 4; k++) s += a[4 * i + k] * b[4 * k + j];
            t[4 * i + j] = s;
        }
    memcpy(c, t, sizeof t);
}

/* out[0..3] = gamma^0..gamma^3 (Minkowski, Dirac rep.), out[4] = gamma_5 =
 * i g0 g1 g2 g3, out[5] = C = i g2 g0 (charge conjugation).  Each 4x4,
 * row-major. */
void orc_dirac(cplx *out)
{
    const cplx iu = _Complex_I;
    cplx sig[3][4] = {{0, 1, 1, 0}, {0, -iu, iu, 0}, {1, 0, 0, -1}};
    cplx *g0 = out, *g5 = out + 64, *C = out + 80;
    memset(out, 0, 6 * 16 * sizeof(cplx));
    g0[0] = 1; g0[5] = 1; g0[10] = -1; g0[15] = -1;
    for (int k = 0; k < 3; k++) {
        cplx *g = out + 16 * (k + 1);
        /* gamma^k = [[0, sigma_k], [-sigma_k, 0]] */
        for (int i = 0; i < 2; i++)
            for (int j = 0; j < 2; j++) {
                g[4 * i + (j + 2)] = sig[k][2 * i + j];
                g[4 * (i + 2) + j] = -sig[k][2 * i + j];
            }
    }
    cplx t[16];
    mm4(out, out + 16, t);
    mm4(t, out + 32, t);
    mm4(t, out + 48, t);
    for (int i = 0; i < 16; i++) g5[i] = iu * t[i];
    mm4(out + 32, out, t);
    for (int i = 0; i < 16; i++) C[i] = iu * t[i];
}

/* Gamma_1, Gamma_2 of the nucleon operators (Sec. 7):
 *   relativistic:     Gamma_1 = 1,     Gamma_2 = C gamma_5
 *   nonrelativistic:  Gamma_1 = P_nr,  Gamma_2 = C gamma_5 P_nr,
 *                     P_nr = (1 + gamma_4)/2 with gamma_4 = gamma^0 here.   */
void orc_gamma(int rel, cplx *G1, cplx *G2)
{
    cplx d[6 * 16], Cg5[16], P[16];
    orc_dirac(d);
    mm4(d + 80, d + 64, Cg5);
    for (int i = 0; i < 16; i++) P[i] = ((i % 5 == 0) ? 1.0 : 0.0) + d[i];
    for (int i = 0; i < 16; i++) P[i] *= 0.5;
    if (rel) {
        for (int i = 0; i < 16; i++) G1[i] = (i % 5 == 0) ? 1.0 : 0.0;
        memcpy(G2, Cg5, sizeof Cg5);
    } else {
        memcpy(G1, P, sizeof P);
        mm4(Cg5, P, G2);
    }
}

/* Levi-Civita symbol in three colours. */
static int eps3(int a, int b, int c)
{
    if (a == b || b == c || a == c) return 0;
    if ((a == 0 && b == 1) || (a == 1 && b == 2) || (a == 2 && b == 0)) return 1;
    return -1;
}

/* ------------------------------------------------------------------------ */
/* The tensors G^B (eq. def_g) and, with several sources, G-tilde
 * (eq. G_tilde): the three source quarks of a baryon share its source.
 * G is the same function of (chi; slot1, slot2, slot3) for proton and
 * neutron; the flavour enters only through which slots carry which flavour.
 * Writes every nonzero entry over the full index range 0..12 N_s - 1.
 * Returns the number of entries.                                         */
int orc_g_nonzero(int rel, int nsrc, int chi, int *xi, cplx *val, int max)
{
    cplx G1[16], G2[16];
    orc_gamma(rel, G1, G2);
    int alpha = chi / nsrc, s = chi % nsrc, n = 0, nx = 12 * nsrc;
    for (int x1 = 0; x1 < nx; x1++)
        for (int x2 = 0; x2 < nx; x2++)
            for (int x3 = 0; x3 < nx; x3++) {
                if (x1 % nsrc != s || x2 % nsrc != s || x3 % nsrc != s) continue;
                int k1 = x1 / nsrc, k2 = x2 / nsrc, k3 = x3 / nsrc;
                cplx v = G1[4 * alpha + k1 / 3] * G2[4 * (k2 / 3) + k3 / 3] *
                         (double)eps3(k1 % 3, k2 % 3, k3 % 3);
                if (v == 0) continue;
                if (n < max) {
                    xi[3 * n] = x1; xi[3 * n + 1] = x2; xi[3 * n + 2] = x3;
                    val[n] = v;
                }
                n++;
            }
    return n;
}

/* ------------------------------------------------------------------------ */
/* Baryon blocks (Sec. 2, with one sink function per source index, Sec. 6):
 *   f(psi; xi1, xi2, xi3) = sum_x w_{s'}(x) eps_abc (Gamma_1)_{alpha beta}
 *        (Gamma_2)_{gamma delta} S_q1[(beta,a), xi1] S_q2[(gamma,b), xi2]
 *        S_q3[(delta,c), xi3],      psi = N_s*alpha + s'.
 * Proton (q1,q2,q3) = (u,u,d), neutron (d,u,d).  No Grassmann sign is
 * attached.  Every propagator entry is multiplied by `scale` on reading.
 * Output: full (not antisymmetrised) fP, fN[psi][xi1][xi2][xi3], psi <
 * npsi, xi < nxi.                                                         */
void orc_blocks(int rel, int nsrc, int npsi, int nxi, int V, const cplx *Su,
                const cplx *Sd, const cplx *sinkw, double scale, cplx *fP,
                cplx *fN)
{
    cplx G1[16], G2[16];
    orc_gamma(rel, G1, G2);
    long nout = (long)npsi * nxi * nxi * nxi;
    memset(fP, 0, nout * sizeof(cplx));
    memset(fN, 0, nout * sizeof(cplx));
#define SP(S, x, row, xi) \
    (scale * (S)[(((long)(x) * nsrc + (xi) % nsrc) * 12 + (row)) * 12 + (xi) / nsrc])
    /* every output entry is one independent sum, computed by one thread */
#pragma omp parallel for collapse(2) schedule(dynamic)
    for (int psi = 0; psi < npsi; psi++) {
        for (int x1 = 0; x1 < nxi; x1++) {
            int alpha = psi / nsrc, sk = psi % nsrc;
            for (int x2 = 0; x2 < nxi; x2++)
                for (int x3 = 0; x3 < nxi; x3++) {
                    cplx sp = 0, sn = 0;
                    for (int x = 0; x < V; x++) {
                        cplx w = sinkw ? sinkw[(long)sk * V + x] : 1.0;
                        for (int a = 0; a < 3; a++)
                            for (int b = 0; b < 3; b++)
                                for (int c = 0; c < 3; c++) {
                                    int e = eps3(a, b, c);
                                    if (!e) continue;
                                    for (int be = 0; be < 4; be++) {
                                        cplx g1 = G1[4 * alpha + be];
                                        if (g1 == 0) continue;
                                        for (int ga = 0; ga < 4; ga++)
                                            for (int de = 0; de < 4; de++) {
                                                cplx g2 = G2[4 * ga + de];
                                                if (g2 == 0) continue;
                                                cplx cf = w * (double)e * g1 * g2;
                                                sp += cf * SP(Su, x, 3 * be + a, x1) *
                                                      SP(Su, x, 3 * ga + b, x2) *
                                                      SP(Sd, x, 3 * de + c, x3);
                                                sn += cf * SP(Sd, x, 3 * be + a, x1) *
                                                      SP(Su, x, 3 * ga + b, x2) *
                                                      SP(Sd, x, 3 * de + c, x3);
                                            }
                                    }
                                }
                    }
                    long o = (((long)psi * nxi + x1) * nxi + x2) * nxi + x3;
                    fP[o] = sp;
                    fN[o] = sn;
                }
        }
    }
#undef SP
}

/* The Lambda block: the same baryon form (Sec. 1, eq. C_baryons) with
 * (q1, q2, q3) = (s, u, d), Gamma_1 and Gamma_2 as for the nucleons:
 *   fL(psi; xi1, xi2, xi3) = sum_x w_{s'}(x) eps_abc (Gamma_1)_{alpha beta}
 *        (Gamma_2)_{gamma delta} S_s[(beta,a), xi1] S_u[(gamma,b), xi2]
 *        S_d[(delta,c), xi3].
 * Same layout and conventions as orc_blocks.                              */
void orc_blocks_lambda(int rel, int nsrc, int npsi, int nxi, int V, const cplx *Su,
                       const cplx *Sd, const cplx *Ss, const cplx *sinkw, double scale,
                       cplx *fL)
{
    cplx G1[16], G2[16];
    orc_gamma(rel, G1, G2);
    long nout = (long)npsi * nxi * nxi * nxi;
    memset(fL, 0, nout * sizeof(cplx));
#define SP(S, x, row, xi) \
    (scale * (S)[(((long)(x) * nsrc + (xi) % nsrc) * 12 + (row)) * 12 + (xi) / nsrc])
#pragma omp parallel for collapse(2) schedule(dynamic)
    for (int psi = 0; psi < npsi; psi++) {
        for (int x1 = 0; x1 < nxi; x1++) {
            int alpha = psi / nsrc, sk = psi % nsrc;
            for (int x2 = 0; x2 < nxi; x2++)
                for (int x3 = 0; x3 < nxi; x3++) {
                    cplx acc = 0;
                    for (int x = 0; x < V; x++) {
                        cplx w = sinkw ? sinkw[(long)sk * V + x] : 1.0;
                        for (int a = 0; a < 3; a++)
                            for (int b = 0; b < 3; b++)
                                for (int c = 0; c < 3; c++) {
                                    int e = eps3(a, b, c);
                                    if (!e) continue;
                                    for (int be = 0; be < 4; be++) {
                                        cplx g1 = G1[4 * alpha + be];
                                        if (g1 == 0) continue;
                                        for (int ga = 0; ga < 4; ga++)
                                            for (int de = 0; de < 4; de++) {
                                                cplx g2 = G2[4 * ga + de];
                                                if (g2 == 0) continue;
                                                acc += w * (double)e * g1 * g2 * SP(Ss, x, 3 * be + a, x1) *
                                                       SP(Su, x, 3 * ga + b, x2) * SP(Sd, x, 3 * de + c, x3);
                                            }
                                    }
                                }
                    }
                    fL[(((long)psi * nxi + x1) * nxi + x2) * nxi + x3] = acc;
                }
        }
    }
#undef SP
}

/* Flavour of quark slot j of a baryon of type t (0 = u, 1 = d, 2 = s):
 * proton (u,u,d), neutron (d,u,d), Lambda (s,u,d).                        */
static int slot_flavour(int t, int j)
{
    if (j == 1) return 0;
    if (j == 2) return 1;
    return t == 0 ? 0 : t == 1 ? 1 : 2;
}

/* ------------------------------------------------------------------------ */
/* Small open-addressing hash map: 4 x uint32 key -> int64 value.          */

typedef struct {
    uint32_t *k; /* 4 per slot */
    long long *v;
    unsigned char *used;
    long cap, n;
} hmap;

static uint64_t hmix(const uint32_t *k)
{
    uint64_t h = 0x9e3779b97f4a7c15ull;
    for (int i = 0; i < 4; i++) {
        h ^= k[i];
        h *= 0xbf58476d1ce4e5b9ull;
        h ^= h >> 31;
    }
    return h;
}

static void hm_init(hmap *m, long cap)
{
    long c = 16;
    while (c < 2 * cap) c <<= 1;
    m->cap = c;
    m->n = 0;
    m->k = calloc((size_t)c * 4, sizeof(uint32_t));
    m->v = calloc((size_t)c, sizeof(long long));
    m->used = calloc((size_t)c, 1);
}

static void hm_free(hmap *m)
{
    free(m->k); free(m->v); free(m->used);
}

static long hm_slot(const hmap *m, const uint32_t *key)
{
    long i = (long)(hmix(key) & (uint64_t)(m->cap - 1));
    while (m->used[i] && memcmp(m->k + 4 * i, key, 16) != 0) i = (i + 1) & (m->cap - 1);
    return i;
}

static void hm_grow(hmap *m)
{
    hmap t;
    hm_init(&t, m->cap);
    for (long i = 0; i < m->cap; i++)
        if (m->used[i]) {
            long j = hm_slot(&t, m->k + 4 * i);
            t.used[j] = 1;
            memcpy(t.k + 4 * j, m->k + 4 * i, 16);
            t.v[j] = m->v[i];
            t.n++;
        }
    hm_free(m);
    *m = t;
}

/* Adds `v` to the value stored at key (inserting with 0 first). */
static void hm_add(hmap *m, const uint32_t *key, long long v)
{
    if (2 * (m->n + 1) > m->cap) hm_grow(m);
    long i = hm_slot(m, key);
    if (!m->used[i]) {
        m->used[i] = 1;
        memcpy(m->k + 4 * i, key, 16);
        m->v[i] = 0;
        m->n++;
    }
    m->v[i] += v;
}

static int key_cmp(const void *a, const void *b)
{
    const uint32_t *x = a, *y = b;
    for (int i = 0; i < 4; i++)
        if (x[i] != y[i]) return x[i] < y[i] ? -1 : 1;
    return 0;
}

static int key3_cmp(const void *a, const void *b)
{
    const uint32_t *x = a, *y = b;
    for (int i = 0; i < 3; i++)
        if (x[i] != y[i]) return x[i] < y[i] ? -1 : 1;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* The tensor L of the unified contraction algorithm (eq. tensor_L), built
 * the way Sec. 2 describes it: by running over every combination of nonzero
 * entries of G^{B_1} ... G^{B_N} and every flavour-preserving permutation.
 * Grouping the terms by the set of u and d indices they use gives L on
 * sorted index sets:
 *   L(alpha; z) = sum over assignments eta of the indices of z to the quark
 *                 slots of  sgn(eta) * prod_k G^{B_k}(alpha_k; eta slots of k),
 * where sgn(eta) is the product of the parities of the u, d and s
 * sequences (slots in baryon order, within a baryon in operator order:
 * proton (u,u,d), neutron (d,u,d), Lambda (s,u,d)); assignments that repeat
 * an index of one flavour cancel and are skipped.
 * types[k] = 0 proton / 1 neutron / 2 Lambda, chis[k] the source index of
 * baryon k.  Output: keys (u mask, d mask, s mask) ascending and their
 * integer values (smask may be NULL without Lambdas); returns the number of
 * nonzero entries (at most max are written).                              */

typedef struct {
    int nb, types[16];
    int nent[16];
    int *xi[16];
    cplx *val[16];
    int seq[3][64];   /* index sequence of each flavour, slots in order */
    hmap *acc;
} uca_state;

static int parity(const int *s, int n)
{
    int inv = 0;
    for (int i = 0; i < n; i++)
        for (int j = i + 1; j < n; j++)
            if (s[i] > s[j]) inv++;
    return (inv & 1) ? -1 : 1;
}

/* n[f], m[f]: length and index set of flavour f's sequence so far */
static void uca_rec(uca_state *st, int k, const int *n, const uint32_t *m, cplx prod)
{
    if (k == st->nb) {
        double re = creal(prod), im = cimag(prod);
        long long iv = (long long)(re < 0 ? re - 0.5 : re + 0.5);
        (void)im;
        uint32_t key[4] = {m[0], m[1], m[2], 0};
        hm_add(st->acc, key, iv * parity(st->seq[0], n[0]) * parity(st->seq[1], n[1]) *
                                 parity(st->seq[2], n[2]));
        return;
    }
    for (int e = 0; e < st->nent[k]; e++) {
        const int *x = st->xi[k] + 3 * e;
        int n2[3] = {n[0], n[1], n[2]};
        uint32_t m2[3] = {m[0], m[1], m[2]};
        int ok = 1;
        for (int j = 0; j < 3 && ok; j++) {
            int f = slot_flavour(st->types[k], j);
            uint32_t bit = 1u << x[j];
            if (m2[f] & bit) ok = 0;
            m2[f] |= bit;
            st->seq[f][n2[f]++] = x[j];
        }
        if (!ok) continue; /* a repeated index of one flavour: the term cancels */
        uca_rec(st, k + 1, n2, m2, prod * st->val[k][e]);
    }
}

long orc_L_uca(int rel, int nsrc, int nb, const int *types, const int *chis,
               uint32_t *umask, uint32_t *dmask, uint32_t *smask, long long *coef, long max)
{
    uca_state st;
    memset(&st, 0, sizeof st);
    st.nb = nb;
    int cap = 12 * nsrc * 12 * nsrc * 12 * nsrc;
    for (int k = 0; k < nb; k++) {
        st.types[k] = types[k];
        st.xi[k] = malloc(sizeof(int) * 3 * cap);
        st.val[k] = malloc(sizeof(cplx) * cap);
        st.nent[k] = orc_g_nonzero(rel, nsrc, chis[k], st.xi[k], st.val[k], cap);
    }
    hmap acc;
    hm_init(&acc, 1 << 12);
    st.acc = &acc;
    const int n0[3] = {0, 0, 0};
    const uint32_t m0[3] = {0, 0, 0};
    uca_rec(&st, 0, n0, m0, 1.0);
    /* collect nonzero values, sorted by (u mask, d mask, s mask) */
    long n = 0;
    uint32_t *tmp = malloc(sizeof(uint32_t) * 5 * (acc.n + 1));
    for (long i = 0; i < acc.cap; i++)
        if (acc.used[i] && acc.v[i] != 0) {
            memcpy(tmp + 5 * n, acc.k + 4 * i, 12);
            long long v = acc.v[i];
            tmp[5 * n + 3] = (uint32_t)(v & 0xffffffffu);
            tmp[5 * n + 4] = (uint32_t)((unsigned long long)v >> 32);
            n++;
        }
    qsort(tmp, n, 20, key3_cmp);
    for (long i = 0; i < n && i < max; i++) {
        umask[i] = tmp[5 * i];
        dmask[i] = tmp[5 * i + 1];
        if (smask) smask[i] = tmp[5 * i + 2];
        coef[i] = (long long)(((unsigned long long)tmp[5 * i + 4] << 32) | tmp[5 * i + 3]);
    }
    free(tmp);
    hm_free(&acc);
    for (int k = 0; k < nb; k++) {
        free(st.xi[k]);
        free(st.val[k]);
    }
    return n;
}

/* ------------------------------------------------------------------------ */
/* The correlator by eq. f_L_contr:  C = sum_xi F(delta; xi) L(alpha; xi).
 * Only index tuples with distinct indices per flavour contribute, and for
 * each sorted set z the sum over the orderings of z is
 *   C = sum_z L(alpha; z) * W(delta; z),
 *   W(delta; z) = sum_{pi_u, pi_d, pi_s} sgn(pi_u) sgn(pi_d) sgn(pi_s)
 *                 prod_k f_{B_k}(delta_k; the slots of k filled from z
 *                                permuted by pi_u, pi_d, pi_s),
 * with the same slot order as in orc_L_uca.  Blocks are the full
 * (unsymmetrised) f of orc_blocks and orc_blocks_lambda (fL and smask may
 * be NULL without Lambdas).                                              */

static int nperms(int n, int *perm, int *sgn, long max)
{
    /* all permutations of 0..n-1 in lexicographic order with their signs */
    int a[16];
    for (int i = 0; i < n; i++) a[i] = i;
    long cnt = 0;
    for (;;) {
        if (cnt < max) {
            memcpy(perm + cnt * n, a, sizeof(int) * n);
            sgn[cnt] = parity(a, n);
        }
        cnt++;
        int i = n - 2;
        while (i >= 0 && a[i] > a[i + 1]) i--;
        if (i < 0) break;
        int j = n - 1;
        while (a[j] < a[i]) j--;
        int t = a[i]; a[i] = a[j]; a[j] = t;
        for (int l = i + 1, r = n - 1; l < r; l++, r--) {
            t = a[l]; a[l] = a[r]; a[r] = t;
        }
    }
    return (int)cnt;
}

static long factl(int n)
{
    long f = 1;
    for (int i = 2; i <= n; i++) f *= i;
    return f;
}

void orc_corr(int nb, const int *types, const int *psis, int npsi, int nxi,
              const cplx *fP, const cplx *fN, const cplx *fL, long nz, const uint32_t *umask,
              const uint32_t *dmask, const uint32_t *smask, const long long *coef, cplx *out)
{
    /* slot bookkeeping: for every flavour, the (baryon, slot) of each
     * position of its slot sequence */
    int sb[3][64], sj[3][64], nf[3] = {0, 0, 0};
    for (int k = 0; k < nb; k++)
        for (int j = 0; j < 3; j++) {
            int f = slot_flavour(types[k], j);
            sb[f][nf[f]] = k;
            sj[f][nf[f]] = j;
            nf[f]++;
        }
    long fct[3];
    int *pm[3], *ps[3];
    for (int f = 0; f < 3; f++) {
        fct[f] = factl(nf[f]);
        pm[f] = malloc(sizeof(int) * (nf[f] ? nf[f] : 1) * fct[f]);
        ps[f] = malloc(sizeof(int) * fct[f]);
        nperms(nf[f], pm[f], ps[f], fct[f]);
    }
    /* W(delta; z) for every z (independent, one thread each), then the sum
     * over z in order */
    cplx *Wz = malloc(sizeof(cplx) * (nz > 0 ? nz : 1));
#pragma omp parallel for schedule(dynamic)
    for (long iz = 0; iz < nz; iz++) {
        int lst[3][32], cnt[3] = {0, 0, 0};
        const uint32_t m[3] = {umask[iz], dmask[iz], smask ? smask[iz] : 0u};
        for (int f = 0; f < 3; f++)
            for (int i = 0; i < 32; i++)
                if (m[f] >> i & 1) lst[f][cnt[f]++] = i;
        cplx W = 0;
        int slot[16][3];
        for (long p = 0; p < fct[0]; p++) {
            for (int j = 0; j < nf[0]; j++) slot[sb[0][j]][sj[0][j]] = lst[0][pm[0][p * nf[0] + j]];
            for (long q = 0; q < fct[1]; q++) {
                for (int j = 0; j < nf[1]; j++) slot[sb[1][j]][sj[1][j]] = lst[1][pm[1][q * nf[1] + j]];
                for (long r = 0; r < fct[2]; r++) {
                    for (int j = 0; j < nf[2]; j++) slot[sb[2][j]][sj[2][j]] = lst[2][pm[2][r * nf[2] + j]];
                    cplx prod = ps[0][p] * ps[1][q] * ps[2][r];
                    for (int k = 0; k < nb; k++) {
                        const cplx *f = types[k] == 0 ? fP : types[k] == 1 ? fN : fL;
                        long o = (((long)psis[k] * nxi + slot[k][0]) * nxi + slot[k][1]) * nxi + slot[k][2];
                        prod *= f[o];
                    }
                    W += prod;
                }
            }
        }
        Wz[iz] = W;
    }
    cplx total = 0;
    for (long iz = 0; iz < nz; iz++) total += (double)coef[iz] * Wz[iz];
    free(Wz);
    (void)npsi;
    *out = total;
    for (int f = 0; f < 3; f++) {
        free(pm[f]);
        free(ps[f]);
    }
}

/* ------------------------------------------------------------------------ */
/* Single-nucleon two-point function written as the Wick contraction of
 * <P_delta(x) Pbar^alpha> with the two u quarks contracted directly or
 * crossed (Sec. 1, 7), summed over sink sites with weight w_0:
 *   C = sum_x w(x) eps_abc eps_a'b'c' G1_{delta beta} G2_{gamma eps}
 *       G1_{alpha beta'} G2_{gamma' eps'} S_d[(eps,c),(eps',c')]
 *       ( S_u[(beta,a),(beta',a')] S_u[(gamma,b),(gamma',b')]
 *       - S_u[(beta,a),(gamma',b')] S_u[(gamma,b),(beta',a')] ).
 * One source only.                                                        */
void orc_proton_closed(int rel, int V, const cplx *Su, const cplx *Sd,
                       const cplx *sinkw, double scale, int delta, int alpha,
                       cplx *out)
{
    cplx G1[16], G2[16];
    orc_gamma(rel, G1, G2);
    cplx tot = 0;
    for (int x = 0; x < V; x++) {
        const cplx *u = Su + (long)x * 144, *d = Sd + (long)x * 144;
        cplx w = sinkw ? sinkw[x] : 1.0;
        for (int a = 0; a < 3; a++) for (int b = 0; b < 3; b++) for (int c = 0; c < 3; c++) {
            int e1 = eps3(a, b, c);
            if (!e1) continue;
            for (int a2 = 0; a2 < 3; a2++) for (int b2 = 0; b2 < 3; b2++) for (int c2 = 0; c2 < 3; c2++) {
                int e2 = eps3(a2, b2, c2);
                if (!e2) continue;
                for (int be = 0; be < 4; be++) for (int ga = 0; ga < 4; ga++) for (int ep = 0; ep < 4; ep++) {
                    cplx s1 = G1[4 * delta + be] * G2[4 * ga + ep];
                    if (s1 == 0) continue;
                    for (int be2 = 0; be2 < 4; be2++) for (int ga2 = 0; ga2 < 4; ga2++) for (int ep2 = 0; ep2 < 4; ep2++) {
                        cplx s2 = G1[4 * alpha + be2] * G2[4 * ga2 + ep2];
                        if (s2 == 0) continue;
                        int r1 = 3 * be + a, r2 = 3 * ga + b, r3 = 3 * ep + c;
                        int c1 = 3 * be2 + a2, c2i = 3 * ga2 + b2, c3 = 3 * ep2 + c2;
                        cplx dir = u[12 * r1 + c1] * u[12 * r2 + c2i];
                        cplx crs = u[12 * r1 + c2i] * u[12 * r2 + c1];
                        tot += w * (double)(e1 * e2) * s1 * s2 * scale * scale * scale *
                               d[12 * r3 + c3] * (dir - crs);
                    }
                }
            }
        }
    }
    *out = tot;
}

/* ------------------------------------------------------------------------ */
/* Literal Wick contraction of < prod_k B_{psi_k} prod_k Bbar^{chi_k} >,
 * with every baryon projected by its own sum over sink sites: for every
 * choice of sink sites, every nonzero colour-spin coefficient of each sink
 * operator and of each source operator, and every flavour-preserving
 * pairing of sink quarks with source quarks, the signed product of
 * propagators.  Written without blocks or L; feasible only for a few
 * baryons on a handful of sites.                                          */
void orc_wick_literal(int rel, int nsrc, int nb, const int *types,
                      const int *psis, const int *chis, int V, const cplx *Su,
                      const cplx *Sd, const cplx *Ss, const cplx *sinkw, double scale, cplx *out)
{
    cplx G1[16], G2[16];
    orc_gamma(rel, G1, G2);
    /* sink coefficient lists: (row1,row2,row3, coef) */
    int nsk[16], *skr[16];
    cplx *skc[16];
    int nso[16], *sox[16];
    cplx *soc[16];
    int cap = 12 * nsrc * 12 * nsrc * 12 * nsrc;
    for (int k = 0; k < nb; k++) {
        skr[k] = malloc(sizeof(int) * 3 * 1728);
        skc[k] = malloc(sizeof(cplx) * 1728);
        int alpha = psis[k] / nsrc, n = 0;
        for (int a = 0; a < 3; a++) for (int b = 0; b < 3; b++) for (int c = 0; c < 3; c++)
            for (int be = 0; be < 4; be++) for (int ga = 0; ga < 4; ga++) for (int de = 0; de < 4; de++) {
                cplx v = (double)eps3(a, b, c) * G1[4 * alpha + be] * G2[4 * ga + de];
                if (v == 0) continue;
                skr[k][3 * n] = 3 * be + a; skr[k][3 * n + 1] = 3 * ga + b; skr[k][3 * n + 2] = 3 * de + c;
                skc[k][n++] = v;
            }
        nsk[k] = n;
        sox[k] = malloc(sizeof(int) * 3 * cap);
        soc[k] = malloc(sizeof(cplx) * cap);
        nso[k] = orc_g_nonzero(rel, nsrc, chis[k], sox[k], soc[k], cap);
    }
    /* flavour slot lists (slot id = 3*k + j) and their permutations */
    int fslot[3][64], nf[3] = {0, 0, 0};
    for (int k = 0; k < nb; k++)
        for (int j = 0; j < 3; j++) {
            int f = slot_flavour(types[k], j);
            fslot[f][nf[f]++] = 3 * k + j;
        }
    const cplx *Sf[3] = {Su, Sd, Ss};
    long fct[3];
    int *pm[3], *ps[3];
    for (int f = 0; f < 3; f++) {
        fct[f] = factl(nf[f]);
        pm[f] = malloc(sizeof(int) * (nf[f] ? nf[f] : 1) * fct[f]);
        ps[f] = malloc(sizeof(int) * fct[f]);
        nperms(nf[f], pm[f], ps[f], fct[f]);
    }

    cplx tot = 0;
    long npos = 1;
    for (int k = 0; k < nb; k++) npos *= V;
    int xs[16], isk[16], iso[16];
    for (long pos = 0; pos < npos; pos++) {
        long r = pos;
        cplx wprod = 1;
        for (int k = 0; k < nb; k++) {
            xs[k] = (int)(r % V);
            r /= V;
            wprod *= sinkw ? sinkw[(long)(psis[k] % nsrc) * V + xs[k]] : 1.0;
        }
        if (wprod == 0) continue;
        /* odometer over sink coefficient choices */
        memset(isk, 0, sizeof isk);
        for (;;) {
            cplx csk = wprod;
            int row[48];
            for (int k = 0; k < nb; k++) {
                csk *= skc[k][isk[k]];
                for (int j = 0; j < 3; j++) row[3 * k + j] = skr[k][3 * isk[k] + j];
            }
            memset(iso, 0, sizeof iso);
            for (;;) {
                cplx cso = csk;
                int col[48];
                for (int k = 0; k < nb; k++) {
                    cso *= soc[k][iso[k]];
                    for (int j = 0; j < 3; j++) col[3 * k + j] = sox[k][3 * iso[k] + j];
                }
                /* every flavour-preserving pairing: sink slot fslot[f][j]
                 * takes the source slot fslot[f][perm(j)] */
                cplx acc = 0;
                for (long p = 0; p < fct[0]; p++)
                    for (long q = 0; q < fct[1]; q++)
                        for (long r = 0; r < fct[2]; r++) {
                            const long pick[3] = {p, q, r};
                            cplx pr = ps[0][p] * ps[1][q] * ps[2][r];
                            for (int f = 0; f < 3 && pr != 0; f++)
                                for (int j = 0; j < nf[f]; j++) {
                                    int sl = fslot[f][j], tl = fslot[f][pm[f][pick[f] * nf[f] + j]];
                                    int xi = col[tl];
                                    pr *= scale * Sf[f][(((long)xs[sl / 3] * nsrc + xi % nsrc) * 12 + row[sl]) * 12 +
                                                        xi / nsrc];
                                }
                            acc += pr;
                        }
                tot += cso * acc;
                int k = 0;
                while (k < nb && ++iso[k] == nso[k]) iso[k++] = 0;
                if (k == nb) break;
            }
            int k = 0;
            while (k < nb && ++isk[k] == nsk[k]) isk[k++] = 0;
            if (k == nb) break;
        }
    }
    *out = tot;
    for (int k = 0; k < nb; k++) {
        free(skr[k]); free(skc[k]); free(sox[k]); free(soc[k]);
    }
    for (int f = 0; f < 3; f++) {
        free(pm[f]);
        free(ps[f]);
    }
}

/* ------------------------------------------------------------------------ */
/* Single-Lambda two-point function by direct Wick contraction: the s, u and
 * d quarks of the Lambda (slots (s,u,d)) each contract with their own
 * source quark, so there is only the direct term:
 *   C = sum_x w(x) eps_abc eps_a'b'c' G1_{delta beta} G2_{gamma eps}
 *       G1_{alpha beta'} G2_{gamma' eps'} S_s[(beta,a),(beta',a')]
 *       S_u[(gamma,b),(gamma',b')] S_d[(eps,c),(eps',c')].
 * One source only.                                                        */
void orc_lambda_closed(int rel, int V, const cplx *Su, const cplx *Sd, const cplx *Ss,
                       const cplx *sinkw, double scale, int delta, int alpha, cplx *out)
{
    cplx G1[16], G2[16];
    orc_gamma(rel, G1, G2);
    cplx tot = 0;
    for (int x = 0; x < V; x++) {
        const cplx *u = Su + (long)x * 144, *d = Sd + (long)x * 144, *st = Ss + (long)x * 144;
        cplx w = sinkw ? sinkw[x] : 1.0;
        for (int a = 0; a < 3; a++) for (int b = 0; b < 3; b++) for (int c = 0; c < 3; c++) {
            int e1 = eps3(a, b, c);
            if (!e1) continue;
            for (int a2 = 0; a2 < 3; a2++) for (int b2 = 0; b2 < 3; b2++) for (int c2 = 0; c2 < 3; c2++) {
                int e2 = eps3(a2, b2, c2);
                if (!e2) continue;
                for (int be = 0; be < 4; be++) for (int ga = 0; ga < 4; ga++) for (int ep = 0; ep < 4; ep++) {
                    cplx s1 = G1[4 * delta + be] * G2[4 * ga + ep];
                    if (s1 == 0) continue;
                    for (int be2 = 0; be2 < 4; be2++) for (int ga2 = 0; ga2 < 4; ga2++) for (int ep2 = 0; ep2 < 4; ep2++) {
                        cplx s2 = G1[4 * alpha + be2] * G2[4 * ga2 + ep2];
                        if (s2 == 0) continue;
                        tot += w * (double)(e1 * e2) * s1 * s2 * scale * scale * scale *
                               st[12 * (3 * be + a) + 3 * be2 + a2] * u[12 * (3 * ga + b) + 3 * ga2 + b2] *
                               d[12 * (3 * ep + c) + 3 * ep2 + c2];
                    }
                }
            }
        }
    }
    *out = tot;
}

/* ------------------------------------------------------------------------ */
/* Required components and operation lists (Sec. 3, 4).  A component is a
 * tuple of four index sets (proton spins, neutron spins, u indices, d
 * indices), stored as four bit masks.                                     */

/* All stage components of the given shape (kP, kN, ku, kd) that are
 * sub-tuples of at least one final component: the components a recursion
 * step must compute so that every final component of interest can be
 * formed.  Output sorted, unique; returns the count.                      */
long orc_req_stage(long nfin, const uint32_t *fin, int kP, int kN, int ku,
                   int kd, uint32_t *out, long max)
{
    hmap set;
    hm_init(&set, 1 << 16);
    const int want[4] = {kP, kN, ku, kd};
    for (long i = 0; i < nfin; i++) {
        const uint32_t *z = fin + 4 * i;
        /* enumerate sub-masks of each group with the wanted popcount */
        uint32_t subs[4][4096];
        int ns[4];
        for (int g = 0; g < 4; g++) {
            ns[g] = 0;
            uint32_t m = z[g], s = m;
            for (;;) {
                if (__builtin_popcount(s) == want[g]) subs[g][ns[g]++] = s;
                if (s == 0) break;
                s = (s - 1) & m;
            }
        }
        for (int a = 0; a < ns[0]; a++) for (int b = 0; b < ns[1]; b++)
            for (int c = 0; c < ns[2]; c++) for (int d = 0; d < ns[3]; d++) {
                uint32_t key[4] = {subs[0][a], subs[1][b], subs[2][c], subs[3][d]};
                hm_add(&set, key, 0);
            }
    }
    long n = 0;
    uint32_t *tmp = malloc(sizeof(uint32_t) * 4 * (set.n + 1));
    for (long i = 0; i < set.cap; i++)
        if (set.used[i]) memcpy(tmp + 4 * n++, set.k + 4 * i, 16);
    qsort(tmp, n, 16, key_cmp);
    if (max > 0) memcpy(out, tmp, sizeof(uint32_t) * 4 * (n < max ? n : max));
    free(tmp);
    hm_free(&set);
    return n;
}

/* sgn(x|y) for one group: product over j in y, i in x with i > j of -1
 * (Sec. 3). */
static int sgn_group(uint32_t x, uint32_t y)
{
    int s = 0;
    for (int j = 0; j < 32; j++)
        if (y >> j & 1) s += __builtin_popcount(j == 31 ? 0u : x >> (j + 1));
    return (s & 1) ? -1 : 1;
}

static long find_key(long n, const uint32_t *keys, const uint32_t *k)
{
    long lo = 0, hi = n - 1;
    while (lo <= hi) {
        long mid = (lo + hi) / 2;
        int c = key_cmp(keys + 4 * mid, k);
        if (c == 0) return mid;
        if (c < 0) lo = mid + 1; else hi = mid - 1;
    }
    return -1;
}

/* The operation list of one recursion step F^(i+1) = F^(i) . f_B
 * (eq. recr_F with the product of eq. antis_product_2): for every required
 * output z, every split z = x + y where y has the shape of the added baryon
 * (proton: one proton spin, two u, one d; neutron: one neutron spin, one u,
 * two d), with sign prod_groups sgn(x|y).  Every x must be in the sorted
 * list xs.  Writes rows (z index, x index, y spin, y u mask, y d mask,
 * sign) when out != NULL; returns the number of operations, or -1 if some
 * x is missing from xs.                                                   */
long orc_lambda_stage(long nz, const uint32_t *zs, int added, long nx,
                      const uint32_t *xs, int64_t *out, long max)
{
    long cnt = 0;
    for (long iz = 0; iz < nz; iz++) {
        const uint32_t *z = zs + 4 * iz;
        int sg = added == 0 ? 0 : 1;      /* spin group of the added baryon */
        int nyu = added == 0 ? 2 : 1, nyd = added == 0 ? 1 : 2;
        for (uint32_t ys = z[sg]; ys; ys &= ys - 1) {
            uint32_t ysp = ys & (~ys + 1);
            uint32_t su = z[2];
            for (;;) {
                if (__builtin_popcount(su) == nyu) {
                    uint32_t sdm = z[3];
                    for (;;) {
                        if (__builtin_popcount(sdm) == nyd) {
                            uint32_t y[4] = {0, 0, su, sdm};
                            y[sg] = ysp;
                            uint32_t x[4];
                            for (int g = 0; g < 4; g++) x[g] = z[g] & ~y[g];
                            int sign = 1;
                            for (int g = 0; g < 4; g++) sign *= sgn_group(x[g], y[g]);
                            long ix = find_key(nx, xs, x);
                            if (ix < 0) return -1;
                            if (out && cnt < max) {
                                int64_t *r = out + 6 * cnt;
                                r[0] = iz; r[1] = ix; r[2] = ysp; r[3] = su; r[4] = sdm; r[5] = sign;
                            }
                            cnt++;
                        }
                        if (sdm == 0) break;
                        sdm = (sdm - 1) & z[3];
                    }
                }
                if (su == 0) break;
                su = (su - 1) & z[2];
            }
        }
    }
    return cnt;
}

/* ------------------------------------------------------------------------ */
/* Upper bounds of Sec. 7 (special cases of eqs. gen_P, gen_Q):
 *   P(nP,nN) = C(nP, Db-nP) C(nN, Db-nN) C(2nP+nN, Dq-2nP-nN)
 *              C(nP+2nN, Dq-nP-2nN)
 *   Q_P, Q_N as in the paper, with C(...) multinomial coefficients,
 * Db = D*N_s baryon spin values and Dq = 3*D*N_s quark index values
 * (Sec. 6 replaces 4 and 12 by 4 N_s and 12 N_s).                         */
static unsigned long long multinom(int n1, int n2, int n3)
{
    if (n1 < 0 || n2 < 0 || n3 < 0) return 0;
    /* (n1+n2+n3)! / (n1! n2! n3!) as binom(n1+n2+n3, n1) * binom(n2+n3, n2) */
    unsigned long long r = 1;
    int n = n1 + n2 + n3;
    for (int i = 1; i <= n1; i++) r = r * (unsigned long long)(n - n1 + i) / i;
    int m = n2 + n3;
    unsigned long long s = 1;
    for (int i = 1; i <= n2; i++) s = s * (unsigned long long)(m - n2 + i) / i;
    return r * s;
}

unsigned long long orc_bound_P(int D, int nsrc, int nP, int nN)
{
    int Db = D * nsrc, Dq = 3 * D * nsrc;
    return multinom(nP, Db - nP, 0) * multinom(nN, Db - nN, 0) *
           multinom(2 * nP + nN, Dq - 2 * nP - nN, 0) *
           multinom(nP + 2 * nN, Dq - nP - 2 * nN, 0);
}

unsigned long long orc_bound_Q(int D, int nsrc, int added, int nP, int nN)
{
    int Db = D * nsrc, Dq = 3 * D * nsrc;
    if (added == 0)
        return multinom(nP, 1, Db - 1 - nP) * multinom(nN, Db - nN, 0) *
               multinom(2 * nP + nN, 2, Dq - 2 - 2 * nP - nN) *
               multinom(nP + 2 * nN, 1, Dq - 1 - nP - 2 * nN);
    return multinom(nP, Db - nP, 0) * multinom(nN, 1, Db - 1 - nN) *
           multinom(2 * nP + nN, 1, Dq - 1 - 2 * nP - nN) *
           multinom(nP + 2 * nN, 2, Dq - 2 - nP - 2 * nN);
}
