/*
 * Oracle, plain C, FP64: divide-and-conquer sector index and matrix-free H*x
 * for sectors too large for the Python oracle.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the bench's
 * CPU-baseline leg load this library.  It shares no code, header or table with
 * the GPU library; it is written from the paper (arXiv:2407.14591) alone.
 *
 *  - sector dimension D_Q(l, m): coefficients of (1 + x + ... + x^{Q-1})^l
 *    by repeated multiplication (App. A);
 *  - local order inside a subsystem: all words in increasing numeric order
 *    (= lexicographic, first site most significant), numbered separately for
 *    each digit sum (Sec. 3.2, table lookup);
 *  - offsets and strides: eq. offset and eq. stride, with Gamma_k the number of
 *    sites to the right of P_k;
 *  - rank: eq. index / eq. ck (Alg. i); unrank: Alg. iii;
 *  - canonical order by nested generation: an odometer over the subsystems,
 *    each level running over its feasible local particle numbers in
 *    increasing order and over the words of that digit sum in numeric order;
 *    no offsets or strides are used;
 *  - H*x row by row: apply the XXZ terms to the row's basis state and gather x
 *    at the rank of each reached state (H is real symmetric).
 *
 * State encoding: ceil(log2 Q) bits per site, site 0 most significant.
 * Invalid input states rank to UINT64_MAX.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_MAXSUB 64
#define ORC_BAD UINT64_MAX

typedef struct {
    int Q, L, n, N, nb, maxm;
    int split[ORC_MAXSUB], start[ORC_MAXSUB], gamma[ORC_MAXSUB], shift[ORC_MAXSUB];
    uint64_t *Dt;                       /* (L+1) x (maxm+1) */
    int32_t *lsum[ORC_MAXSUB];          /* digit sum of a word, -1 if a digit >= Q */
    uint64_t *lidx[ORC_MAXSUB];         /* index of a word among words of its digit sum */
    uint64_t *linv[ORC_MAXSUB];         /* words listed by (digit sum, index) */
    uint64_t *lstart[ORC_MAXSUB];       /* first position of each digit sum in linv */
    uint64_t *off[ORC_MAXSUB];          /* [lam][m] offset_k(m, lam) */
    uint64_t *str[ORC_MAXSUB];          /* [lam][m] stride_k(m, lam) */
    uint64_t dim;
} orc_sector;

static uint64_t Dget(const orc_sector *s, int l, int m) {
    if (l < 0 || m < 0 || m > (s->Q - 1) * l) return 0;
    return s->Dt[(size_t)l * (s->maxm + 1) + m];
}

void orc_sector_free(orc_sector *s) {
    if (!s) return;
    free(s->Dt);
    for (int k = 0; k < s->N; ++k) {
        free(s->lsum[k]); free(s->lidx[k]); free(s->linv[k]); free(s->lstart[k]);
        free(s->off[k]); free(s->str[k]);
    }
    free(s);
}

uint64_t orc_dim(const orc_sector *s) { return s->dim; }

orc_sector *orc_sector_create(int Q, int L, int n, int N, const int *split) {
    if (Q < 2 || L < 1 || N < 1 || N > ORC_MAXSUB || n < 0 || n > (Q - 1) * L) return NULL;
    int nb = 0;
    while ((1 << nb) < Q) ++nb;
    if (nb * L > 64) return NULL;
    int tot = 0;
    for (int k = 0; k < N; ++k) {
        if (split[k] < 1 || nb * split[k] > 24) return NULL;
        tot += split[k];
    }
    if (tot != L) return NULL;
    orc_sector *s = (orc_sector *)calloc(1, sizeof(orc_sector));
    s->Q = Q; s->L = L; s->n = n; s->N = N; s->nb = nb; s->maxm = (Q - 1) * L;
    int acc = 0;
    for (int k = 0; k < N; ++k) {
        s->split[k] = split[k];
        s->start[k] = acc;
        acc += split[k];
        s->gamma[k] = L - acc;
        s->shift[k] = nb * (L - acc);
    }
    /* D table by repeated multiplication with (1 + x + ... + x^{Q-1}) */
    s->Dt = (uint64_t *)calloc((size_t)(L + 1) * (s->maxm + 1), sizeof(uint64_t));
    s->Dt[0] = 1;
    for (int l = 1; l <= L; ++l)
        for (int m = 0; m <= (Q - 1) * l; ++m) {
            uint64_t v = 0;
            for (int d = 0; d < Q && d <= m; ++d) v += Dget(s, l - 1, m - d);
            s->Dt[(size_t)l * (s->maxm + 1) + m] = v;
        }
    s->dim = Dget(s, L, n);
    for (int k = 0; k < N; ++k) {
        int Lk = split[k];
        uint64_t W = 1ull << (nb * Lk);
        int mk = (Q - 1) * Lk;
        s->lsum[k] = (int32_t *)malloc(W * sizeof(int32_t));
        s->lidx[k] = (uint64_t *)malloc(W * sizeof(uint64_t));
        s->linv[k] = (uint64_t *)malloc(W * sizeof(uint64_t));
        s->lstart[k] = (uint64_t *)calloc(mk + 2, sizeof(uint64_t));
        uint64_t *cnt = (uint64_t *)calloc(mk + 1, sizeof(uint64_t));
        for (uint64_t w = 0; w < W; ++w) {
            int sum = 0, ok = 1;
            for (int i = 0; i < Lk; ++i) {
                int d = (int)((w >> (nb * i)) & ((1u << nb) - 1));
                if (d >= Q) ok = 0;
                sum += d;
            }
            s->lsum[k][w] = ok ? sum : -1;
            if (ok) s->lidx[k][w] = cnt[sum]++;
        }
        for (int m = 0; m <= mk; ++m) s->lstart[k][m + 1] = s->lstart[k][m] + cnt[m];
        memset(cnt, 0, (mk + 1) * sizeof(uint64_t));
        for (uint64_t w = 0; w < W; ++w)
            if (s->lsum[k][w] >= 0) {
                int m = s->lsum[k][w];
                s->linv[k][s->lstart[k][m] + cnt[m]++] = w;
            }
        free(cnt);
        /* offsets and strides for every (lam, m) */
        s->off[k] = (uint64_t *)calloc((size_t)(n + 1) * (mk + 1), sizeof(uint64_t));
        s->str[k] = (uint64_t *)calloc((size_t)(n + 1) * (mk + 1), sizeof(uint64_t));
        int g = s->gamma[k];
        for (int lam = 0; lam <= n; ++lam) {
            int nlow = n - lam - (Q - 1) * g;
            if (nlow < 0) nlow = 0;
            for (int m = 0; m <= mk; ++m) {
                uint64_t o = 0;
                for (int j = nlow; j < m; ++j) o += Dget(s, Lk, j) * Dget(s, g, n - lam - j);
                s->off[k][(size_t)lam * (mk + 1) + m] = o;
                s->str[k][(size_t)lam * (mk + 1) + m] = Dget(s, g, n - lam - m);
            }
        }
    }
    return s;
}

static inline uint64_t subword(const orc_sector *s, uint64_t st, int k) {
    return (st >> s->shift[k]) & ((1ull << (s->nb * s->split[k])) - 1ull);
}

/* Alg. i: index = sum_k offset_k(n_k, lam_k) + stride_k(n_k, lam_k) * index_k */
uint64_t orc_rank(const orc_sector *s, uint64_t st) {
    if (s->nb * s->L < 64 && (st >> (s->nb * s->L))) return ORC_BAD;
    uint64_t idx = 0;
    int lam = 0;
    for (int k = 0; k < s->N; ++k) {
        uint64_t w = subword(s, st, k);
        int m = s->lsum[k][w];
        if (m < 0 || lam + m > s->n) return ORC_BAD;
        int mk = (s->Q - 1) * s->split[k];
        size_t e = (size_t)lam * (mk + 1) + m;
        idx += s->off[k][e] + s->str[k][e] * s->lidx[k][w];
        lam += m;
    }
    return lam == s->n ? idx : ORC_BAD;
}

/* Alg. iii: find n_k, peel off offset and stride, invert the local table */
uint64_t orc_unrank(const orc_sector *s, uint64_t idx) {
    if (idx >= s->dim) return ORC_BAD;
    uint64_t st = 0;
    int lam = 0;
    for (int k = 0; k < s->N - 1; ++k) {
        int Lk = s->split[k], mk = (s->Q - 1) * Lk, g = s->gamma[k];
        int lo = s->n - lam - (s->Q - 1) * g;
        if (lo < 0) lo = 0;
        int hi = s->n - lam < mk ? s->n - lam : mk;
        int m = -1;
        for (int c = lo; c <= hi; ++c) {
            size_t e = (size_t)lam * (mk + 1) + c;
            uint64_t a = s->off[k][e], len = Dget(s, Lk, c) * s->str[k][e];
            if (idx >= a && idx < a + len) { m = c; break; }
        }
        if (m < 0) return ORC_BAD;
        size_t e = (size_t)lam * (mk + 1) + m;
        idx -= s->off[k][e];
        uint64_t i = idx / s->str[k][e];
        idx -= i * s->str[k][e];
        st |= s->linv[k][s->lstart[k][m] + i] << s->shift[k];
        lam += m;
    }
    int k = s->N - 1;
    int m = s->n - lam;
    if (m < 0 || m > (s->Q - 1) * s->split[k]) return ORC_BAD;
    st |= s->linv[k][s->lstart[k][m] + idx] << s->shift[k];
    return st;
}

void orc_rank_batch(const orc_sector *s, const uint64_t *st, uint64_t *out, int64_t count) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < count; ++i) out[i] = orc_rank(s, st[i]);
}

void orc_unrank_batch(const orc_sector *s, const uint64_t *idx, uint64_t *out, int64_t count) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < count; ++i) out[i] = orc_unrank(s, idx[i]);
}

/* ---- canonical order by nested generation ------------------------------- */

typedef struct {
    int m[ORC_MAXSUB];        /* local particle number per level */
    uint64_t pos[ORC_MAXSUB]; /* position inside the list of words with that digit sum */
    int started, done;
} orc_iter;

static int level_mlo(const orc_sector *s, int k, int lam) {
    int lo = s->n - lam - (s->Q - 1) * s->gamma[k];
    return lo < 0 ? 0 : lo;
}
static int level_mhi(const orc_sector *s, int k, int lam) {
    int mk = (s->Q - 1) * s->split[k];
    return s->n - lam < mk ? s->n - lam : mk;
}

static void reset_from(const orc_sector *s, orc_iter *it, int k0) {
    int lam = 0;
    for (int k = 0; k < k0; ++k) lam += it->m[k];
    for (int k = k0; k < s->N; ++k) {
        it->m[k] = level_mlo(s, k, lam);
        it->pos[k] = 0;
        lam += it->m[k];
    }
}

orc_iter *orc_iter_create(const orc_sector *s) {
    orc_iter *it = (orc_iter *)calloc(1, sizeof(orc_iter));
    reset_from(s, it, 0);
    return it;
}
void orc_iter_free(orc_iter *it) { free(it); }

static uint64_t iter_state(const orc_sector *s, const orc_iter *it) {
    uint64_t st = 0;
    for (int k = 0; k < s->N; ++k)
        st |= s->linv[k][s->lstart[k][it->m[k]] + it->pos[k]] << s->shift[k];
    return st;
}

static int iter_advance(const orc_sector *s, orc_iter *it) {
    for (int k = s->N - 1; k >= 0; --k) {
        int lam = 0;
        for (int j = 0; j < k; ++j) lam += it->m[j];
        uint64_t cnt = s->lstart[k][it->m[k] + 1] - s->lstart[k][it->m[k]];
        if (it->pos[k] + 1 < cnt) {                /* next word, same digit sum */
            it->pos[k]++;
            reset_from(s, it, k + 1);
            return 1;
        }
        if (it->m[k] + 1 <= level_mhi(s, k, lam)) { /* next digit sum */
            it->m[k]++;
            it->pos[k] = 0;
            reset_from(s, it, k + 1);
            return 1;
        }
    }
    return 0;
}

/* Write up to max_count further states of the canonical order; returns how many. */
int64_t orc_iter_next(const orc_sector *s, orc_iter *it, uint64_t *out, int64_t max_count) {
    int64_t c = 0;
    if (it->done) return 0;
    if (!it->started) {
        it->started = 1;
        if (max_count == 0) return 0;
        out[c++] = iter_state(s, it);
    }
    while (c < max_count) {
        if (!iter_advance(s, it)) { it->done = 1; break; }
        out[c++] = iter_state(s, it);
    }
    return c;
}

/* ---- H*x ---------------------------------------------------------------- */

typedef struct {
    int nbonds;
    const int32_t *bi, *bj;
    const double *jxy, *jz, *h;  /* h may be NULL */
} orc_terms;

static inline double xget(const double *x, const float *xf, uint64_t i) {
    return x ? x[i] : (double)xf[i];
}

static void row_apply(const orc_sector *s, const orc_terms *t, const double *x, const float *xf,
                      int k, uint64_t row, double *yrow) {
    const int Q = s->Q, L = s->L, nb = s->nb;
    const double S = 0.5 * (Q - 1);
    const uint64_t dm = (1ull << nb) - 1;
    uint64_t st = orc_unrank(s, row);
    double diag = 0.0;
    for (int c = 0; c < k; ++c) yrow[c] = 0.0;
    for (int b = 0; b < t->nbonds; ++b) {
        int i = t->bi[b], j = t->bj[b];
        int si = nb * (L - 1 - i), sj = nb * (L - 1 - j);
        int di = (int)((st >> si) & dm), dj = (int)((st >> sj) & dm);
        diag += t->jz[b] * (di - S) * (dj - S);
        for (int dir = 0; dir < 2; ++dir) {
            int a_d = dir ? dj : di, c_d = dir ? di : dj;
            int a_s = dir ? sj : si, c_s = dir ? si : sj;
            if (a_d < Q - 1 && c_d > 0) {
                double ma = a_d - S, mc = c_d - S;
                double amp = 0.5 * t->jxy[b] * sqrt(S * (S + 1) - ma * (ma + 1)) *
                             sqrt(S * (S + 1) - mc * (mc - 1));
                uint64_t sp = st + (1ull << a_s) - (1ull << c_s);
                uint64_t col = orc_rank(s, sp);
                for (int c = 0; c < k; ++c) yrow[c] += amp * xget(x, xf, col * (uint64_t)k + c);
            }
        }
    }
    if (t->h)
        for (int i = 0; i < L; ++i) diag += t->h[i] * ((int)((st >> (nb * (L - 1 - i))) & dm) - S);
    for (int c = 0; c < k; ++c) yrow[c] += diag * xget(x, xf, row * (uint64_t)k + c);
}

/* y[r - first] = (H x)_r for r in [first, first + count); x is [dim][k] row-major. */
void orc_hx_range(const orc_sector *s, int nbonds, const int32_t *bi, const int32_t *bj,
                  const double *jxy, const double *jz, const double *h, const double *x, int k,
                  uint64_t first, int64_t count, double *y) {
    orc_terms t = {nbonds, bi, bj, jxy, jz, h};
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < count; ++r) row_apply(s, &t, x, NULL, k, first + r, y + r * k);
}

/* y[i] = (H x)_{rows[i]} for a list of rows. */
void orc_hx_rows(const orc_sector *s, int nbonds, const int32_t *bi, const int32_t *bj,
                 const double *jxy, const double *jz, const double *h, const double *x, int k,
                 const uint64_t *rows, int64_t count, double *y) {
    orc_terms t = {nbonds, bi, bj, jxy, jz, h};
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t r = 0; r < count; ++r) row_apply(s, &t, x, NULL, k, rows[r], y + r * k);
}

/* Same as orc_hx_rows but reading x as FP32 (values widened to FP64). */
void orc_hx_rows_xf32(const orc_sector *s, int nbonds, const int32_t *bi, const int32_t *bj,
                      const double *jxy, const double *jz, const double *h, const float *xf,
                      int k, const uint64_t *rows, int64_t count, double *y) {
    orc_terms t = {nbonds, bi, bj, jxy, jz, h};
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t r = 0; r < count; ++r) row_apply(s, &t, NULL, xf, k, rows[r], y + r * k);
}

/*
 * Coupling and field derivatives of a scalar loss with upstream gradient g for
 * y = H(theta) x (the sums O5 of the gradient definitions; H is linear in the
 * couplings): for every bond b of the list
 *     gxy[b] = sum_r sum_c g[r][c] (A_b x)[r][c],  A_b = (S+_i S-_j + S-_i S+_j)/2,
 *     gz[b]  = sum_r sum_c g[r][c] (Z_b x)[r][c],  Z_b = Sz_i Sz_j,
 * and, if gh != NULL, gh[i] = sum_r sum_c g[r][c] Sz_i(r) x[r][c] for every site,
 * over the rows [first, first + count).  Row by row from the definition (each
 * reached state ranked with eq. index); per-thread partial sums added at the end.
 */
void orc_bond_sums(const orc_sector *s, int nbonds, const int32_t *bi, const int32_t *bj,
                   const double *x, const double *g, int k, uint64_t first, int64_t count,
                   double *gxy, double *gz, double *gh) {
    const int Q = s->Q, L = s->L, nb = s->nb;
    const double S = 0.5 * (Q - 1);
    const uint64_t dm = (1ull << nb) - 1;
    const int nacc = 2 * nbonds + L;
    double *tot = calloc((size_t)nacc, sizeof(double));
#pragma omp parallel
    {
        double *acc = calloc((size_t)nacc, sizeof(double));
#pragma omp for schedule(static)
        for (int64_t r = 0; r < count; ++r) {
            const uint64_t row = first + (uint64_t)r;
            const uint64_t st = orc_unrank(s, row);
            double gx_row = 0.0; /* sum_c g[row][c] x[row][c] */
            for (int c = 0; c < k; ++c) gx_row += g[row * (uint64_t)k + c] * x[row * (uint64_t)k + c];
            for (int b = 0; b < nbonds; ++b) {
                int si = nb * (L - 1 - bi[b]), sj = nb * (L - 1 - bj[b]);
                int di = (int)((st >> si) & dm), dj = (int)((st >> sj) & dm);
                acc[2 * b + 1] += (di - S) * (dj - S) * gx_row;
                for (int dir = 0; dir < 2; ++dir) {
                    int a_d = dir ? dj : di, c_d = dir ? di : dj;
                    int a_s = dir ? sj : si, c_s = dir ? si : sj;
                    if (a_d < Q - 1 && c_d > 0) {
                        double ma = a_d - S, mc = c_d - S;
                        double amp = 0.5 * sqrt(S * (S + 1) - ma * (ma + 1)) * sqrt(S * (S + 1) - mc * (mc - 1));
                        uint64_t col = orc_rank(s, st + (1ull << a_s) - (1ull << c_s));
                        for (int c = 0; c < k; ++c)
                            acc[2 * b] += amp * g[row * (uint64_t)k + c] * x[col * (uint64_t)k + c];
                    }
                }
            }
            if (gh)
                for (int i = 0; i < L; ++i)
                    acc[2 * nbonds + i] += ((int)((st >> (nb * (L - 1 - i))) & dm) - S) * gx_row;
        }
#pragma omp critical
        for (int q = 0; q < nacc; ++q) tot[q] += acc[q];
        free(acc);
    }
    for (int b = 0; b < nbonds; ++b) {
        gxy[b] = tot[2 * b];
        gz[b] = tot[2 * b + 1];
    }
    if (gh)
        for (int i = 0; i < L; ++i) gh[i] = tot[2 * nbonds + i];
    free(tot);
}

void orc_set_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
