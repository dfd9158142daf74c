/*
 * LEAD oracle -- plain single-threaded FP64 reference.  TEST INFRASTRUCTURE
 * ONLY: loaded by the test suite, the smoke check and the benchmark's CPU
 * baseline, never by the decoder library.
 *
 * Section references are to the LEAD paper (arXiv 2605.17796):
 *   Sec. II-A   left-right Cayley complex, squares {(g,0),(ag,1),(gb,1),(agb,0)},
 *               TNC condition, local views Q(v) ~ A x B
 *   Sec. II-B   Z generators C_A (x) C_B on V0, X generators C_A^perp (x) C_B^perp
 *               on V1, CSS condition
 *   Alg. 1      LEAD: Phase 1 local decoding + confidence boost, Phase 2
 *               soft-information regularisation, Phase 3 global decoding
 *   Sec. IV-A   success criterion (residual in the stabiliser group)
 *   Appendix A  worked example of the local check layout and aggregation
 *
 * Readings of points the paper leaves open are the ones listed in the design
 * notes: min-sum with scale beta, flooding schedule, sgn(0)=+1, e=[L<0],
 * magnitudes clamped to llr_clamp, probability-domain boost and averaging,
 * RREF(G_A) (x) RREF(G_B) local check rows in a-major order, V1 local
 * coordinates (a,b) -> square (h*b, a, b^-1).
 */
#include "lead_oracle.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ */
/* small helpers                                                       */
/* ------------------------------------------------------------------ */

static void set_err(char *err, int errlen, const char *msg) {
    if (err && errlen > 0) {
        strncpy(err, msg, (size_t)errlen - 1);
        err[errlen - 1] = 0;
    }
}

static int get_bit(const uint64_t *w, int i) { return (int)((w[i >> 6] >> (i & 63)) & 1u); }
static void put_bit(uint64_t *w, int i, int b) {
    if (b) w[i >> 6] |= (uint64_t)1 << (i & 63);
    else   w[i >> 6] &= ~((uint64_t)1 << (i & 63));
}
static int popcount64(uint64_t x) { int c = 0; while (x) { x &= x - 1; c++; } return c; }
static double clampd(double x, double lim) { return x > lim ? lim : (x < -lim ? -lim : x); }

/* GF(2) matrix with packed rows. */
typedef struct { int rows, cols, words; uint64_t *d; } bitmat;

static bitmat bm_new(int rows, int cols) {
    bitmat m; m.rows = rows; m.cols = cols; m.words = (cols + 63) / 64;
    m.d = (uint64_t *)calloc((size_t)(rows > 0 ? rows : 1) * (size_t)m.words, sizeof(uint64_t));
    return m;
}
static uint64_t *bm_row(const bitmat *m, int r) { return m->d + (size_t)r * (size_t)m->words; }
static void bm_free(bitmat *m) { free(m->d); m->d = NULL; }

/* In-place reduced row echelon form; returns the rank.  pivots[r] = pivot
 * column of row r for r < rank (pivots may be NULL). */
static int bm_rref(bitmat *m, int *pivots) {
    int rank = 0;
    for (int col = 0; col < m->cols && rank < m->rows; col++) {
        int piv = -1;
        for (int r = rank; r < m->rows; r++)
            if (get_bit(bm_row(m, r), col)) { piv = r; break; }
        if (piv < 0) continue;
        if (piv != rank) {
            uint64_t *a = bm_row(m, piv), *b = bm_row(m, rank);
            for (int w = 0; w < m->words; w++) { uint64_t t = a[w]; a[w] = b[w]; b[w] = t; }
        }
        uint64_t *pr = bm_row(m, rank);
        for (int r = 0; r < m->rows; r++) {
            if (r == rank) continue;
            uint64_t *rr = bm_row(m, r);
            if (get_bit(rr, col))
                for (int w = 0; w < m->words; w++) rr[w] ^= pr[w];
        }
        if (pivots) pivots[rank] = col;
        rank++;
    }
    return rank;
}

/* Reduce vector v (cols bits) against an RREF matrix with given pivots. */
static void bm_reduce(const bitmat *rref, const int *pivots, int rank, uint64_t *v) {
    for (int r = 0; r < rank; r++)
        if (get_bit(v, pivots[r])) {
            const uint64_t *pr = bm_row(rref, r);
            for (int w = 0; w < rref->words; w++) v[w] ^= pr[w];
        }
}

/* ------------------------------------------------------------------ */
/* the code                                                            */
/* ------------------------------------------------------------------ */

typedef struct {
    /* a check matrix as explicit edge lists (the Tanner graph) */
    int rows, cols, nedges;
    int *row_ptr, *row_col;      /* edges of check c: row_col[row_ptr[c] .. row_ptr[c+1]) */
    int *col_ptr, *col_edge;     /* edges touching variable j (indices into row order)     */
} tanner;

struct oracle_code {
    int order, delta, kA, kB;
    int n, r[2], m[2], rank[2], k, eloc[2];
    int *view[2];                 /* [order][delta^2] qubit ids          */
    uint8_t *hloc[2];             /* [r][delta^2]                          */
    uint8_t *H[2];                /* [m][n] dense                          */
    tanner loc[2], glob[2];
    bitmat rref_other[2];         /* RREF of the other type's H (rowspace test) */
    int *piv_other[2];
    int rank_other[2];
    bitmat logical[2];            /* k rows: operators that detect failure      */
};

static void tanner_from_dense(tanner *t, int rows, int cols, const uint8_t *H) {
    t->rows = rows; t->cols = cols;
    t->row_ptr = (int *)calloc((size_t)rows + 1, sizeof(int));
    int ne = 0;
    for (int c = 0; c < rows; c++) {
        t->row_ptr[c] = ne;
        for (int j = 0; j < cols; j++) ne += H[(size_t)c * cols + j] ? 1 : 0;
    }
    t->row_ptr[rows] = ne;
    t->nedges = ne;
    t->row_col = (int *)malloc(sizeof(int) * (size_t)(ne > 0 ? ne : 1));
    int e = 0;
    for (int c = 0; c < rows; c++)
        for (int j = 0; j < cols; j++)
            if (H[(size_t)c * cols + j]) t->row_col[e++] = j;
    t->col_ptr = (int *)calloc((size_t)cols + 1, sizeof(int));
    for (e = 0; e < ne; e++) t->col_ptr[t->row_col[e] + 1]++;
    for (int j = 0; j < cols; j++) t->col_ptr[j + 1] += t->col_ptr[j];
    int *fill = (int *)calloc((size_t)cols, sizeof(int));
    t->col_edge = (int *)malloc(sizeof(int) * (size_t)(ne > 0 ? ne : 1));
    for (int c = 0; c < rows; c++)
        for (e = t->row_ptr[c]; e < t->row_ptr[c + 1]; e++) {
            int j = t->row_col[e];
            t->col_edge[t->col_ptr[j] + fill[j]++] = e;
        }
    free(fill);
}

static void tanner_free(tanner *t) {
    free(t->row_ptr); free(t->row_col); free(t->col_ptr); free(t->col_edge);
}

void oracle_free(oracle_code *c) {
    if (!c) return;
    for (int t = 0; t < 2; t++) {
        free(c->view[t]); free(c->hloc[t]); free(c->H[t]);
        tanner_free(&c->loc[t]); tanner_free(&c->glob[t]);
        bm_free(&c->rref_other[t]); free(c->piv_other[t]); bm_free(&c->logical[t]);
    }
    free(c);
}

/* RREF basis of the row space spanned by `k` rows of length `len`; also the
 * RREF basis of its dual (length-len vectors orthogonal to every row).
 * Returns the rank; rows written as u64 with bit c = coordinate c. */
static int local_code_bases(int len, int k, const uint64_t *gen, uint64_t *rref_rows,
                            uint64_t *dual_rows, int *dual_count) {
    bitmat g = bm_new(k, len);
    for (int i = 0; i < k; i++) bm_row(&g, i)[0] = gen[i];
    int piv[64];
    int rank = bm_rref(&g, piv);
    for (int i = 0; i < rank; i++) rref_rows[i] = bm_row(&g, i)[0];
    /* null space: one vector per free column f: x_f = 1, x_piv(r) = g[r][f] */
    bitmat ns = bm_new(len - rank > 0 ? len - rank : 1, len);
    int nn = 0;
    for (int f = 0; f < len; f++) {
        int is_piv = 0;
        for (int r = 0; r < rank; r++) if (piv[r] == f) is_piv = 1;
        if (is_piv) continue;
        uint64_t v = (uint64_t)1 << f;
        for (int r = 0; r < rank; r++)
            if ((rref_rows[r] >> f) & 1) v |= (uint64_t)1 << piv[r];
        bm_row(&ns, nn)[0] = v;
        nn++;
    }
    ns.rows = nn;
    int drank = bm_rref(&ns, NULL);
    for (int i = 0; i < drank; i++) dual_rows[i] = bm_row(&ns, i)[0];
    *dual_count = drank;
    bm_free(&g); bm_free(&ns);
    return rank;
}

/* minimum weight of a non-zero vector in the span of `k` rows (k small) */
static int min_distance(int k, const uint64_t *rows) {
    int best = 1 << 30;
    for (long combo = 1; combo < (1L << k); combo++) {
        uint64_t w = 0;
        for (int i = 0; i < k; i++) if ((combo >> i) & 1) w ^= rows[i];
        int pc = popcount64(w);
        if (pc < best) best = pc;
    }
    return best;
}

int oracle_build(int order, const uint16_t *mul, int delta, const int *A, const int *B,
                 int kA, const uint64_t *GA, int kB, const uint64_t *GB,
                 oracle_code **out, char *err, int errlen) {
    char msg[256];
    *out = NULL;
    if (order < 1 || delta < 2 || delta > 8 || kA < 1 || kA >= delta || kB < 1 || kB >= delta) {
        set_err(err, errlen, "argument out of range (2 <= delta <= 8, 1 <= k < delta)");
        return -1;
    }
    const int N = order, D = delta, D2 = delta * delta;

    /* ---- O-1: group axioms by brute force (Sec. II-A takes G a finite group) */
    for (int i = 0; i < N * N; i++)
        if (mul[i] >= N) { set_err(err, errlen, "table entry out of range"); return -2; }
    int e = -1;
    for (int x = 0; x < N && e < 0; x++) {
        int ok = 1;
        for (int g = 0; g < N; g++)
            if (mul[x * N + g] != g || mul[g * N + x] != g) { ok = 0; break; }
        if (ok) e = x;
    }
    if (e < 0) { set_err(err, errlen, "no identity element"); return -2; }
    for (int a = 0; a < N; a++)
        for (int b = 0; b < N; b++)
            for (int c = 0; c < N; c++)
                if (mul[mul[a * N + b] * N + c] != mul[a * N + mul[b * N + c]]) {
                    set_err(err, errlen, "table is not associative");
                    return -2;
                }
    int *inv = (int *)malloc(sizeof(int) * (size_t)N);
    for (int g = 0; g < N; g++) {
        inv[g] = -1;
        for (int h = 0; h < N; h++) if (mul[g * N + h] == e && mul[h * N + g] == e) { inv[g] = h; break; }
        if (inv[g] < 0) { free(inv); set_err(err, errlen, "element without inverse"); return -2; }
    }

    /* ---- O-2: A = A^-1, B = B^-1, identity excluded, distinct, TNC */
    int iotaA[8], iotaB[8];
    for (int s = 0; s < 2; s++) {
        const int *S = s == 0 ? A : B;
        int *iota = s == 0 ? iotaA : iotaB;
        for (int i = 0; i < D; i++) {
            if (S[i] < 0 || S[i] >= N) { free(inv); set_err(err, errlen, "generator out of range"); return -1; }
            if (S[i] == e) { free(inv); set_err(err, errlen, "generating set contains the identity"); return -3; }
            for (int j = 0; j < i; j++)
                if (S[j] == S[i]) { free(inv); set_err(err, errlen, "generating set has a repeated element"); return -3; }
        }
        for (int i = 0; i < D; i++) {
            iota[i] = -1;
            for (int j = 0; j < D; j++) if (S[j] == inv[S[i]]) iota[i] = j;
            if (iota[i] < 0) {
                snprintf(msg, sizeof msg, "set %c is not closed under inverses (element %d)", s ? 'B' : 'A', S[i]);
                free(inv); set_err(err, errlen, msg); return -3;
            }
        }
    }
    for (int i = 0; i < D; i++)
        for (int j = 0; j < D; j++)
            for (int g = 0; g < N; g++)
                if (mul[A[i] * N + g] == mul[g * N + B[j]]) {
                    snprintf(msg, sizeof msg, "TNC violated: a=%d g=%d b=%d", A[i], g, B[j]);
                    free(inv); set_err(err, errlen, msg); return -4;
                }

    oracle_code *c = (oracle_code *)calloc(1, sizeof(oracle_code));
    c->order = N; c->delta = D; c->kA = kA; c->kB = kB;

    /* ---- O-3: local codes, RREF bases of C and C^perp, distances */
    uint64_t gA[8], hA[8], gB[8], hB[8];
    int dA, dB;
    int rA = local_code_bases(D, kA, GA, gA, hA, &dA);
    int rB = local_code_bases(D, kB, GB, gB, hB, &dB);
    if (rA != kA || rB != kB) { free(inv); oracle_free(c); set_err(err, errlen, "local generator matrix is not full rank"); return -5; }
    if (min_distance(kA, gA) < 2 || min_distance(kB, gB) < 2 ||
        min_distance(dA, hA) < 2 || min_distance(dB, hB) < 2) {
        free(inv); oracle_free(c); set_err(err, errlen, "local code or its dual has distance < 2"); return -5;
    }

    /* ---- O-4: squares.  Triple (g,i,j) is the square
     *      {(g,0), (A_i g,1), (g B_j,1), (A_i g B_j,0)}; its other V0
     *      representative is (A_i g B_j, iotaA(i), iotaB(j)).  Qubit id =
     *      rank of the lexicographically smaller representative. */
    int ntrip = N * D2;
    int *qid = (int *)malloc(sizeof(int) * (size_t)ntrip);
    int nq = 0;
    for (int g = 0; g < N; g++)
        for (int i = 0; i < D; i++)
            for (int j = 0; j < D; j++) {
                int g2 = mul[mul[A[i] * N + g] * N + B[j]];
                int i2 = iotaA[i], j2 = iotaB[j];
                int t1 = (g * D + i) * D + j, t2 = (g2 * D + i2) * D + j2;
                if (t1 == t2) { free(inv); free(qid); oracle_free(c); set_err(err, errlen, "degenerate square"); return -4; }
                if (t1 < t2) qid[t1] = nq++;
            }
    for (int g = 0; g < N; g++)
        for (int i = 0; i < D; i++)
            for (int j = 0; j < D; j++) {
                int g2 = mul[mul[A[i] * N + g] * N + B[j]];
                int t1 = (g * D + i) * D + j, t2 = (g2 * D + iotaA[i]) * D + iotaB[j];
                if (t1 > t2) qid[t1] = qid[t2];
            }
    c->n = nq;

    /* ---- O-5: views.  V0: view0[g][i*D+j] = qubit(g,i,j) (eq. of the square set).
     *      V1: view1[h][i*D+j] = qubit(h*B_j, i, iotaB(j)), the square whose
     *      corner (g B_j',1) is (h,1). */
    for (int t = 0; t < 2; t++) c->view[t] = (int *)malloc(sizeof(int) * (size_t)ntrip);
    for (int g = 0; g < N; g++)
        for (int i = 0; i < D; i++)
            for (int j = 0; j < D; j++) {
                c->view[0][g * D2 + i * D + j] = qid[(g * D + i) * D + j];
                int g1 = mul[g * N + B[j]];
                c->view[1][g * D2 + i * D + j] = qid[(g1 * D + i) * D + iotaB[j]];
            }
    free(qid);
    free(inv);

    /* ---- O-6: local checks (rows rA*kB + rB, columns a*D + b) and global H */
    int kk[2][2] = {{kA, kB}, {dA, dB}};
    const uint64_t *rowsA[2] = {gA, hA}, *rowsB[2] = {gB, hB};
    for (int t = 0; t < 2; t++) {
        int ra = kk[t][0], rb = kk[t][1];
        int r = ra * rb;
        c->r[t] = r;
        c->hloc[t] = (uint8_t *)calloc((size_t)r * D2, 1);
        for (int x = 0; x < ra; x++)
            for (int y = 0; y < rb; y++)
                for (int a = 0; a < D; a++)
                    for (int b = 0; b < D; b++)
                        c->hloc[t][(size_t)(x * rb + y) * D2 + a * D + b] =
                            (uint8_t)(((rowsA[t][x] >> a) & 1) & ((rowsB[t][y] >> b) & 1));
        c->m[t] = N * r;
        c->H[t] = (uint8_t *)calloc((size_t)c->m[t] * (size_t)c->n, 1);
        for (int v = 0; v < N; v++)
            for (int rho = 0; rho < r; rho++)
                for (int jj = 0; jj < D2; jj++)
                    if (c->hloc[t][(size_t)rho * D2 + jj])
                        c->H[t][(size_t)(v * r + rho) * c->n + c->view[t][v * D2 + jj]] ^= 1;
        tanner_from_dense(&c->loc[t], r, D2, c->hloc[t]);
        tanner_from_dense(&c->glob[t], c->m[t], c->n, c->H[t]);
        c->eloc[t] = c->loc[t].nedges;
    }

    /* ---- O-7: CSS condition (every X row orthogonal to every Z row), ranks,
     *      k, logical operators */
    bitmat Hb[2];
    int *piv[2];
    for (int t = 0; t < 2; t++) {
        Hb[t] = bm_new(c->m[t], c->n);
        for (int row = 0; row < c->m[t]; row++)
            for (int q = 0; q < c->n; q++)
                if (c->H[t][(size_t)row * c->n + q]) put_bit(bm_row(&Hb[t], row), q, 1);
    }
    for (int x = 0; x < c->m[1]; x++)
        for (int z = 0; z < c->m[0]; z++) {
            int par = 0;
            const uint64_t *hx = bm_row(&Hb[1], x), *hz = bm_row(&Hb[0], z);
            for (int w = 0; w < Hb[0].words; w++) par ^= popcount64(hx[w] & hz[w]) & 1;
            if (par) {
                bm_free(&Hb[0]); bm_free(&Hb[1]); oracle_free(c);
                set_err(err, errlen, "CSS condition H_X H_Z^T = 0 fails");
                return -5;
            }
        }
    for (int t = 0; t < 2; t++) {
        piv[t] = (int *)malloc(sizeof(int) * (size_t)(c->m[t] > 0 ? c->m[t] : 1));
        c->rank[t] = bm_rref(&Hb[t], piv[t]);
    }
    c->k = c->n - c->rank[0] - c->rank[1];
    /* For check type t the residual is an error of the kind H_t detects; it is
     * trivial iff it lies in the row space of the other type (those are the
     * stabilisers of the same Pauli kind).  Logicals: a basis of
     * ker(H_other) modulo rowspace(H_t). */
    for (int t = 0; t < 2; t++) {
        int o = 1 - t;
        c->rref_other[t] = Hb[o];           /* shared storage, freed once below */
        c->piv_other[t] = piv[o];
        c->rank_other[t] = c->rank[o];
    }
    for (int t = 0; t < 2; t++) {
        int o = 1 - t;
        /* kernel of H_other from its RREF */
        const bitmat *R = &Hb[o];
        int rank = c->rank[o];
        char *is_piv = (char *)calloc((size_t)c->n, 1);
        for (int rr = 0; rr < rank; rr++) is_piv[piv[o][rr]] = 1;
        /* basis being built: rows of H_t then accepted logicals, kept in RREF-like form */
        bitmat span = bm_new(c->m[t] + c->k + 1, c->n);
        int *spiv = (int *)malloc(sizeof(int) * (size_t)(c->m[t] + c->k + 1));
        int srank = 0;
        for (int rr = 0; rr < c->rank[t]; rr++) {
            memcpy(bm_row(&span, srank), bm_row(&Hb[t], rr), sizeof(uint64_t) * (size_t)span.words);
            spiv[srank] = piv[t][rr];
            srank++;
        }
        c->logical[t] = bm_new(c->k > 0 ? c->k : 1, c->n);
        c->logical[t].rows = 0;
        uint64_t *vec = (uint64_t *)calloc((size_t)span.words, sizeof(uint64_t));
        uint64_t *red = (uint64_t *)calloc((size_t)span.words, sizeof(uint64_t));
        for (int f = 0; f < c->n && c->logical[t].rows < c->k; f++) {
            if (is_piv[f]) continue;
            memset(vec, 0, sizeof(uint64_t) * (size_t)span.words);
            put_bit(vec, f, 1);
            for (int rr = 0; rr < rank; rr++)
                if (get_bit(bm_row(R, rr), f)) put_bit(vec, piv[o][rr], 1);
            /* reduce against the current span (rows with distinct pivots, each
             * reduced so that its pivot is its lowest set column among pivots) */
            memcpy(red, vec, sizeof(uint64_t) * (size_t)span.words);
            for (int rr = 0; rr < srank; rr++)
                if (get_bit(red, spiv[rr]))
                    for (int w = 0; w < span.words; w++) red[w] ^= bm_row(&span, rr)[w];
            int p = -1;
            for (int q = 0; q < c->n; q++) if (get_bit(red, q)) { p = q; break; }
            if (p < 0) continue;
            /* keep the span's rows eliminated at the new pivot */
            for (int rr = 0; rr < srank; rr++)
                if (get_bit(bm_row(&span, rr), p))
                    for (int w = 0; w < span.words; w++) bm_row(&span, rr)[w] ^= red[w];
            memcpy(bm_row(&span, srank), red, sizeof(uint64_t) * (size_t)span.words);
            spiv[srank++] = p;
            memcpy(bm_row(&c->logical[t], c->logical[t].rows), vec, sizeof(uint64_t) * (size_t)span.words);
            c->logical[t].rows++;
        }
        free(vec); free(red); free(spiv); free(is_piv); bm_free(&span);
    }
    /* Hb[0] is rref_other[1], Hb[1] is rref_other[0]: owned there. */
    *out = c;
    return 0;
}

void oracle_info(const oracle_code *c, int *info) {
    info[OI_ORDER] = c->order; info[OI_DELTA] = c->delta; info[OI_N] = c->n;
    info[OI_RZ] = c->r[0]; info[OI_RX] = c->r[1]; info[OI_MZ] = c->m[0]; info[OI_MX] = c->m[1];
    info[OI_RANKZ] = c->rank[0]; info[OI_RANKX] = c->rank[1]; info[OI_K] = c->k;
    info[OI_ELOCZ] = c->eloc[0]; info[OI_ELOCX] = c->eloc[1];
}

void oracle_views(const oracle_code *c, int type, int32_t *out) {
    for (int i = 0; i < c->order * c->delta * c->delta; i++) out[i] = c->view[type][i];
}

void oracle_hloc(const oracle_code *c, int type, uint8_t *out) {
    memcpy(out, c->hloc[type], (size_t)c->r[type] * c->delta * c->delta);
}

void oracle_H(const oracle_code *c, int type, uint8_t *out) {
    memcpy(out, c->H[type], (size_t)c->m[type] * (size_t)c->n);
}

void oracle_logicals(const oracle_code *c, int type, uint8_t *out) {
    for (int l = 0; l < c->logical[type].rows; l++)
        for (int q = 0; q < c->n; q++) out[(size_t)l * c->n + q] = (uint8_t)get_bit(bm_row(&c->logical[type], l), q);
}

void oracle_syndrome(const oracle_code *c, int type, int shots, const uint64_t *err,
                     int err_words, uint64_t *synd, int synd_words) {
    const tanner *t = &c->glob[type];
    for (int s = 0; s < shots; s++) {
        const uint64_t *e = err + (size_t)s * err_words;
        uint64_t *out = synd + (size_t)s * synd_words;
        memset(out, 0, sizeof(uint64_t) * (size_t)synd_words);
        for (int row = 0; row < t->rows; row++) {
            int par = 0;
            for (int x = t->row_ptr[row]; x < t->row_ptr[row + 1]; x++) par ^= get_bit(e, t->row_col[x]);
            put_bit(out, row, par);
        }
    }
}

/* ------------------------------------------------------------------ */
/* belief propagation (the LocalDecoder / GlobalDecoder of Alg. 1)      */
/* ------------------------------------------------------------------ */

typedef struct { double *msg, *mu; uint64_t rng; } bp_work;

/* SplitMix64 (Steele, Lea, Flood 2014): the perturbation stream. */
static uint64_t splitmix64(uint64_t *state) {
    uint64_t z = (*state += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* x * (1 + eps * xi), xi uniform in [-1, 1); identity when eps == 0. */
static double perturbed(double x, double eps, uint64_t *state) {
    if (eps == 0.0) return x;
    double xi = (double)(splitmix64(state) >> 11) * (1.0 / 9007199254740992.0) * 2.0 - 1.0;
    return x * (1.0 + eps * xi);
}

/* Flooding BP on Tanner graph t.
 *   mu_{j->c} = clamp(lam_j + sum_{c' ni j, c' != c} m_{c'->j})
 *   min-sum:  m_{c->j} = beta (-1)^{s_c} prod_{j'!=j} sgn(mu_{j'->c}) min_{j'!=j} |mu_{j'->c}|
 *   sum-prod: m_{c->j} = (-1)^{s_c} 2 atanh(prod_{j'!=j} tanh(mu_{j'->c}/2))
 *   L_j = clamp(lam_j + sum_{c ni j} m_{c->j}),  e_j = [L_j < 0]
 * stopping after iteration t if early_exit and H e = s.  Returns iterations
 * run; *conv = [H e = s] at the end.  *margin lowered to the smallest |mu| or
 * |L| computed. */
static int bp_run(const tanner *t, const uint8_t *s, const double *lam, const oracle_params *p,
                  int max_iter, double *L, uint8_t *e, int *conv, double *margin, bp_work *w) {
    const double lim = p->llr_clamp;
    for (int x = 0; x < t->nedges; x++) w->msg[x] = 0.0;
    int it = 0, ok = 0;
    for (int iter = 1; iter <= max_iter; iter++) {
        it = iter;
        /* variable-to-check messages, each excluding its own check */
        for (int c = 0; c < t->rows; c++)
            for (int x = t->row_ptr[c]; x < t->row_ptr[c + 1]; x++) {
                int j = t->row_col[x];
                double acc = lam[j];
                for (int y = t->col_ptr[j]; y < t->col_ptr[j + 1]; y++)
                    if (t->col_edge[y] != x) acc += w->msg[t->col_edge[y]];
                w->mu[x] = clampd(perturbed(acc, p->perturb, &w->rng), lim);
                if (margin && fabs(w->mu[x]) < *margin) *margin = fabs(w->mu[x]);
            }
        /* check-to-variable messages, each excluding its own variable */
        for (int c = 0; c < t->rows; c++)
            for (int x = t->row_ptr[c]; x < t->row_ptr[c + 1]; x++) {
                double out;
                if (p->bp == OR_MINSUM) {
                    int neg = s[c] ? 1 : 0;
                    double mn = INFINITY;
                    for (int y = t->row_ptr[c]; y < t->row_ptr[c + 1]; y++) {
                        if (y == x) continue;
                        if (w->mu[y] < 0) neg ^= 1;       /* sgn(0) = +1 */
                        if (fabs(w->mu[y]) < mn) mn = fabs(w->mu[y]);
                    }
                    out = p->ms_scale * (neg ? -mn : mn);
                } else {
                    /* in extended precision: near saturation the product is
                     * 1 - O(e^-|mu|) (1 - 2e-13 at |mu| = 30), and in double
                     * its distance from 1, which sets the message, would keep
                     * only three or four digits (message errors up to 6e-4) */
                    long double prod = s[c] ? -1.0L : 1.0L;
                    for (int y = t->row_ptr[c]; y < t->row_ptr[c + 1]; y++) {
                        if (y == x) continue;
                        prod *= tanhl((long double)w->mu[y] / 2.0L);
                    }
                    out = (double)(2.0L * atanhl(prod));
                }
                w->msg[x] = perturbed(out, p->perturb, &w->rng);
            }
        /* posteriors and hard decisions */
        for (int j = 0; j < t->cols; j++) {
            double acc = lam[j];
            for (int y = t->col_ptr[j]; y < t->col_ptr[j + 1]; y++) acc += w->msg[t->col_edge[y]];
            L[j] = clampd(perturbed(acc, p->perturb, &w->rng), lim);
            if (margin && fabs(L[j]) < *margin) *margin = fabs(L[j]);
            e[j] = L[j] < 0 ? 1 : 0;
        }
        ok = 1;
        for (int c = 0; c < t->rows && ok; c++) {
            int par = 0;
            for (int x = t->row_ptr[c]; x < t->row_ptr[c + 1]; x++) par ^= e[t->row_col[x]];
            if (par != (s[c] ? 1 : 0)) ok = 0;
        }
        if (ok && p->early_exit) break;
    }
    if (max_iter < 1) {
        for (int j = 0; j < t->cols; j++) { L[j] = clampd(lam[j], lim); e[j] = L[j] < 0; }
        ok = 1;
        for (int c = 0; c < t->rows && ok; c++) {
            int par = 0;
            for (int x = t->row_ptr[c]; x < t->row_ptr[c + 1]; x++) par ^= e[t->row_col[x]];
            if (par != (s[c] ? 1 : 0)) ok = 0;
        }
    }
    *conv = ok;
    return it;
}

static void work_alloc(bp_work *w, int nedges) {
    w->rng = 0;
    w->msg = (double *)malloc(sizeof(double) * (size_t)(nedges > 0 ? nedges : 1));
    w->mu = (double *)malloc(sizeof(double) * (size_t)(nedges > 0 ? nedges : 1));
}
static void work_free(bp_work *w) { free(w->msg); free(w->mu); }

int oracle_bp(int rows, int cols, const uint8_t *H, const uint8_t *s, const double *lam,
              const oracle_params *p, int max_iter, double *L, uint8_t *e, int *conv) {
    tanner t;
    tanner_from_dense(&t, rows, cols, H);
    bp_work w;
    work_alloc(&w, t.nedges);
    int it = bp_run(&t, s, lam, p, max_iter, L, e, conv, NULL, &w);
    work_free(&w);
    tanner_free(&t);
    return it;
}

/* ------------------------------------------------------------------ */
/* Ordered statistics decoding (post-processing of local and global BP) */
/* ------------------------------------------------------------------ */

/* Cost unit of the combination sweep: the weight ln(1/p_j) of setting bit j,
 * with p_j = 1 / (1 + e^{lambda_j}) the probability the decoder's prior
 * gives it, in units of 1/64 and rounded to the nearest integer, so that
 * candidate costs are exact integer sums:
 *   ln(1/p) = ln(1 + e^lambda) = max(lambda, 0) + log1p(e^{-|lambda|}). */
long oracle_osd_weight(double lambda) {
    const double w = (lambda > 0.0 ? lambda : 0.0) + log1p(exp(-fabs(lambda)));
    return (long)nearbyint(64.0 * w);
}

/* Ordered statistics decoding of H e = s (H: rows x cols, dense).  The
 * variables are ranked by their BP posterior LLR L, most likely in error
 * first: by round(64 L) ascending, equal keys in position order
 * (reliabilities that agree to 1/64 count as equal, so exact ties of
 * symmetric positions stay ties under last-digit rounding).  Gauss-Jordan
 * elimination over GF(2) takes the columns in that order; the first `rank`
 * linearly independent ones form the information set S, the others (in rank
 * order) the set T.
 *   order 0 (OSD-0): the estimate is the solution supported on S.
 *   order lambda >= 1 (combination sweep): candidates are the OSD-0
 *   solution, then for every column t of T the solution with e_T = {t},
 *   then for every pair a < b among the first lambda columns of T the one
 *   with e_T = {a, b} (e_S follows from e_T: e_S = s' + A e_T in the reduced
 *   system [I | A | s']).  The estimate is the first candidate of least cost
 *   sum over set bits of oracle_osd_weight(prior[j]).
 * Returns 0, or -1 when s is not in the column space of H (e is then all
 * zero). */
static double osd_weight_exact(double lambda) {
    return (lambda > 0.0 ? lambda : 0.0) + log1p(exp(-fabs(lambda)));
}

int oracle_osd(int rows, int cols, const uint8_t *H, const uint8_t *s, const double *L,
               const double *prior, int order, uint8_t *e) {
    return oracle_osd_ex(rows, cols, H, s, L, prior, order, 0, e);
}

/* exact = 1: keys are L itself and candidate costs sums of
 * osd_weight_exact (FP64), otherwise as described above. */
int oracle_osd_ex(int rows, int cols, const uint8_t *H, const uint8_t *s, const double *L,
                  const double *prior, int order, int exact, uint8_t *e) {
    const int words = cols / 64 + 1;          /* bit `cols` holds s */
    int *ord = (int *)malloc(sizeof(int) * (size_t)cols);
    int *pivcol = (int *)malloc(sizeof(int) * (size_t)(rows > 0 ? rows : 1));
    uint8_t *ispiv = (uint8_t *)calloc((size_t)(cols > 0 ? cols : 1), 1);
    double *key = (double *)malloc(sizeof(double) * (size_t)(cols > 0 ? cols : 1));
    uint64_t *M = (uint64_t *)calloc((size_t)rows * words, sizeof(uint64_t));
    for (int j = 0; j < cols; j++) {
        ord[j] = j;
        key[j] = exact ? L[j] : nearbyint(L[j] * 64.0);   /* round half to even */
    }
    for (int a = 1; a < cols; a++) {          /* stable insertion sort */
        int x = ord[a], b = a;
        while (b > 0 && key[ord[b - 1]] > key[x]) { ord[b] = ord[b - 1]; b--; }
        ord[b] = x;
    }
    /* augmented rows [H | s], bit-packed */
    for (int r = 0; r < rows; r++) {
        uint64_t *row = M + (size_t)r * words;
        for (int j = 0; j < cols; j++)
            if (H[(size_t)r * cols + j]) row[j >> 6] |= 1ull << (j & 63);
        if (s[r]) row[cols >> 6] |= 1ull << (cols & 63);
    }
    int rank = 0;
    for (int t = 0; t < cols && rank < rows; t++) {
        const int c = ord[t];
        int pr = -1;
        for (int r = rank; r < rows; r++)
            if ((M[(size_t)r * words + (c >> 6)] >> (c & 63)) & 1) { pr = r; break; }
        if (pr < 0) continue;                 /* dependent on the columns before it */
        uint64_t *P = M + (size_t)rank * words;
        if (pr != rank)
            for (int w = 0; w < words; w++) {
                uint64_t tmp = M[(size_t)pr * words + w];
                M[(size_t)pr * words + w] = P[w];
                P[w] = tmp;
            }
        for (int r = 0; r < rows; r++) {
            uint64_t *row = M + (size_t)r * words;
            if (r != rank && ((row[c >> 6] >> (c & 63)) & 1))
                for (int w = 0; w < words; w++) row[w] ^= P[w];
        }
        ispiv[c] = 1;
        pivcol[rank++] = c;
    }
#define OSD_BIT(r, j) ((int)((M[(size_t)(r) * words + ((j) >> 6)] >> ((j) & 63)) & 1))
    int ok = 1;
    for (int r = rank; r < rows; r++)
        if (OSD_BIT(r, cols)) ok = 0;
    memset(e, 0, (size_t)cols);
    if (ok) {
        for (int k = 0; k < rank; k++) e[pivcol[k]] = (uint8_t)OSD_BIT(k, cols);
        if (order > 0 && rank < cols) {
            /* T in rank order */
            int nt = 0;
            int *T = (int *)malloc(sizeof(int) * (size_t)cols);
            double *q = (double *)malloc(sizeof(double) * (size_t)cols);
            for (int t = 0; t < cols; t++)
                if (!ispiv[ord[t]]) T[nt++] = ord[t];
            /* integer weights are exact in a double (|w| < 2^53), so the
             * sums below are the integer sums */
            for (int j = 0; j < cols; j++)
                q[j] = exact ? osd_weight_exact(prior[j]) : (double)oracle_osd_weight(prior[j]);
            /* cost of the candidate with e_T = {a} or {a, b} (b < 0: none) */
            double best = 0;
            int ba = -1, bb = -1;
            for (int k = 0; k < rank; k++)
                if (OSD_BIT(k, cols)) best += q[pivcol[k]];
            for (int x = 0; x < nt; x++) {
                const int a = T[x];
                double c = q[a];
                for (int k = 0; k < rank; k++)
                    if (OSD_BIT(k, cols) ^ OSD_BIT(k, a)) c += q[pivcol[k]];
                if (c < best) { best = c; ba = a; bb = -1; }
            }
            const int lam = order < nt ? order : nt;
            for (int x = 0; x < lam; x++)
                for (int y = x + 1; y < lam; y++) {
                    const int a = T[x], b = T[y];
                    double c = q[a] + q[b];
                    for (int k = 0; k < rank; k++)
                        if (OSD_BIT(k, cols) ^ OSD_BIT(k, a) ^ OSD_BIT(k, b)) c += q[pivcol[k]];
                    if (c < best) { best = c; ba = a; bb = b; }
                }
            if (ba >= 0) {
                for (int k = 0; k < rank; k++)
                    e[pivcol[k]] = (uint8_t)(OSD_BIT(k, cols) ^ OSD_BIT(k, ba) ^ (bb >= 0 ? OSD_BIT(k, bb) : 0));
                e[ba] = 1;
                if (bb >= 0) e[bb] = 1;
            }
            free(T); free(q);
        }
    }
#undef OSD_BIT
    free(ord); free(pivcol); free(ispiv); free(key); free(M);
    return ok ? 0 : -1;
}

int oracle_osd0(int rows, int cols, const uint8_t *H, const uint8_t *s, const double *L, uint8_t *e) {
    return oracle_osd(rows, cols, H, s, L, NULL, 0, e);
}

/* ------------------------------------------------------------------ */
/* LEAD (Algorithm 1)                                                   */
/* ------------------------------------------------------------------ */

/* Phase 2 of Alg. 1: for each qubit i, p_i = alpha * Average{p_{v,i} over
 * every view v whose support holds i}, returned as an LLR
 * lambda'_i = clamp(ln(1 - p_i) - ln p_i).  view: nviews x vsize qubit ids;
 * pv: nviews x vsize local error probabilities. */
void oracle_aggregate(int n, int nviews, int vsize, const int32_t *view, const double *pv,
                      double alpha, double llr_clamp, double *phat, double *lam) {
    double *sum = (double *)calloc((size_t)n, sizeof(double));
    int *cnt = (int *)calloc((size_t)n, sizeof(int));
    for (int v = 0; v < nviews; v++)
        for (int j = 0; j < vsize; j++) {
            sum[view[v * vsize + j]] += pv[v * vsize + j];
            cnt[view[v * vsize + j]] += 1;
        }
    for (int i = 0; i < n; i++) {
        double ph = cnt[i] ? alpha * (sum[i] / (double)cnt[i]) : 0.0;
        if (phat) phat[i] = ph;
        if (lam) lam[i] = clampd(log(1.0 - ph) - log(ph), llr_clamp);
    }
    free(sum); free(cnt);
}

int oracle_decode(const oracle_code *c, int type, const oracle_params *p, int shots,
                  const uint64_t *synd, int synd_words, const double *prior,
                  uint64_t *ehat, int ehat_words, double *post, double *lam_out,
                  int32_t *stats, double *margin_out, double *local_llr) {
    if (type != OR_Z && type != OR_X) return -1;
    const int N = c->order, D2 = c->delta * c->delta, n = c->n, r = c->r[type], m = c->m[type];
    const tanner *loc = &c->loc[type], *glob = &c->glob[type];
    const int *view = c->view[type];
    if (synd_words * 64 < m || (ehat && ehat_words * 64 < n)) return -1;

    bp_work wl, wg;
    work_alloc(&wl, loc->nedges);
    work_alloc(&wg, glob->nedges);
    uint8_t *s = (uint8_t *)malloc((size_t)m);
    uint8_t *sv = (uint8_t *)malloc((size_t)r);
    double *lamv = (double *)malloc(sizeof(double) * (size_t)D2);
    double *Lv = (double *)malloc(sizeof(double) * (size_t)D2);
    uint8_t *ev = (uint8_t *)malloc((size_t)D2);
    double *pall = (double *)malloc(sizeof(double) * (size_t)N * D2);
    double *lamp = (double *)malloc(sizeof(double) * (size_t)n);
    double *Lg = (double *)malloc(sizeof(double) * (size_t)n);
    uint8_t *eg = (uint8_t *)malloc((size_t)n);
    uint8_t *eo = (uint8_t *)malloc((size_t)n);

    for (int shot = 0; shot < shots; shot++) {
        const uint64_t *sw = synd + (size_t)shot * synd_words;
        const double *lam = prior + (size_t)shot * n;
        for (int i = 0; i < m; i++) s[i] = (uint8_t)get_bit(sw, i);
        double margin = INFINITY;
        wl.rng = p->perturb_seed * 0x100000001B3ull + (uint64_t)shot * 2;
        wg.rng = p->perturb_seed * 0x100000001B3ull + (uint64_t)shot * 2 + 1;

        int it_sum = 0, it_max = 0, nconv = 0, nosd = 0;

        /* Phase 1: local decoding on every vertex of the decoded side */
        for (int v = 0; v < N; v++) {
            /* local syndrome: the checks of vertex v are rows v*r .. v*r+r-1 */
            for (int rho = 0; rho < r; rho++) sv[rho] = s[v * r + rho];
            /* local priors: the channel LLRs of the qubits in Q(v) */
            for (int j = 0; j < D2; j++) lamv[j] = lam[view[v * D2 + j]];
            int conv_v = 0;
            int it_v = bp_run(loc, sv, lamv, p, p->max_iter_local, Lv, ev, &conv_v, &margin, &wl);
            it_sum += it_v;
            if (it_v > it_max) it_max = it_v;
            nconv += conv_v;
            /* local post-processing: OSD (order osd_order, costs from the
             * view's channel priors) where BP left the local syndrome
             * unsatisfied; its estimate replaces BP's decisions */
            if (p->local_osd && !conv_v && oracle_osd_ex(r, D2, c->hloc[type], sv, Lv, lamv, p->osd_order, p->osd_exact, ev) == 0) {
                conv_v = 1;
                nosd++;
            }
            /* soft output as error probabilities, then the confidence boost:
             * if H_v e_v = s_v, p_{v,j} <- max(p_{v,j}, 0.5) where e_{v,j} = 1 */
            double *pv = pall + (size_t)v * D2;
            for (int j = 0; j < D2; j++) {
                pv[j] = 1.0 / (1.0 + exp(Lv[j]));
                if (p->boost && conv_v && ev[j] && pv[j] < 0.5) pv[j] = 0.5;
            }
            if (local_llr)
                for (int j = 0; j < D2; j++)
                    local_llr[((size_t)shot * N + v) * D2 + j] = Lv[j];
        }

        /* Phase 2: p_i = alpha * Average(S_i), converted back to an LLR */
        oracle_aggregate(n, N, D2, view, pall, p->alpha, p->llr_clamp, NULL, lamp);
        if (p->perturb > 0.0)
            for (int i = 0; i < n; i++) lamp[i] = clampd(perturbed(lamp[i], p->perturb, &wl.rng), p->llr_clamp);
        if (lam_out)
            for (int i = 0; i < n; i++) lam_out[(size_t)shot * n + i] = lamp[i];

        int conv = 0, it_g = 0;
        if (p->stage == OR_STAGE_FULL) {
            /* Phase 3: global BP with the regularised prior */
            it_g = bp_run(glob, s, lamp, p, p->max_iter_global, Lg, eg, &conv, &margin, &wg);
            /* global post-processing: OSD-0 on H_t with the global posteriors
             * where global BP left the syndrome unsatisfied (when s is not
             * in the column space of H_t, BP's estimate stays) */
            if (p->global_osd && !conv && oracle_osd_ex(m, n, c->H[type], s, Lg, lamp, p->osd_order, p->osd_exact, eo) == 0) {
                memcpy(eg, eo, (size_t)n);
                conv = 2;
            }
            if (post)
                for (int i = 0; i < n; i++) post[(size_t)shot * n + i] = Lg[i];
            if (ehat) {
                uint64_t *ew = ehat + (size_t)shot * ehat_words;
                memset(ew, 0, sizeof(uint64_t) * (size_t)ehat_words);
                for (int i = 0; i < n; i++) put_bit(ew, i, eg[i]);
            }
        }
        if (stats) {
            int32_t *st = stats + (size_t)shot * 6;
            st[0] = conv; st[1] = it_g; st[2] = it_sum; st[3] = it_max; st[4] = nconv; st[5] = nosd;
        }
        if (margin_out) margin_out[shot] = margin;
    }
    free(s); free(sv); free(lamv); free(Lv); free(ev); free(pall);
    free(lamp); free(Lg); free(eg); free(eo);
    work_free(&wl); work_free(&wg);
    return 0;
}

int oracle_global_bp(const oracle_code *c, int type, const oracle_params *p, int shots,
                     const uint64_t *synd, int synd_words, const double *prior,
                     uint64_t *ehat, int ehat_words, double *post, int32_t *stats) {
    const int n = c->n, m = c->m[type];
    const tanner *glob = &c->glob[type];
    bp_work wg;
    work_alloc(&wg, glob->nedges);
    uint8_t *s = (uint8_t *)malloc((size_t)m);
    double *Lg = (double *)malloc(sizeof(double) * (size_t)n);
    uint8_t *eg = (uint8_t *)malloc((size_t)n);
    uint8_t *eo = (uint8_t *)malloc((size_t)n);
    for (int shot = 0; shot < shots; shot++) {
        const uint64_t *sw = synd + (size_t)shot * synd_words;
        for (int i = 0; i < m; i++) s[i] = (uint8_t)get_bit(sw, i);
        int conv = 0;
        int it = bp_run(glob, s, prior + (size_t)shot * n, p, p->max_iter_global, Lg, eg, &conv, NULL, &wg);
        /* BP followed by OSD-0 where BP misses the syndrome */
        if (p->global_osd && !conv &&
            oracle_osd_ex(m, n, c->H[type], s, Lg, prior + (size_t)shot * n, p->osd_order, p->osd_exact, eo) == 0) {
            memcpy(eg, eo, (size_t)n);
            conv = 2;
        }
        if (post) for (int i = 0; i < n; i++) post[(size_t)shot * n + i] = Lg[i];
        if (ehat) {
            uint64_t *ew = ehat + (size_t)shot * ehat_words;
            memset(ew, 0, sizeof(uint64_t) * (size_t)ehat_words);
            for (int i = 0; i < n; i++) put_bit(ew, i, eg[i]);
        }
        if (stats) { stats[(size_t)shot * 2] = conv; stats[(size_t)shot * 2 + 1] = it; }
    }
    free(s); free(Lg); free(eg); free(eo);
    work_free(&wg);
    return 0;
}

int oracle_logical_failure(const oracle_code *c, int type, const uint64_t *residual, int route) {
    int words = (c->n + 63) / 64;
    if (route == 0) {
        for (int l = 0; l < c->logical[type].rows; l++) {
            const uint64_t *lr = bm_row(&c->logical[type], l);
            int par = 0;
            for (int w = 0; w < words; w++) par ^= popcount64(lr[w] & residual[w]) & 1;
            if (par) return 1;
        }
        return 0;
    }
    uint64_t *v = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)words);
    memcpy(v, residual, sizeof(uint64_t) * (size_t)words);
    bm_reduce(&c->rref_other[type], c->piv_other[type], c->rank_other[type], v);
    int nz = 0;
    for (int w = 0; w < words; w++) nz |= v[w] != 0;
    free(v);
    return nz;
}
