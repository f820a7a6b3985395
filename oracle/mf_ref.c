/*
 * ORACLE (test infrastructure only; never linked into the product path).
 *
 * Plain FP64 reference for y = H x, H = sum_t c_t (1 x .. x O_a x .. x O_b x .. x 1), written as the
 * row of that Kronecker sum evaluated one target index at a time (Sec. I defines H as this sum; Sec. III
 * fixes the flattening: site 0 is the most significant mixed-radix digit).
 *
 * For a target index F with local digits n_0 .. n_{N-1}, an entry H[F, F'] of one term is nonzero only
 * where F' differs from F in the digits of the term's own sites, and there it is the product of the local
 * matrix elements O_a[n_a][n'_a] O_b[n_b][n'_b] (the identity factors contribute delta(n_l, n'_l)).  So
 *
 *     y_F = sum_t c_t sum_{n'_a} sum_{n'_b} O_a[n_a][n'_a] O_b[n_b][n'_b] x[encode(n with n_a -> n'_a,
 *                                                                                   n_b -> n'_b)]
 *
 * where encode is the mixed-radix integer of the digit vector (Sec. III, Eqs. encode and decode), which is
 * linear in the digits, so replacing n_a by n'_a moves the index by (n'_a - n_a) M_a.  The
 * local matrices are dense d x d arrays built here from their closed forms; exact zeros are skipped (an
 * entry that is zero contributes nothing), which is the only thing that keeps the cost per row small.
 *
 * Local matrices (basis index n = m + s for a spin, n = occupation for a boson):
 *   spin  : S_z = diag(m); S_+ raises m by one with the ladder element sqrt(s(s+1) - m(m+1)) of the source
 *           projection m (Sec. IV.A); S_- is its transpose; (S_z)^2, (S_+)^2, (S_-)^2 are matrix products
 *           (App. B: the zero-field-splitting channels are powers of the one-step operators);
 *   boson : n = diag(n); a^dagger |n> = sqrt(n + 1) |n + 1> (App. C); a is its transpose; n^2, a^dagger^2,
 *           a^2 are matrix products;
 *   general one-site operators (App. B local monomials): the caller's dense matrix.
 *
 * Couplings are complex; x and y are interleaved (re, im) FP64 arrays.  The code is deliberately plain:
 * every row decodes all its digits with one division and one modulo each, and every term walks the full
 * row of its local matrices.
 */
#include <complex.h>
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { KIND_SPIN = 0, KIND_BOSON = 1 };
/* operator codes of the term list (built-in local operators); codes >= OP_GENERAL are general matrices */
enum { OP_Z = 0, OP_Z2 = 1, OP_RAISE = 2, OP_LOWER = 3, OP_RAISE2 = 4, OP_LOWER2 = 5, OP_GENERAL = 16 };

#define MAXSITES 64
#define MAXD 1024

/* multipliers M_k = prod_{l > k} d_l (site 0 most significant) and D = prod_l d_l */
static int multipliers(int32_t N, const int32_t* twok, int64_t* M, int64_t* D) {
    if (N <= 0 || N > MAXSITES) return -1;
    int64_t acc = 1;
    for (int k = N - 1; k >= 0; --k) {
        if (twok[k] < 0 || twok[k] + 1 > MAXD) return -1;
        M[k] = acc;
        acc *= (int64_t)(twok[k] + 1);
    }
    *D = acc;
    return 0;
}

static void decode(int32_t N, const int32_t* twok, const int64_t* M, int64_t F, int* n) {
    for (int l = 0; l < N; ++l) n[l] = (int)((F / M[l]) % (int64_t)(twok[l] + 1));
}

static int64_t encode(int32_t N, const int64_t* M, const int* n) {
    int64_t F = 0;
    for (int l = 0; l < N; ++l) F += (int64_t)n[l] * M[l];
    return F;
}

/* C = A B for d x d row-major matrices */
static void matmul(int d, const double* A, const double* B, double* C) {
    for (int i = 0; i < d; ++i)
        for (int j = 0; j < d; ++j) {
            double s = 0.0;
            for (int k = 0; k < d; ++k) s += A[i * d + k] * B[k * d + j];
            C[i * d + j] = s;
        }
}

/* dense local matrix of built-in operator op on a site of the given kind and local dimension d */
static int builtin_matrix(int kind, int twok, int op, double* out) {
    const int d = twok + 1;
    double* z = calloc((size_t)d * d, sizeof(double));
    double* up = calloc((size_t)d * d, sizeof(double));
    double* dn = calloc((size_t)d * d, sizeof(double));
    if (!z || !up || !dn) {
        free(z), free(up), free(dn);
        return -1;
    }
    for (int n = 0; n < d; ++n) {
        if (kind == KIND_SPIN) {
            const double s = 0.5 * twok, m = n - s;
            z[n * d + n] = m;
            if (n + 1 < d) up[(n + 1) * d + n] = sqrt(s * (s + 1.0) - m * (m + 1.0));
        } else {
            z[n * d + n] = n;
            if (n + 1 < d) up[(n + 1) * d + n] = sqrt(n + 1.0);
        }
    }
    for (int i = 0; i < d; ++i)
        for (int j = 0; j < d; ++j) dn[i * d + j] = up[j * d + i];
    int rc = 0;
    switch (op) {
        case OP_Z: memcpy(out, z, sizeof(double) * d * d); break;
        case OP_Z2: matmul(d, z, z, out); break;
        case OP_RAISE: memcpy(out, up, sizeof(double) * d * d); break;
        case OP_LOWER: memcpy(out, dn, sizeof(double) * d * d); break;
        case OP_RAISE2: matmul(d, up, up, out); break;
        case OP_LOWER2: matmul(d, dn, dn, out); break;
        default: rc = -1;
    }
    free(z), free(up), free(dn);
    return rc;
}

/* the local matrix of operator op on site s: built-in, or general matrix g = op - OP_GENERAL, whose d x d
 * entries sit at gen_mat + gen_off[g] */
static int local_matrix(const int32_t* kind, const int32_t* twok, int s, int op, int32_t n_gen,
                        const int64_t* gen_off, const double* gen_mat, double* out) {
    const int d = twok[s] + 1;
    if (op >= OP_GENERAL) {
        const int g = op - OP_GENERAL;
        if (g >= n_gen) return -1;
        memcpy(out, gen_mat + gen_off[g], sizeof(double) * d * d);
        return 0;
    }
    return builtin_matrix(kind[s], twok[s], op, out);
}

/*
 * y = H x over all rows (rows == NULL, nrows == D) or over the target indices rows[0 .. nrows-1].
 * term    : [n_terms][4] = (site_a, op_a, site_b, op_b); site_b = -1 for a one-site term
 * coef    : [n_terms][2] complex coefficient c_t (theta of the term's parameter times its weight)
 * gen_off : [n_gen] offsets into gen_mat of the general operators' dense matrices (row-major, d x d of the
 *           site the operator is used on)
 */
int mf_ref_apply(int32_t N, const int32_t* kind, const int32_t* twok, int32_t n_terms, const int32_t* term,
                 const double* coef, int32_t n_gen, const int64_t* gen_off, const double* gen_mat, int64_t D,
                 const double* x, double* y, int64_t nrows, const int64_t* rows) {
    int64_t M[MAXSITES], Dchk;
    if (multipliers(N, twok, M, &Dchk) != 0 || Dchk != D) return -1;
    if (rows == NULL && nrows != D) return -1;
    /* one dense matrix per term side, built once */
    int64_t* moff = malloc(sizeof(int64_t) * (2 * (size_t)n_terms + 1));
    size_t total = 0;
    for (int t = 0; t < n_terms; ++t) {
        const int32_t* tt = term + 4 * t;
        if (tt[0] < 0 || tt[0] >= N || tt[2] >= N || tt[2] == tt[0]) {
            free(moff);
            return -1;
        }
        moff[2 * t] = (int64_t)total;
        total += (size_t)(twok[tt[0]] + 1) * (twok[tt[0]] + 1);
        moff[2 * t + 1] = (int64_t)total;
        if (tt[2] >= 0) total += (size_t)(twok[tt[2]] + 1) * (twok[tt[2]] + 1);
    }
    double* mats = calloc(total + 1, sizeof(double));
    int rc = 0;
    for (int t = 0; t < n_terms && rc == 0; ++t) {
        const int32_t* tt = term + 4 * t;
        rc |= local_matrix(kind, twok, tt[0], tt[1], n_gen, gen_off, gen_mat, mats + moff[2 * t]);
        if (tt[2] >= 0) rc |= local_matrix(kind, twok, tt[2], tt[3], n_gen, gen_off, gen_mat, mats + moff[2 * t + 1]);
    }
    if (rc != 0) {
        free(mats), free(moff);
        return -1;
    }
    const double complex* xc = (const double complex*)x;
    const double complex* cc = (const double complex*)coef;
    double complex* yc = (double complex*)y;

#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < nrows; ++r) {
        const int64_t F = rows ? rows[r] : r;
        int n[MAXSITES];
        decode(N, twok, M, F, n);
        double complex acc = 0.0;
        for (int t = 0; t < n_terms; ++t) {
            const int32_t* tt = term + 4 * t;
            const int a = tt[0], b = tt[2];
            const int da = twok[a] + 1;
            const double* Oa = mats + moff[2 * t];
            double complex part = 0.0;
            for (int na = 0; na < da; ++na) {
                const double ea = Oa[n[a] * da + na];
                if (ea == 0.0) continue;
                /* the encode is linear in the digits: replacing n_a by na moves the index by (na - n_a) M_a */
                const int64_t Fa = F + (int64_t)(na - n[a]) * M[a];
                if (b < 0) {
                    part += ea * xc[Fa];
                    continue;
                }
                const int db = twok[b] + 1;
                const double* Ob = mats + moff[2 * t + 1];
                for (int nb = 0; nb < db; ++nb) {
                    const double eb = Ob[n[b] * db + nb];
                    if (eb == 0.0) continue;
                    part += ea * eb * xc[Fa + (int64_t)(nb - n[b]) * M[b]];
                }
            }
            acc += cc[t] * part;
        }
        yc[r] = acc;
    }
    free(mats), free(moff);
    return 0;
}

/*
 * Source index of every term for the target rows F0 .. F0+count-1: the index whose digits equal the
 * target's except n_a - q_a on site a (and n_b - q_b on site b), re-encoded (Sec. III), or -1 when such a
 * digit falls outside 0 .. d - 1.
 * terms : [n_terms][4] = (site_a, q_a, site_b, q_b), q the operator's digit shift; site_b = -1 for a
 *         one-site term.
 */
int mf_ref_sources(int32_t N, const int32_t* twok, int32_t n_terms, const int32_t* terms, int64_t F0,
                   int64_t count, int64_t* out) {
    int64_t M[MAXSITES], D;
    if (multipliers(N, twok, M, &D) != 0) return -1;
    if (F0 < 0 || count < 0 || F0 + count > D) return -1;
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < count; ++r) {
        int n[MAXSITES];
        decode(N, twok, M, F0 + r, n);
        for (int t = 0; t < n_terms; ++t) {
            const int32_t* tt = terms + 4 * t;
            int src[MAXSITES];
            memcpy(src, n, sizeof(int) * N);
            int ok = 1;
            src[tt[0]] -= tt[1];
            ok &= src[tt[0]] >= 0 && src[tt[0]] <= twok[tt[0]];
            if (tt[2] >= 0) {
                src[tt[2]] -= tt[3];
                ok &= src[tt[2]] >= 0 && src[tt[2]] <= twok[tt[2]];
            }
            out[r * n_terms + t] = ok ? encode(N, M, src) : -1;
        }
    }
    return 0;
}

/* Threads the row loops use: n > 0 sets them (omp_set_num_threads); returns the current count. */
int mf_ref_threads(int32_t n) {
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
}
