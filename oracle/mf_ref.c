/*
 * ORACLE (test infrastructure only; never linked into the product path).
 *
 * Plain FP64 reference for the target-driven matrix-free map y = H x of
 * "Spin Hamiltonian as Matrix-Free Linear Map": for every target index F the
 * digits are decoded with the mixed-radix rule (Sec. III, Eq. decode), the
 * one-site terms are applied with the ladder rules of Sec. IV.A and the pair
 * terms with the shift/offset rules of Sec. IV.B (Eqs. src_digit_two_site and
 * sourceoffset), in the order of the pseudocode of App. A: diagonal, S_+ and
 * S_- per site, then every pair and every (alpha, beta) channel.
 *
 * Extensions, each from the paper's own text:
 *   - a one-site (S_z)^2 coupling (the diagonal channel of the zero-field
 *     splitting, App. B), applied right after the h_z term of the same site;
 *   - truncated boson digits (App. C): the local digit is the occupation n,
 *     "z" is the number operator, "+" is a^dagger and "-" is a, with the
 *     square-root factors evaluated on the source occupation;
 *   - one-site (S_+)^2 and (S_-)^2 couplings (the q = +-2 channels of App. B,
 *     Eq. generic_local_shift, as in the zero-field-splitting E term): source
 *     digit n -+ 2, coefficient the product of the two one-step ladder elements
 *     taken on the reconstructed source projection.
 *
 * Couplings are complex; x and y are interleaved (re, im) FP64 arrays.
 * The code is deliberately plain: one division and one modulo per digit,
 * the ladder element recomputed from its closed form for every use.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

enum { KIND_SPIN = 0, KIND_BOSON = 1 };
enum { AL_Z = 0, AL_P = 1, AL_M = 2, AL_PP = 3, AL_MM = 4 }; /* alpha in {z, +, -}; ++, -- one-site only */

#define MAXSITES 64

/* delta(z) = 0, delta(+) = +1, delta(-) = -1 (App. A); q = +-2 for (S_+-)^2 (App. B) */
static int delta_of(int alpha) {
    switch (alpha) {
        case AL_Z: return 0;
        case AL_P: return 1;
        case AL_M: return -1;
        case AL_PP: return 2;
        default: return -2;
    }
}

/* projection of a local digit: m = n - s for a spin (notation guide), n for a boson */
static double proj(int kind, int twok, int n) {
    return kind == KIND_SPIN ? (double)n - 0.5 * (double)twok : (double)n;
}

/* Lambda(alpha; s, m) of App. A evaluated on the source projection m (spin),
 * and its boson counterpart on the source occupation (App. C). */
static double lambda_local(int kind, int twok, int alpha, double m) {
    if (alpha == AL_Z) return m;
    if (kind == KIND_SPIN) {
        double s = 0.5 * (double)twok;
        if (alpha == AL_P) return sqrt(s * (s + 1.0) - m * (m + 1.0));
        return sqrt(s * (s + 1.0) - m * (m - 1.0));
    }
    if (alpha == AL_P) return sqrt(m + 1.0); /* a^dagger |n> = sqrt(n+1) |n+1> */
    return sqrt(m);                           /* a |n> = sqrt(n) |n-1>          */
}

static int multipliers(int32_t N, const int32_t* twok, int64_t* M, int64_t* D) {
    if (N <= 0 || N > MAXSITES) return -1;
    /* M_k = prod_{l > k} d_l, M_{N-1} = 1  (Sec. III) */
    int64_t acc = 1;
    for (int k = N - 1; k >= 0; --k) {
        M[k] = acc;
        acc *= (int64_t)(twok[k] + 1);
    }
    *D = acc;
    return 0;
}

/*
 * onsite : [N][6] complex couplings (h_z, h_zz, h_+, h_-, h_++, h_--) as interleaved doubles, i.e.
 *          [N][6][2]; h_++ multiplies (S_+)^2 (or a^dagger^2), h_-- multiplies (S_-)^2 (or a^2)
 * pair_i, pair_j : the P active pairs
 * J      : [P][3][3] complex couplings J^{alpha beta}, alpha, beta in (z, +, -), i.e. [P][3][3][2]
 * x      : [D] complex input;  y : [nrows] complex output
 * rows   : NULL for all rows 0..D-1 (then nrows must equal D), else the target indices to evaluate
 */
int mf_ref_matvec(int32_t N, const int32_t* kind, const int32_t* twok, const double* onsite,
                  int32_t P, const int32_t* pair_i, const int32_t* pair_j, const double* J,
                  int64_t D, const double* x, double* y, int64_t nrows, const int64_t* rows) {
    int64_t M[MAXSITES], Dchk;
    if (multipliers(N, twok, M, &Dchk) != 0 || Dchk != D) return -1;
    if (rows == NULL && nrows != D) return -1;
    const double complex* xc = (const double complex*)x;
    double complex* yc = (double complex*)y;
    const double complex* h = (const double complex*)onsite;
    const double complex* Jc = (const double complex*)J;

#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < nrows; ++r) {
        int64_t F = rows ? rows[r] : r;
        int n[MAXSITES];
        for (int i = 0; i < N; ++i) n[i] = (int)((F / M[i]) % (int64_t)(twok[i] + 1));
        double complex acc = 0.0;

        for (int i = 0; i < N; ++i) {
            int d = twok[i] + 1;
            double m = proj(kind[i], twok[i], n[i]);
            acc += h[6 * i + 0] * m * xc[F];
            acc += h[6 * i + 1] * (m * m) * xc[F];
            if (n[i] > 0) {
                int64_t src = F - M[i];
                double ms = proj(kind[i], twok[i], n[i] - 1);
                acc += h[6 * i + 2] * lambda_local(kind[i], twok[i], AL_P, ms) * xc[src];
            }
            if (n[i] < d - 1) {
                int64_t src = F + M[i];
                double ms = proj(kind[i], twok[i], n[i] + 1);
                acc += h[6 * i + 3] * lambda_local(kind[i], twok[i], AL_M, ms) * xc[src];
            }
            if (n[i] >= 2) { /* (S_+)^2: source digit n - 2, coefficient C_+^(2) on the source m */
                int64_t src = F - 2 * M[i];
                double ms = proj(kind[i], twok[i], n[i] - 2);
                double c2 = lambda_local(kind[i], twok[i], AL_P, ms + 1.0) * lambda_local(kind[i], twok[i], AL_P, ms);
                acc += h[6 * i + 4] * c2 * xc[src];
            }
            if (n[i] <= d - 3) { /* (S_-)^2: source digit n + 2, coefficient C_-^(2) on the source m */
                int64_t src = F + 2 * M[i];
                double ms = proj(kind[i], twok[i], n[i] + 2);
                double c2 = lambda_local(kind[i], twok[i], AL_M, ms - 1.0) * lambda_local(kind[i], twok[i], AL_M, ms);
                acc += h[6 * i + 5] * c2 * xc[src];
            }
        }

        for (int p = 0; p < P; ++p) {
            int i = pair_i[p], j = pair_j[p];
            for (int a = 0; a < 3; ++a) {
                for (int b = 0; b < 3; ++b) {
                    int nsi = n[i] - delta_of(a);
                    int nsj = n[j] - delta_of(b);
                    if (nsi < 0 || nsi > twok[i] || nsj < 0 || nsj > twok[j]) continue;
                    int64_t src = F - (int64_t)delta_of(a) * M[i] - (int64_t)delta_of(b) * M[j];
                    double msi = proj(kind[i], twok[i], nsi);
                    double msj = proj(kind[j], twok[j], nsj);
                    acc += Jc[9 * p + 3 * a + b] * lambda_local(kind[i], twok[i], a, msi) *
                           lambda_local(kind[j], twok[j], b, msj) * xc[src];
                }
            }
        }
        yc[r] = acc;
    }
    return 0;
}

/*
 * General one-site bands (App. B: any local monomial (S_+)^p (S_z)^r (S_-)^l is one band of the local
 * matrix): term t couples site a with shift qa and table ta (ta[n] = <n|O_a|n - qa> at target digit n) and,
 * when b >= 0, site b with qb and tb.  Adds to y (rows as in mf_ref_matvec):
 *   y_F += c_t ta[n_a] tb[n_b] x[F - qa M_a - qb M_b]   when n_a - qa and n_b - qb are digits.
 * gterm : [n_gen][4] = (a, qa, b, qb);  toff : [n_gen][2] offsets of ta, tb in tab;  c : [n_gen][2] complex.
 */
int mf_ref_general_add(int32_t N, const int32_t* twok, int32_t n_gen, const int32_t* gterm,
                       const int64_t* toff, const double* tab, const double* c, int64_t D, const double* x,
                       double* y, int64_t nrows, const int64_t* rows) {
    int64_t M[MAXSITES], Dm;
    if (multipliers(N, twok, M, &Dm) != 0 || Dm != D) return -1;
    const double complex* xc = (const double complex*)x;
    double complex* yc = (double complex*)y;
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < nrows; ++r) {
        int64_t F = rows ? rows[r] : r;
        double complex acc = 0.0;
        for (int t = 0; t < n_gen; ++t) {
            const int32_t* g = gterm + 4 * t;
            int a = g[0], qa = g[1], b = g[2], qb = g[3];
            int na = (int)((F / M[a]) % (int64_t)(twok[a] + 1));
            if (na - qa < 0 || na - qa > twok[a]) continue;
            double f = tab[toff[2 * t] + na];
            int64_t src = F - (int64_t)qa * M[a];
            if (b >= 0) {
                int nb = (int)((F / M[b]) % (int64_t)(twok[b] + 1));
                if (nb - qb < 0 || nb - qb > twok[b]) continue;
                f *= tab[toff[2 * t + 1] + nb];
                src -= (int64_t)qb * M[b];
            }
            acc += (c[2 * t] + I * c[2 * t + 1]) * f * xc[src];
        }
        yc[r] += acc;
    }
    return 0;
}

/*
 * Source index of every term for the target rows F0 .. F0+count-1 (Eq. sourceoffset, with the
 * admissibility test on the source digits): out[r][t] = I, or -1 when the term cannot reach F.
 * terms : [n_terms][4] = (site_a, alpha_a, site_b, alpha_b), alpha in (z, +, -, ++, --) = (0..4);
 *         site_b = -1 for one-site terms.
 */
int mf_ref_sources(int32_t N, const int32_t* twok, int32_t n_terms, const int32_t* terms,
                   int64_t F0, int64_t count, int64_t* out) {
    int64_t M[MAXSITES], D;
    if (multipliers(N, twok, M, &D) != 0) return -1;
    if (F0 < 0 || F0 + count > D) return -1;
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < count; ++r) {
        int64_t F = F0 + r;
        for (int t = 0; t < n_terms; ++t) {
            const int32_t* tt = terms + 4 * t;
            int i = tt[0], j = tt[2];
            int ni = (int)((F / M[i]) % (int64_t)(twok[i] + 1));
            int nsi = ni - delta_of(tt[1]);
            int64_t src = F - (int64_t)delta_of(tt[1]) * M[i];
            int ok = (nsi >= 0 && nsi <= twok[i]);
            if (j >= 0) {
                int nj = (int)((F / M[j]) % (int64_t)(twok[j] + 1));
                int nsj = nj - delta_of(tt[3]);
                src -= (int64_t)delta_of(tt[3]) * M[j];
                ok = ok && (nsj >= 0 && nsj <= twok[j]);
            }
            out[r * n_terms + t] = ok ? src : -1;
        }
    }
    return 0;
}
