/*
 * Plain FP64 CPU oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the tests, the smoke check and the benchmark's CPU-baseline leg load this
 * library.  It shares no code, header, table or helper with the GPU library and
 * must never be reached from the product path.
 *
 * Everything is the textbook definition written out as loops: one multiply and
 * one add per step (built with -ffp-contract=off, so no fused multiply-add),
 * round-to-nearest-even, summation index ascending.  OpenMP is used only over
 * independent output columns / instances; it does not change any sum.
 *
 * What the operations are:
 *  - LTimes / LPlusTimes: the discrete-ordinates moment operators of the Kripke
 *    proxy application (ClangJIT paper, section 5.2, Kripke case study and its
 *    footnote naming LTimes and LPlusTimes).  The paper does not write the
 *    contraction down; the standard operator is
 *        phi[nm,g,z]  = sum_d  L[nm,d]  * psi[d,g,z]
 *        psi'[d,g,z]  = sum_nm L+[d,nm] * phi[nm,g,z]
 *    over the six nestings DGZ, DZG, GDZ, GZD, ZDG, ZGD that the paper lists in
 *    its Kripke layout-dispatch listing (section 5.2).  A nesting name gives the
 *    storage order of the three axes, rightmost fastest; phi uses the same order
 *    with D replaced by NM; L is row-major [NM][D], L+ row-major [D][NM].
 *  - Scattering (a reading: the paper names Kripke's scattering kernel among
 *    the de-multiversioned ones, section 5.2 footnote, but does not define it):
 *    the standard within-group-to-group scattering source of discrete-ordinates
 *    transport,
 *        phi_out[nm,g,z] = sum_g' S[mat(z)][n(nm)][g][g'] * phi[nm,g',z]
 *    where n(nm) = floor(sqrt(nm)) is the Legendre degree of moment nm (moments
 *    ordered by degree, nm = n^2 + n + m), mat(z) the zone's material, and S
 *    row-major [nmat][n_max + 1][G][G] (row g receives from column g').  phi
 *    and phi_out use the moment arrays' storage order.
 *  - Tensor-product mass operator (a reading: the paper specializes Laghos'
 *    partial-assembly kernels on the numbers of dofs and quadrature points,
 *    section 5.3, without writing the operator down): per element e,
 *        y_e[i] = sum_q B(q,i) D_e[q] sum_j B(q,j) x_e[j],
 *        B(q,i) = prod_k B1[q_k][i_k]
 *    over multi-indices i, j (D1D^dim dofs) and q (Q1D^dim points), with B1 the
 *    row-major [Q1D][D1D] one-dimensional basis at the points and the first
 *    index component fastest in x_e, y_e and D_e.
 *  - Batched small products: C_i = A_i * B_i, square, row-major, as in the
 *    paper's RAJA small matrix-multiply benchmark (section 5.1), one product per
 *    instance of a packed batch.
 *  - BF16 split emulation: hi = RNE_bf16(x), lo = RNE_bf16(x - hi) (split
 *    products after Henry, Tang & Heinecke, ARITH 2019), evaluated in FP64.
 *  - Cost-model MLP: in -> H -> H -> 1 with ReLU, mean-squared-error loss,
 *    backpropagation, and the Adam update (Kingma & Ba, ICLR 2015).  This is the
 *    adaptive, profile-guided specialization of the paper's future work
 *    (section 6) realized as a learned picker.
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { ORC_DGZ = 0, ORC_DZG = 1, ORC_GDZ = 2, ORC_GZD = 3, ORC_ZDG = 4, ORC_ZGD = 5 };

/* Offset of logical element (a, g, z) of an (A, G, Z) array stored in `layout`
 * order (rightmost axis fastest).  Returns (size_t)-1 for an unknown layout. */
static size_t orc_index(int layout, size_t a, size_t g, size_t z, size_t A, size_t G, size_t Z)
{
    switch (layout) {
    case ORC_DGZ: return (a * G + g) * Z + z;
    case ORC_DZG: return (a * Z + z) * G + g;
    case ORC_GDZ: return (g * A + a) * Z + z;
    case ORC_GZD: return (g * Z + z) * A + a;
    case ORC_ZDG: return (z * A + a) * G + g;
    case ORC_ZGD: return (z * G + g) * A + a;
    default: return (size_t)-1;
    }
}

int orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}

/* phi[nm,g,z] = sum_{d ascending} L[nm*D + d] * psi[d,g,z]; overwrites phi.
 * Returns 0, or -1 for an unknown layout. */
int orc_ltimes(int layout, int64_t Z, int64_t G, int64_t D, int64_t NM,
               const double *L, const double *psi, double *phi)
{
    if (layout < 0 || layout > 5) return -1;
    int64_t ncol = G * Z;
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < ncol; ++c) {
        size_t g = (size_t)(c / Z), z = (size_t)(c % Z);
        for (int64_t nm = 0; nm < NM; ++nm) {
            double acc = 0.0;
            for (int64_t d = 0; d < D; ++d) {
                double prod = L[nm * D + d] * psi[orc_index(layout, (size_t)d, g, z, (size_t)D, (size_t)G, (size_t)Z)];
                acc = acc + prod;
            }
            phi[orc_index(layout, (size_t)nm, g, z, (size_t)NM, (size_t)G, (size_t)Z)] = acc;
        }
    }
    return 0;
}

/* psi'[d,g,z] = sum_{nm ascending} Lplus[d*NM + nm] * phi[nm,g,z]; overwrites psi'. */
int orc_lplustimes(int layout, int64_t Z, int64_t G, int64_t D, int64_t NM,
                   const double *Lplus, const double *phi, double *psi_out)
{
    if (layout < 0 || layout > 5) return -1;
    int64_t ncol = G * Z;
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < ncol; ++c) {
        size_t g = (size_t)(c / Z), z = (size_t)(c % Z);
        for (int64_t d = 0; d < D; ++d) {
            double acc = 0.0;
            for (int64_t nm = 0; nm < NM; ++nm) {
                double prod = Lplus[d * NM + nm] * phi[orc_index(layout, (size_t)nm, g, z, (size_t)NM, (size_t)G, (size_t)Z)];
                acc = acc + prod;
            }
            psi_out[orc_index(layout, (size_t)d, g, z, (size_t)D, (size_t)G, (size_t)Z)] = acc;
        }
    }
    return 0;
}

/* sum_d |L[nm,d]| * |psi[d,g,z]|: the scale of the componentwise error bound
 * of one LTimes output.  Same shapes and layout rules as orc_ltimes. */
int orc_ltimes_absscale(int layout, int64_t Z, int64_t G, int64_t D, int64_t NM,
                        const double *L, const double *psi, double *scale)
{
    if (layout < 0 || layout > 5) return -1;
    int64_t ncol = G * Z;
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < ncol; ++c) {
        size_t g = (size_t)(c / Z), z = (size_t)(c % Z);
        for (int64_t nm = 0; nm < NM; ++nm) {
            double acc = 0.0;
            for (int64_t d = 0; d < D; ++d)
                acc = acc + fabs(L[nm * D + d]) * fabs(psi[orc_index(layout, (size_t)d, g, z, (size_t)D, (size_t)G, (size_t)Z)]);
            scale[orc_index(layout, (size_t)nm, g, z, (size_t)NM, (size_t)G, (size_t)Z)] = acc;
        }
    }
    return 0;
}

/* Legendre degree of moment nm: the largest n with n*n <= nm. */
static int64_t orc_degree(int64_t nm)
{
    int64_t n = 0;
    while ((n + 1) * (n + 1) <= nm) ++n;
    return n;
}

/* phi_out[nm,g,z] = sum_{g' ascending} S[mat[z]][n(nm)][g][g'] * phi[nm,g',z];
 * overwrites phi_out.  Returns 0, -1 for an unknown layout, -2 for a material
 * index outside [0, nmat).  With `absolute` set it forms the error scale
 * sum_g' |S[..][g][g']| |phi[nm,g',z]| instead. */
static int orc_scatter_impl(int layout, int64_t Z, int64_t G, int64_t NM, int64_t nmat, const double *S,
                            const int32_t *mat, const double *phi, double *out, int absolute)
{
    if (layout < 0 || layout > 5) return -1;
    for (int64_t z = 0; z < Z; ++z)
        if (mat[z] < 0 || mat[z] >= nmat) return -2;
    const int64_t nl = orc_degree(NM - 1) + 1;
    int64_t ncol = NM * Z;
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < ncol; ++c) {
        int64_t nm = c / Z, z = c % Z;
        const double *Sm = S + ((int64_t)mat[z] * nl + orc_degree(nm)) * G * G;
        for (int64_t g = 0; g < G; ++g) {
            double acc = 0.0;
            for (int64_t gp = 0; gp < G; ++gp) {
                double x = phi[orc_index(layout, (size_t)nm, (size_t)gp, (size_t)z, (size_t)NM, (size_t)G, (size_t)Z)];
                double prod = absolute ? fabs(Sm[g * G + gp]) * fabs(x) : Sm[g * G + gp] * x;
                acc = acc + prod;
            }
            out[orc_index(layout, (size_t)nm, (size_t)g, (size_t)z, (size_t)NM, (size_t)G, (size_t)Z)] = acc;
        }
    }
    return 0;
}

int orc_scattering(int layout, int64_t Z, int64_t G, int64_t NM, int64_t nmat, const double *S,
                   const int32_t *mat, const double *phi, double *phi_out)
{
    return orc_scatter_impl(layout, Z, G, NM, nmat, S, mat, phi, phi_out, 0);
}

int orc_scattering_absscale(int layout, int64_t Z, int64_t G, int64_t NM, int64_t nmat, const double *S,
                            const int32_t *mat, const double *phi, double *scale)
{
    return orc_scatter_impl(layout, Z, G, NM, nmat, S, mat, phi, scale, 1);
}

/* prod_k B1[q_k][i_k] for flat indices q (base Q1D) and i (base D1D), first component fastest;
 * with `absolute` the product of magnitudes. */
static double orc_basis(const double *B1, int64_t dim, int64_t D1D, int64_t Q1D, int64_t q, int64_t i, int absolute)
{
    double b = 1.0;
    for (int64_t k = 0; k < dim; ++k) {
        double v = B1[(q % Q1D) * D1D + (i % D1D)];
        b = b * (absolute ? fabs(v) : v);
        q /= Q1D;
        i /= D1D;
    }
    return b;
}

/* y_e = B^T diag(D_e) B x_e for e < NE (the definition above, sums ascending); with
 * `absolute` every factor by its magnitude (the componentwise error scale). */
static int orc_mass_impl(int64_t dim, int64_t D1D, int64_t Q1D, int64_t NE, const double *B1, const double *Dq,
                         const double *X, double *Y, int absolute)
{
    if (dim < 1 || dim > 3 || D1D < 1 || Q1D < 1) return -1;
    int64_t nd = 1, nq = 1;
    for (int64_t k = 0; k < dim; ++k) { nd *= D1D; nq *= Q1D; }
    int failed = 0;
#pragma omp parallel for schedule(static) reduction(|| : failed)
    for (int64_t e = 0; e < NE; ++e) {
        const double *x = X + e * nd;
        const double *dq = Dq + e * nq;
        double *y = Y + e * nd;
        double *u = (double *)malloc((size_t)nq * sizeof(double));   /* B x_e scaled by D_e, one value per point */
        if (!u) { failed = 1; continue; }
        for (int64_t q = 0; q < nq; ++q) {
            double acc = 0.0;
            for (int64_t j = 0; j < nd; ++j) acc = acc + orc_basis(B1, dim, D1D, Q1D, q, j, absolute) * (absolute ? fabs(x[j]) : x[j]);
            u[q] = acc * (absolute ? fabs(dq[q]) : dq[q]);
        }
        for (int64_t i = 0; i < nd; ++i) {
            double acc = 0.0;
            for (int64_t q = 0; q < nq; ++q) acc = acc + orc_basis(B1, dim, D1D, Q1D, q, i, absolute) * u[q];
            y[i] = acc;
        }
        free(u);
    }
    return failed ? -2 : 0;
}

int orc_mass(int64_t dim, int64_t D1D, int64_t Q1D, int64_t NE, const double *B1, const double *Dq, const double *X,
             double *Y)
{
    return orc_mass_impl(dim, D1D, Q1D, NE, B1, Dq, X, Y, 0);
}

int orc_mass_absscale(int64_t dim, int64_t D1D, int64_t Q1D, int64_t NE, const double *B1, const double *Dq,
                      const double *X, double *Y)
{
    return orc_mass_impl(dim, D1D, Q1D, NE, B1, Dq, X, Y, 1);
}

/* C_i = A_i * B_i for i < count; instance i is n[i] x n[i], row-major, stored at
 * element offset off[i] of each packed array.  k ascending. */
int orc_bgemm(int64_t count, const int32_t *n, const int64_t *off,
              const double *A, const double *B, double *C)
{
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < count; ++i) {
        int64_t s = n[i];
        const double *a = A + off[i];
        const double *b = B + off[i];
        double *c = C + off[i];
        for (int64_t r = 0; r < s; ++r)
            for (int64_t col = 0; col < s; ++col) {
                double acc = 0.0;
                for (int64_t k = 0; k < s; ++k) {
                    double prod = a[r * s + k] * b[k * s + col];
                    acc = acc + prod;
                }
                c[r * s + col] = acc;
            }
    }
    return 0;
}

/* ---------------------------------------------------------------- BF16 split */

/* Nearest bfloat16 value of x (8 significant bits), ties to even, computed from
 * the definition: x = m * 2^e with 0.5 <= |m| < 1; keep m rounded to 8 bits.
 * Valid for normal bf16 results (|x| >= 2^-126), which covers every input the
 * tests use; 0, inf and nan pass through. */
double orc_bf16_round(double x)
{
    if (x == 0.0 || isnan(x) || isinf(x)) return x;
    int e;
    double m = frexp(x, &e);            /* x = m * 2^e, 0.5 <= |m| < 1 */
    double scaled = m * 256.0;          /* exact */
    double r = nearbyint(scaled);       /* default rounding mode: ties to even */
    return ldexp(r, e - 8);
}

/* FP64 emulation of the split-BF16 LTimes.  mode 0: sum hiL*hiPsi;
 * mode 1 (compensated): sum (hiL*hiPsi + hiL*loPsi + loL*hiPsi).  Every product
 * of two bf16 values and every sum is formed in FP64, so this is the value the
 * split scheme aims at, without FP32 accumulation error. */
int orc_ltimes_bf16_emul(int mode, int layout, int64_t Z, int64_t G, int64_t D, int64_t NM,
                         const double *L, const double *psi, double *phi)
{
    if (layout < 0 || layout > 5 || mode < 0 || mode > 1) return -1;
    int64_t ncol = G * Z;
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < ncol; ++c) {
        size_t g = (size_t)(c / Z), z = (size_t)(c % Z);
        for (int64_t nm = 0; nm < NM; ++nm) {
            double acc = 0.0;
            for (int64_t d = 0; d < D; ++d) {
                double l = L[nm * D + d];
                double p = psi[orc_index(layout, (size_t)d, g, z, (size_t)D, (size_t)G, (size_t)Z)];
                double lh = orc_bf16_round(l), ll = orc_bf16_round(l - lh);
                double ph = orc_bf16_round(p), pl = orc_bf16_round(p - ph);
                double term = lh * ph;
                if (mode == 1) term = term + lh * pl + ll * ph;
                acc = acc + term;
            }
            phi[orc_index(layout, (size_t)nm, g, z, (size_t)NM, (size_t)G, (size_t)Z)] = acc;
        }
    }
    return 0;
}

/* ------------------------------------------------------------------ MLP model */
/*
 * Parameter vector theta (FP64), packed in this order:
 *   W1[H][F], b1[H], W2[H][H], b2[H], w3[H], b3[1]      (total H*F + H*H + 3H + 1)
 * Forward for one row x (F features):
 *   z1 = W1 x + b1, h1 = max(z1, 0); z2 = W2 h1 + b2, h2 = max(z2, 0); y = w3 . h2 + b3
 * Loss over a batch of R rows with targets t: (1/R) sum_r (y_r - t_r)^2.
 * ReLU'(z) is taken as 1 for z > 0 and 0 otherwise.
 */
int64_t orc_mlp_nparams(int64_t F, int64_t H) { return H * F + H * H + 3 * H + 1; }

static void orc_mlp_row(int64_t F, int64_t H, const double *th, const double *x,
                        double *z1, double *h1, double *z2, double *h2, double *y)
{
    const double *W1 = th, *b1 = W1 + H * F, *W2 = b1 + H, *b2 = W2 + H * H, *w3 = b2 + H, *b3 = w3 + H;
    for (int64_t j = 0; j < H; ++j) {
        double acc = 0.0;
        for (int64_t k = 0; k < F; ++k) acc = acc + W1[j * F + k] * x[k];
        z1[j] = acc + b1[j];
        h1[j] = z1[j] > 0.0 ? z1[j] : 0.0;
    }
    for (int64_t j = 0; j < H; ++j) {
        double acc = 0.0;
        for (int64_t k = 0; k < H; ++k) acc = acc + W2[j * H + k] * h1[k];
        z2[j] = acc + b2[j];
        h2[j] = z2[j] > 0.0 ? z2[j] : 0.0;
    }
    double acc = 0.0;
    for (int64_t k = 0; k < H; ++k) acc = acc + w3[k] * h2[k];
    *y = acc + b3[0];
}

/* y[r] for R rows of X (row-major R x F).  H <= 1024. */
int orc_mlp_forward(int64_t R, int64_t F, int64_t H, const double *theta, const double *X, double *y)
{
    if (H > 1024) return -1;
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < R; ++r) {
        double z1[1024], h1[1024], z2[1024], h2[1024];
        orc_mlp_row(F, H, theta, X + r * F, z1, h1, z2, h2, &y[r]);
    }
    return 0;
}

/* Loss and its gradient with respect to theta (same packing), by backprop.
 * Serial over rows, so the gradient sum is in ascending row order. */
double orc_mlp_loss_grad(int64_t R, int64_t F, int64_t H, const double *theta,
                         const double *X, const double *t, double *grad)
{
    if (H > 1024) return NAN;
    int64_t P = orc_mlp_nparams(F, H);
    for (int64_t p = 0; p < P; ++p) grad[p] = 0.0;
    const double *W2 = theta + H * F + H, *w3 = W2 + H * H + H;
    double *gW1 = grad, *gb1 = gW1 + H * F, *gW2 = gb1 + H, *gb2 = gW2 + H * H, *gw3 = gb2 + H, *gb3 = gw3 + H;
    double z1[1024], h1[1024], z2[1024], h2[1024], dz2[1024], dz1[1024];
    double loss = 0.0;
    for (int64_t r = 0; r < R; ++r) {
        const double *x = X + r * F;
        double y;
        orc_mlp_row(F, H, theta, x, z1, h1, z2, h2, &y);
        double e = y - t[r];
        loss = loss + e * e;
        double dy = 2.0 * e / (double)R;
        gb3[0] = gb3[0] + dy;
        for (int64_t k = 0; k < H; ++k) {
            gw3[k] = gw3[k] + dy * h2[k];
            dz2[k] = z2[k] > 0.0 ? dy * w3[k] : 0.0;
        }
        for (int64_t j = 0; j < H; ++j) {
            gb2[j] = gb2[j] + dz2[j];
            for (int64_t k = 0; k < H; ++k) gW2[j * H + k] = gW2[j * H + k] + dz2[j] * h1[k];
        }
        for (int64_t k = 0; k < H; ++k) {
            double acc = 0.0;
            for (int64_t j = 0; j < H; ++j) acc = acc + W2[j * H + k] * dz2[j];
            dz1[k] = z1[k] > 0.0 ? acc : 0.0;
        }
        for (int64_t j = 0; j < H; ++j) {
            gb1[j] = gb1[j] + dz1[j];
            for (int64_t k = 0; k < F; ++k) gW1[j * F + k] = gW1[j * F + k] + dz1[j] * x[k];
        }
    }
    return loss / (double)R;
}

/* One Adam step (Kingma & Ba 2015, Algorithm 1) at step number `step` (>= 1):
 * m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2; mh = m/(1-b1^step); vh = v/(1-b2^step);
 * p = p - lr * mh / (sqrt(vh) + eps). */
int orc_adam(int64_t n, double *p, const double *g, double *m, double *v, int64_t step,
             double lr, double b1, double b2, double eps)
{
    if (step < 1) return -1;
    double c1 = 1.0 - pow(b1, (double)step), c2 = 1.0 - pow(b2, (double)step);
    for (int64_t i = 0; i < n; ++i) {
        m[i] = b1 * m[i] + (1.0 - b1) * g[i];
        v[i] = b2 * v[i] + (1.0 - b2) * g[i] * g[i];
        double mh = m[i] / c1, vh = v[i] / c2;
        p[i] = p[i] - lr * mh / (sqrt(vh) + eps);
    }
    return 0;
}
