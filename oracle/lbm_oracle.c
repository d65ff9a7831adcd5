/*
 * lbm_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, double-precision CPU statement of what the list-based
 * lattice Boltzmann hot path computes.  It exists to check the GPU library
 * against; only the test-suite, the smoke check and the CPU-baseline leg of
 * the benchmark load it.  It shares no code, header, table or constant with
 * the GPU library: its velocity set, numbering keys and collision are written
 * out again here, from the definitions below.
 *
 * What it states (paper = Wittmann, Zeiser, Hager, Wellein, "Domain
 * decomposition and locality optimization for large-scale lattice Boltzmann
 * simulations"):
 *
 *  - Numbering scheme (Sec. 3, "Numbering scheme"): every box cell, fluid or
 *    solid, gets a unique key I(x,y,z) from an injective index function:
 *    lexicographic with or without blocking, Z curve with 1-bit or 2-bit
 *    interleave (Sec. 7, single node performance), the Hilbert curve (named
 *    in Sec. 3), or any injective f -- here a keyed Feistel bijection for a
 *    random control ordering.
 *  - Contiguous index (Sec. 3, "Contiguous index generation"): fluid cells
 *    get I_c = their rank among fluid keys.  The paper's octree merge of
 *    incell runs computes exactly this rank; the oracle computes it by
 *    sorting (0-based; solid cells get -1 instead of the paper's 0).
 *  - Adjacency (Sec. 1, Sec. 2, Sec. 3 last paragraph): 18 neighbour entries
 *    per fluid cell, found by inspecting its neighbourhood in the full
 *    representation; a solid neighbour encodes bounce-back implicitly by
 *    pointing at the cell's own opposite population.
 *  - Flow step (Sec. 1, Sec. 7): D3Q19 two-relaxation-time collision with the
 *    pull scheme on a structure-of-arrays PDF list.  The paper names TRT but
 *    prints no equations; the TRT equilibrium, forcing and partial
 *    bounce-back used here are the standard literature forms (incompressible
 *    second-order equilibrium, force term 3 w_i c_i.G added after collision,
 *    out = (1 - ns) f* + ns g_opp).
 *  - Moments: rho = sum g, u = j + G/2 from the gathered populations.
 *  - Adjoint: the transposed Jacobian of one step, applied to lambda and
 *    scattered back through the same adjacency; derivative of the step with
 *    respect to the partial-bounce-back solid fraction.
 *
 * Compile: gcc -O2 -std=c99 -fPIC -shared -fopenmp -ffp-contract=off.
 * Floating point contraction is off so that every operation rounds as written.
 */
#include <complex.h>
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ECAPACITY (-2)
#define ORC_EOVERFLOW (-3)

enum { ORD_LEX = 0, ORD_BLOCKED = 1, ORD_MORTON1 = 2, ORD_MORTON2 = 3, ORD_RANDOM = 4,
       ORD_HILBERT = 5 };

/* ---- D3Q19 velocity set: rest, 6 axis links, 12 diagonal links.
 * Opposite pairs are (1,2), (3,4), ..., (17,18). */
static const int CX[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
static const int CY[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
static const int CZ[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
static const double W[19] = {
    1.0 / 3.0,
    1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0,
    1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0,
    1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};

static int opposite(int i) {
    if (i == 0) return 0;
    return (i % 2 == 1) ? i + 1 : i - 1;
}

int orc_velocity(int i, int* c) {
    if (i < 0 || i > 18) return ORC_EINVAL;
    c[0] = CX[i]; c[1] = CY[i]; c[2] = CZ[i];
    return opposite(i);
}

double orc_weight(int i) { return (i >= 0 && i < 19) ? W[i] : 0.0; }

/* ---- numbering keys ---------------------------------------------------- */

/* One output of the SplitMix64 generator (Steele, Lea, Flood, OOPSLA 2014)
 * whose state before the step was x. */
uint64_t orc_splitmix64(uint64_t x) {
    uint64_t z = x + 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* Half width h of the random ordering's key space [0, 4^h): the smallest
 * h >= 1 with 4^h >= n_box. */
int orc_feistel_half_bits(uint64_t n_box) {
    int h = 1;
    while (h < 31 && ((uint64_t)1 << (2 * h)) < n_box) ++h;
    return h;
}

/* Four-round balanced Feistel network on 2h-bit words.  Word v splits into a
 * high half L and a low half R; round r maps (L, R) -> (R, L xor F_r(R)) with
 * F_r(R) = splitmix64(seed xor (r << 32) xor R) masked to h bits. */
uint64_t orc_feistel(uint64_t seed, int h, uint64_t v) {
    uint64_t mask = ((uint64_t)1 << h) - 1;
    uint64_t L = (v >> h) & mask, R = v & mask;
    for (uint64_t r = 0; r < 4; ++r) {
        uint64_t F = orc_splitmix64(seed ^ (r << 32) ^ R) & mask;
        uint64_t nl = R, nr = L ^ F;
        L = nl;
        R = nr;
    }
    return (L << h) | R;
}

/* Hilbert curve key on the 2^B cube (Skilling, "Programming the Hilbert
 * curve", AIP Conf. Proc. 707, 2004).  The coordinates are turned into the
 * "transposed" Hilbert index: from the top level down, every lower-order
 * bit pattern is reflected or exchanged with the x word so that each
 * sub-cube is entered in the orientation the curve needs, then the three
 * words are Gray-coded.  The key reads the transposed words level by level,
 * x's bit the most significant of each 3-bit digit. */
static uint64_t hilbert_key(int B, uint64_t x, uint64_t y, uint64_t z) {
    if (B == 0) return 0;
    uint64_t X[3] = {x, y, z};
    const uint64_t top = (uint64_t)1 << (B - 1);
    for (uint64_t q = top; q > 1; q >>= 1) {
        const uint64_t low = q - 1;
        for (int i = 0; i < 3; ++i) {
            if (X[i] & q) {
                X[0] ^= low;
            } else {
                uint64_t swap = (X[0] ^ X[i]) & low;
                X[0] ^= swap;
                X[i] ^= swap;
            }
        }
    }
    X[1] ^= X[0];
    X[2] ^= X[1];
    uint64_t flip = 0;
    for (uint64_t q = top; q > 1; q >>= 1)
        if (X[2] & q) flip ^= q - 1;
    for (int i = 0; i < 3; ++i) X[i] ^= flip;
    uint64_t key = 0;
    for (int j = B - 1; j >= 0; --j)
        for (int i = 0; i < 3; ++i) key = (key << 1) | ((X[i] >> j) & 1);
    return key;
}

static int bits_to_hold(int64_t n) {
    int b = 0;
    while (((int64_t)1 << b) < n) ++b;
    return b;
}

/* Key I(x,y,z) of a box cell for the given ordering. */
uint64_t orc_key(int order, uint64_t param, int64_t nx, int64_t ny, int64_t nz,
                 int64_t x, int64_t y, int64_t z) {
    uint64_t lin = (uint64_t)(x + nx * (y + ny * z));
    switch (order) {
    case ORD_LEX:
        return lin;
    case ORD_BLOCKED: {
        /* cubic blocks of edge b visited block-lexicographically, cells
         * lexicographically inside each block; edge blocks are truncated */
        int64_t b = (int64_t)param;
        int64_t nbx = (nx + b - 1) / b, nby = (ny + b - 1) / b;
        int64_t X = x / b, Y = y / b, Z = z / b;
        uint64_t block = (uint64_t)((Z * nby + Y) * nbx + X);
        uint64_t inner = (uint64_t)(((z % b) * b + (y % b)) * b + (x % b));
        return block * (uint64_t)(b * b * b) + inner;
    }
    case ORD_MORTON1: {
        /* bit k of x, y, z goes to bit 3k, 3k+1, 3k+2 */
        uint64_t key = 0;
        for (int k = 0; k < 21; ++k) {
            key |= (uint64_t)((x >> k) & 1) << (3 * k);
            key |= (uint64_t)((y >> k) & 1) << (3 * k + 1);
            key |= (uint64_t)((z >> k) & 1) << (3 * k + 2);
        }
        return key;
    }
    case ORD_MORTON2: {
        /* 2-bit group k of x, y, z goes to bits [6k, 6k+2), [6k+2, 6k+4),
         * [6k+4, 6k+6) */
        uint64_t key = 0;
        for (int k = 0; k < 10; ++k) {
            key |= (uint64_t)((x >> (2 * k)) & 3) << (6 * k);
            key |= (uint64_t)((y >> (2 * k)) & 3) << (6 * k + 2);
            key |= (uint64_t)((z >> (2 * k)) & 3) << (6 * k + 4);
        }
        return key;
    }
    case ORD_RANDOM: {
        uint64_t n_box = (uint64_t)(nx * ny * nz);
        return orc_feistel(param, orc_feistel_half_bits(n_box), lin);
    }
    case ORD_HILBERT: {
        int64_t dmax = nx > ny ? nx : ny;
        if (nz > dmax) dmax = nz;
        return hilbert_key(bits_to_hold(dmax), (uint64_t)x, (uint64_t)y, (uint64_t)z);
    }
    default:
        return 0;
    }
}

/* ---- compaction and adjacency ------------------------------------------ */

typedef struct {
    uint64_t key;
    int64_t lin;
} keyed_cell;

static int by_key(const void* a, const void* b) {
    uint64_t ka = ((const keyed_cell*)a)->key, kb = ((const keyed_cell*)b)->key;
    return (ka > kb) - (ka < kb);
}

/*
 * Build the sparse representation of one geometry.
 *   flag[lin], lin = x + nx*(y + ny*z): nonzero = fluid.
 *   periodic: bit0 x, bit1 y, bit2 z.
 *   index_of[lin] (n_box entries, may be NULL): I_c of a fluid cell, -1 solid.
 *   cell_of[m] (cap entries): lin of the fluid cell with I_c = m.
 *   adj[k*stride + base + m], k in [0,18): PDF slot pulled for direction
 *   i = k+1 by cell m: i*stride + base + I_c(upstream) if the upstream cell
 *   x - c_i (wrapped in periodic directions) is fluid, else the bounce-back
 *   slot opp(i)*stride + base + m.
 * Returns ORC_ECAPACITY (with *n_fluid set) when cap is too small.
 */
int orc_build(int64_t nx, int64_t ny, int64_t nz, uint32_t periodic, int order,
              uint64_t param, const uint8_t* flag, int64_t base, int64_t stride,
              int32_t* index_of, int32_t* cell_of, uint32_t* adj, int64_t cap,
              int64_t* n_fluid) {
    if (nx <= 0 || ny <= 0 || nz <= 0 || !flag || !n_fluid) return ORC_EINVAL;
    if (order < ORD_LEX || order > ORD_HILBERT) return ORC_EINVAL;
    if (order == ORD_BLOCKED && param == 0) return ORC_EINVAL;
    int64_t n_box = nx * ny * nz;
    if (n_box >= ((int64_t)1 << 31)) return ORC_EOVERFLOW;

    int64_t nf = 0;
    for (int64_t lin = 0; lin < n_box; ++lin) nf += flag[lin] != 0;
    *n_fluid = nf;
    if (!cell_of) return ORC_OK; /* count only */
    if (nf > cap) return ORC_ECAPACITY;
    if (adj && (stride < base + nf || 19 * stride >= ((int64_t)1 << 32))) return ORC_EOVERFLOW;

    keyed_cell* kc = (keyed_cell*)malloc(sizeof(keyed_cell) * (size_t)(nf > 0 ? nf : 1));
    int32_t* idx = (int32_t*)malloc(sizeof(int32_t) * (size_t)n_box);
    if (!kc || !idx) {
        free(kc);
        free(idx);
        return ORC_EINVAL;
    }
    int64_t m = 0;
    for (int64_t z = 0; z < nz; ++z)
        for (int64_t y = 0; y < ny; ++y)
            for (int64_t x = 0; x < nx; ++x) {
                int64_t lin = x + nx * (y + ny * z);
                if (flag[lin]) {
                    kc[m].key = orc_key(order, param, nx, ny, nz, x, y, z);
                    kc[m].lin = lin;
                    ++m;
                }
            }
    qsort(kc, (size_t)nf, sizeof(keyed_cell), by_key);

    for (int64_t lin = 0; lin < n_box; ++lin) idx[lin] = -1;
    for (int64_t r = 0; r < nf; ++r) {
        idx[kc[r].lin] = (int32_t)r;
        cell_of[r] = (int32_t)kc[r].lin;
    }
    if (index_of) memcpy(index_of, idx, sizeof(int32_t) * (size_t)n_box);

    if (adj) {
        int64_t dims[3] = {nx, ny, nz};
        for (int64_t r = 0; r < nf; ++r) {
            int64_t lin = kc[r].lin;
            int64_t p[3] = {lin % nx, (lin / nx) % ny, lin / (nx * ny)};
            for (int i = 1; i < 19; ++i) {
                int c[3] = {CX[i], CY[i], CZ[i]};
                int64_t q[3];
                int inside = 1;
                for (int d = 0; d < 3; ++d) {
                    q[d] = p[d] - c[d];
                    if (q[d] < 0 || q[d] >= dims[d]) {
                        if (periodic & (1u << d))
                            q[d] = (q[d] + dims[d]) % dims[d];
                        else
                            inside = 0;
                    }
                }
                int32_t up = -1;
                if (inside) up = idx[q[0] + nx * (q[1] + ny * q[2])];
                uint64_t slot;
                if (up >= 0)
                    slot = (uint64_t)i * (uint64_t)stride + (uint64_t)base + (uint64_t)up;
                else
                    slot = (uint64_t)opposite(i) * (uint64_t)stride + (uint64_t)base + (uint64_t)r;
                adj[(int64_t)(i - 1) * stride + base + r] = (uint32_t)slot;
            }
        }
    }
    free(kc);
    free(idx);
    return ORC_OK;
}

/* ---- relaxation rates --------------------------------------------------
 * TRT: tau_minus follows from the "magic" parameter
 * Lambda = (tau_plus - 1/2)(tau_minus - 1/2). */
void orc_rates(double tau_plus, double magic, double* s_plus, double* s_minus) {
    double tau_minus = 0.5 + magic / (tau_plus - 0.5);
    *s_plus = 1.0 / tau_plus;
    *s_minus = 1.0 / tau_minus;
}

/* ---- equilibrium initialisation ----------------------------------------
 * f_i = w_i [rho0 + 3 c_i.u0 + 9/2 (c_i.u0)^2 - 3/2 |u0|^2]; in shifted
 * storage the stored value is f_i - w_i, computed as w_i [(rho0 - 1) + ...]. */
void orc_init(int64_t n0, int64_t n1, int64_t stride, int shifted, double rho0,
              const double* u0, double* f) {
    double ux = u0 ? u0[0] : 0.0, uy = u0 ? u0[1] : 0.0, uz = u0 ? u0[2] : 0.0;
    double uu = ux * ux + uy * uy + uz * uz;
    double r = shifted ? rho0 - 1.0 : rho0;
    for (int i = 0; i < 19; ++i) {
        double cu = CX[i] * ux + CY[i] * uy + CZ[i] * uz;
        double v = W[i] * (r + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
        for (int64_t n = n0; n < n1; ++n) f[(int64_t)i * stride + n] = v;
    }
}

/* Neumaier's compensated addition: s + c carries the running sum. */
static void neumaier_add(double* s, double* c, double v) {
    double t = *s + v;
    if (fabs(*s) >= fabs(v))
        *c += (*s - t) + v;
    else
        *c += (v - t) + *s;
    *s = t;
}

/* ---- the flow step, moments: written once for real and once for complex
 * scalars (the complex instance serves complex-step differentiation). */
#define SCALAR double
#define FN(name) name
#include "trt_step.inc"
#undef SCALAR
#undef FN

#define SCALAR double complex
#define FN(name) name##_c
#include "trt_step.inc"
#undef SCALAR
#undef FN

/* ---- adjoint step --------------------------------------------------------
 * One forward step maps f^t to f^{t+1}: gather g_k(n) = f^t[A_k(n)] (A_0(n) is
 * the cell's own rest slot, A_k for k >= 1 the adjacency entry), then
 * out_i = (1 - ns) f*_i(g) + ns g_opp(i).  Its transposed Jacobian applied to
 * mu = lambda^{t+1}[.][n] gives nu_k = sum_i mu_i d out_i / d g_k, which is
 * scattered to lambda^t[A_k(n)]; the pull is a permutation of PDF slots, so
 * every slot of lambda^t is written exactly once.
 *
 * With Pi+- the symmetric/antisymmetric projections and
 *   d e+_i / d g_k = w_i [1 + 9 (c_i.j)(c_i.c_k) - 3 j.c_k],
 *   d e-_i / d g_k = 3 w_i c_i.c_k,
 * the contraction is
 *   nu_k = (1-ns)[mu_k - s+ mu+_k - s- mu-_k
 *                 + s+ (m0 + 9 c_k.m2 - 3 m0 c_k.j) + 3 s- c_k.m1] + ns mu_opp(k)
 * with m0 = sum w_i mu_i, m1 = sum w_i mu_i c_i, m2 = sum w_i mu_i (c_i.j) c_i.
 * The solid-fraction derivative is d out_i / d ns = g_opp(i) - f*_i, so
 * grad[n] += sum_i mu_i (g_opp(i) - f*_i).
 *
 * lam_next == NULL writes the seed lambda^T = dJ/df^T of the objective
 * J = mean over cells [n0, n1) of u_x, u_x = j_x + G_x/2 from the gathered
 * populations: lambda^T[A_k(n)] = c_kx / (n1 - n0).
 */
void orc_step_adjoint(double tau_plus, double magic, const double* G, int64_t n0, int64_t n1,
                      int64_t stride, const uint32_t* adj, const double* f_t, const double* ns,
                      const double* lam_next, double* lam_t, double* grad) {
    double sp, sm;
    orc_rates(tau_plus, magic, &sp, &sm);
    double inv_n = 1.0 / (double)(n1 - n0);
    int64_t n;
#pragma omp parallel for schedule(static)
    for (n = n0; n < n1; ++n) {
        uint64_t A[19];
        A[0] = (uint64_t)n;
        for (int k = 1; k < 19; ++k) A[k] = adj[(int64_t)(k - 1) * stride + n];
        if (!lam_next) {
            for (int k = 0; k < 19; ++k) lam_t[A[k]] = CX[k] * inv_n;
            continue;
        }
        double g[19], mu[19], fstar[19];
        for (int k = 0; k < 19; ++k) g[k] = f_t[A[k]];
        for (int k = 0; k < 19; ++k) mu[k] = lam_next[(int64_t)k * stride + n];
        double rho = 0, jx = 0, jy = 0, jz = 0;
        for (int i = 0; i < 19; ++i) {
            rho += g[i];
            jx += CX[i] * g[i];
            jy += CY[i] * g[i];
            jz += CZ[i] * g[i];
        }
        double jj = jx * jx + jy * jy + jz * jz;
        for (int i = 0; i < 19; ++i) {
            int o = opposite(i);
            double cu = CX[i] * jx + CY[i] * jy + CZ[i] * jz;
            double ep = W[i] * (rho + 4.5 * cu * cu - 1.5 * jj);
            double em = 3.0 * W[i] * cu;
            double gp = 0.5 * (g[i] + g[o]), gm = 0.5 * (g[i] - g[o]);
            double force = 3.0 * W[i] * (CX[i] * G[0] + CY[i] * G[1] + CZ[i] * G[2]);
            fstar[i] = g[i] - sp * (gp - ep) - sm * (gm - em) + force;
        }
        double s = ns ? ns[n] : 0.0;
        if (ns && grad) {
            double acc = 0.0;
            for (int i = 0; i < 19; ++i) acc += mu[i] * (g[opposite(i)] - fstar[i]);
            grad[n] += acc;
        }
        double m0 = 0, m1[3] = {0, 0, 0}, m2[3] = {0, 0, 0};
        for (int i = 0; i < 19; ++i) {
            double cu = CX[i] * jx + CY[i] * jy + CZ[i] * jz;
            m0 += W[i] * mu[i];
            m1[0] += W[i] * mu[i] * CX[i];
            m1[1] += W[i] * mu[i] * CY[i];
            m1[2] += W[i] * mu[i] * CZ[i];
            m2[0] += W[i] * mu[i] * cu * CX[i];
            m2[1] += W[i] * mu[i] * cu * CY[i];
            m2[2] += W[i] * mu[i] * cu * CZ[i];
        }
        for (int k = 0; k < 19; ++k) {
            int o = opposite(k);
            double ckj = CX[k] * jx + CY[k] * jy + CZ[k] * jz;
            double ckm1 = CX[k] * m1[0] + CY[k] * m1[1] + CZ[k] * m1[2];
            double ckm2 = CX[k] * m2[0] + CY[k] * m2[1] + CZ[k] * m2[2];
            double mup = 0.5 * (mu[k] + mu[o]), mum = 0.5 * (mu[k] - mu[o]);
            double col = mu[k] - sp * mup - sm * mum + sp * (m0 + 9.0 * ckm2 - 3.0 * m0 * ckj)
                         + 3.0 * sm * ckm1;
            lam_t[A[k]] = ns ? (1.0 - s) * col + s * mu[o] : col;
        }
    }
}

/* ---- threading controls for timing runs --------------------------------- */
#ifdef _OPENMP
#include <omp.h>
void orc_set_threads(int n) { if (n > 0) omp_set_num_threads(n); }
int orc_max_threads(void) { return omp_get_max_threads(); }
#else
void orc_set_threads(int n) { (void)n; }
int orc_max_threads(void) { return 1; }
#endif
