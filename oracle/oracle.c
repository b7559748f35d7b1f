/*
 * FP64 CPU oracle of the state-vector method of Yao (arXiv:1912.10877).
 *
 * TEST INFRASTRUCTURE ONLY. This file is the plain, slow, obviously correct statement of
 * what the GPU path computes. Only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark may load it; the product path never calls it. It shares no code, header,
 * table or constant with the HIP path.
 *
 * Conventions (paper Sec. "Instructions on Quantum Registers" and "Batched Quantum
 * Registers"): qubit q is bit q of the amplitude index (little-endian readout); a batched
 * register holds B states and the amplitude of basis index i in batch slot b is psi[i*B+b].
 * A k-qubit matrix M acting on locs l_0..l_{k-1} has row/column index r = sum_j bit(l_j)<<j,
 * stored row-major M[r*2^k + s]. A control (c, v) passes when bit c of the index equals v
 * (v = 0 is the paper's "inverse control").
 *
 * Every loop follows the definition; nothing is blocked, fused or reordered. The gate loop
 * is split over OpenMP threads by output index only, which leaves every result bit-identical
 * to a single-threaded run; every reduction runs sequentially in index order.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

#define ORC_MAXK 6
#define ORC_MAXC 8

enum {
    ORC_X = 0, ORC_Y, ORC_Z, ORC_H, ORC_S, ORC_SDAG, ORC_T, ORC_TDAG,
    ORC_RX, ORC_RY, ORC_RZ, ORC_SHIFT, ORC_ROT, ORC_DENSE
};

/* One instruction of a circuit (the paper's put / control blocks lowered to locations). */
typedef struct {
    int kind;
    int param;               /* index into params, or -1 for the fixed angle below */
    int k;                   /* number of target qubits */
    int nctrl;
    int locs[ORC_MAXK];
    int ctrls[ORC_MAXC];
    int cvals[ORC_MAXC];
    double theta;            /* fixed angle when param < 0 */
    const cplx* G;           /* rot generator / dense matrix, 2^k x 2^k, else NULL */
} orc_gate;

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------------------ */
/* Gate matrices.                                                                        */
/* ------------------------------------------------------------------------------------ */

static int is_param_kind(int kind)
{
    return kind == ORC_RX || kind == ORC_RY || kind == ORC_RZ || kind == ORC_SHIFT || kind == ORC_ROT;
}

/* The Pauli matrices and the fixed gates, written out. */
static void set2(cplx* U, cplx a, cplx b, cplx c, cplx d)
{
    U[0] = a; U[1] = b; U[2] = c; U[3] = d;
}

static void pauli_matrix(int which, cplx* S)
{
    if (which == ORC_X) set2(S, 0, 1, 1, 0);
    else if (which == ORC_Y) set2(S, 0, -I, I, 0);
    else set2(S, 1, 0, 0, -1);
}

/* Generator Sigma of a rotation R_Sigma(theta) = exp(-i Sigma theta / 2) (Sec. "Forward
 * Mode"): a Pauli matrix for Rx/Ry/Rz, the supplied Hermitian reflexive matrix for rot. */
static void rotation_generator(const orc_gate* g, cplx* S)
{
    if (g->kind == ORC_RX) pauli_matrix(ORC_X, S);
    else if (g->kind == ORC_RY) pauli_matrix(ORC_Y, S);
    else if (g->kind == ORC_RZ) pauli_matrix(ORC_Z, S);
    else {
        long d = 1L << g->k;
        memcpy(S, g->G, sizeof(cplx) * d * d);
    }
}

/* U(theta) of one gate, 2^k x 2^k row-major. Returns the dimension. */
long orc_gate_matrix(const orc_gate* g, double theta, cplx* U)
{
    long d = 1L << g->k;
    switch (g->kind) {
    case ORC_X: pauli_matrix(ORC_X, U); break;
    case ORC_Y: pauli_matrix(ORC_Y, U); break;
    case ORC_Z: pauli_matrix(ORC_Z, U); break;
    case ORC_H: set2(U, 1 / sqrt(2.0), 1 / sqrt(2.0), 1 / sqrt(2.0), -1 / sqrt(2.0)); break;
    case ORC_S: set2(U, 1, 0, 0, I); break;
    case ORC_SDAG: set2(U, 1, 0, 0, -I); break;
    case ORC_T: set2(U, 1, 0, 0, cexp(I * M_PI / 4)); break;
    case ORC_TDAG: set2(U, 1, 0, 0, cexp(-I * M_PI / 4)); break;
    case ORC_SHIFT: set2(U, 1, 0, 0, cexp(I * theta)); break;  /* diag(1, e^{i theta}) */
    case ORC_RX: case ORC_RY: case ORC_RZ: case ORC_ROT: {
        /* exp(-i theta Sigma / 2) = cos(theta/2) 1 - i sin(theta/2) Sigma, since Sigma^2 = 1 */
        cplx* S = malloc(sizeof(cplx) * d * d);
        rotation_generator(g, S);
        for (long r = 0; r < d; ++r)
            for (long s = 0; s < d; ++s)
                U[r * d + s] = (r == s ? cos(theta / 2) : 0) - I * sin(theta / 2) * S[r * d + s];
        free(S);
        break;
    }
    case ORC_DENSE: memcpy(U, g->G, sizeof(cplx) * d * d); break;
    default: return -1;
    }
    return d;
}

/* dU/dtheta of a parametric gate, written from the same definitions. */
long orc_gate_deriv(const orc_gate* g, double theta, cplx* D)
{
    long d = 1L << g->k;
    if (g->kind == ORC_SHIFT) {
        set2(D, 0, 0, 0, I * cexp(I * theta));
        return d;
    }
    if (g->kind == ORC_RX || g->kind == ORC_RY || g->kind == ORC_RZ || g->kind == ORC_ROT) {
        cplx* S = malloc(sizeof(cplx) * d * d);
        rotation_generator(g, S);
        for (long r = 0; r < d; ++r)
            for (long s = 0; s < d; ++s)
                D[r * d + s] = (r == s ? -0.5 * sin(theta / 2) : 0) - 0.5 * I * cos(theta / 2) * S[r * d + s];
        free(S);
        return d;
    }
    return -1;
}

static void conj_transpose(long d, const cplx* U, cplx* Ud)
{
    for (long r = 0; r < d; ++r)
        for (long s = 0; s < d; ++s)
            Ud[s * d + r] = conj(U[r * d + s]);
}

/* ------------------------------------------------------------------------------------ */
/* Applying an operator to a register.                                                   */
/* ------------------------------------------------------------------------------------ */

/* out = F in, where F acts as M on the locs of every index whose controls pass, and as the
 * identity (identity_outside = 1) or as zero (identity_outside = 0) on the other indices:
 *   out[i] = sum_s M[r(i), s] in[i with bit l_j set to bit j of s]. */
void orc_apply_op(int n, long B, const cplx* in, cplx* out, const cplx* M, int k, const int* locs,
                  int nctrl, const int* ctrls, const int* cvals, int identity_outside)
{
    const long N = 1L << n;
    const long d = 1L << k;
#pragma omp parallel for schedule(static) if ((1L << n) * B >= (1L << 14))
    for (long i = 0; i < N; ++i) {
        int pass = 1;
        for (int m = 0; m < nctrl; ++m)
            if (((i >> ctrls[m]) & 1) != cvals[m]) pass = 0;
        long r = 0;
        for (int j = 0; j < k; ++j) r |= ((i >> locs[j]) & 1L) << j;
        for (long b = 0; b < B; ++b) {
            if (!pass) {
                out[i * B + b] = identity_outside ? in[i * B + b] : 0;
                continue;
            }
            cplx acc = 0;
            for (long s = 0; s < d; ++s) {
                long idx = i;
                for (int j = 0; j < k; ++j) {
                    idx &= ~(1L << locs[j]);
                    idx |= ((s >> j) & 1L) << locs[j];
                }
                acc += M[r * d + s] * in[idx * B + b];
            }
            out[i * B + b] = acc;
        }
    }
}

/* psi <- F psi in place through a scratch copy. */
void orc_apply(int n, long B, cplx* psi, const cplx* U, int k, const int* locs, int nctrl,
               const int* ctrls, const int* cvals)
{
    const long len = (1L << n) * B;
    cplx* tmp = malloc(sizeof(cplx) * len);
    orc_apply_op(n, B, psi, tmp, U, k, locs, nctrl, ctrls, cvals, 1);
    memcpy(psi, tmp, sizeof(cplx) * len);
    free(tmp);
}

static double gate_theta(const orc_gate* g, const double* params)
{
    return g->param >= 0 ? params[g->param] : g->theta;
}

/* Sec. "Representing Quantum Circuits": a chain applies its blocks first to last. */
void orc_forward(int n, long B, cplx* psi, int ngates, const orc_gate* gates, const double* params)
{
    cplx U[1 << (2 * ORC_MAXK)];
    for (int t = 0; t < ngates; ++t) {
        orc_gate_matrix(&gates[t], gate_theta(&gates[t], params), U);
        orc_apply(n, B, psi, U, gates[t].k, gates[t].locs, gates[t].nctrl, gates[t].ctrls, gates[t].cvals);
    }
}

/* ------------------------------------------------------------------------------------ */
/* Observables.                                                                          */
/* ------------------------------------------------------------------------------------ */

/* out = P psi for the Pauli string with X on bits of x only, Z on bits of z only and Y on
 * bits of both, applied one single-qubit factor at a time. */
void orc_pauli_apply(int n, long B, const cplx* psi, cplx* out, uint64_t x, uint64_t z)
{
    const long len = (1L << n) * B;
    memcpy(out, psi, sizeof(cplx) * len);
    for (int q = 0; q < n; ++q) {
        int bx = (x >> q) & 1, bz = (z >> q) & 1;
        if (!bx && !bz) continue;
        cplx S[4];
        pauli_matrix(bx && bz ? ORC_Y : (bx ? ORC_X : ORC_Z), S);
        orc_apply(n, B, out, S, 1, &q, 0, NULL, NULL);
    }
}

/* out = H psi with H = sum_t coef[t] P_t (Listing "Heisenberg Hamiltonian": sum of blocks). */
void orc_hpsi(int n, long B, const cplx* psi, cplx* out, int nterms, const double* coef,
              const uint64_t* x, const uint64_t* z)
{
    const long len = (1L << n) * B;
    cplx* tmp = malloc(sizeof(cplx) * len);
    memset(out, 0, sizeof(cplx) * len);
    for (int t = 0; t < nterms; ++t) {
        orc_pauli_apply(n, B, psi, tmp, x[t], z[t]);
        for (long e = 0; e < len; ++e) out[e] += coef[t] * tmp[e];
    }
    free(tmp);
}

/* <a|b> for each batch slot, summed in index order. */
static void inner(int n, long B, const cplx* a, const cplx* b, cplx* res)
{
    const long N = 1L << n;
    for (long s = 0; s < B; ++s) {
        cplx acc = 0;
        for (long i = 0; i < N; ++i) acc += conj(a[i * B + s]) * b[i * B + s];
        res[s] = acc;
    }
}

/* expect(H, reg) (Sec. "Forward Mode"): <psi|H|psi> per batch slot, real and imaginary part. */
void orc_expect(int n, long B, const cplx* psi, int nterms, const double* coef, const uint64_t* x,
                const uint64_t* z, double* e_re, double* e_im)
{
    const long len = (1L << n) * B;
    cplx* hp = malloc(sizeof(cplx) * len);
    cplx* res = malloc(sizeof(cplx) * B);
    orc_hpsi(n, B, psi, hp, nterms, coef, x, z);
    inner(n, B, psi, hp, res);
    for (long s = 0; s < B; ++s) {
        e_re[s] = creal(res[s]);
        if (e_im) e_im[s] = cimag(res[s]);
    }
    free(res);
    free(hp);
}

/* Energy of psi0 pushed through the circuit (the paper's expect(h, reg => circuit)). */
void orc_energy(int n, long B, const cplx* psi0, int ngates, const orc_gate* gates, const double* params,
                int nterms, const double* coef, const uint64_t* x, const uint64_t* z, double* e_re)
{
    const long len = (1L << n) * B;
    cplx* psi = malloc(sizeof(cplx) * len);
    memcpy(psi, psi0, sizeof(cplx) * len);
    orc_forward(n, B, psi, ngates, gates, params);
    orc_expect(n, B, psi, nterms, coef, x, z, e_re, NULL);
    free(psi);
}

/* ------------------------------------------------------------------------------------ */
/* Reverse mode with uncomputation (Sec. "Reverse Mode", eqs. apply-back and outer-product) */
/* ------------------------------------------------------------------------------------ */

/* L = <psi_N|H|psi_N>. Forward: psi_{k+1} = U_k psi_k. The adjoint of the output state is
 * psibar_N = dL/dpsi_N^* = H psi_N (Wirtinger). Backward, gate by gate from the last:
 *   psi_k    = U_k^dagger psi_{k+1}          (uncompute)
 *   Ubar_k   = psibar_{k+1} <psi_k|          (outer product, never formed)
 *   thetabar = 2 Re Tr(Ubar_k^dagger dF_k/dtheta) = 2 Re <psibar_{k+1}| dF_k/dtheta |psi_k>
 *   psibar_k = U_k^dagger psibar_{k+1}
 * where F_k is the full-register operator of gate k (its matrix on the controlled subspace,
 * identity elsewhere), so dF_k/dtheta is dU_k/dtheta there and zero elsewhere. Gradients
 * of a shared parameter add up (Sec. "Reverse Mode"). grad is [B][nparams], one gradient
 * per batch slot; the paper's batched gradient is its sum over slots.
 * On return psi0_back holds the uncomputed input state (for the reversibility check). */
void orc_adjoint(int n, long B, const cplx* psi0, int ngates, const orc_gate* gates, const double* params,
                 int nparams, int nterms, const double* coef, const uint64_t* x, const uint64_t* z,
                 double* energy, double* grad, cplx* psi0_back)
{
    const long len = (1L << n) * B;
    cplx* psi = malloc(sizeof(cplx) * len);
    cplx* prev = malloc(sizeof(cplx) * len);
    cplx* bar = malloc(sizeof(cplx) * len);
    cplx* dpsi = malloc(sizeof(cplx) * len);
    cplx* res = malloc(sizeof(cplx) * B);
    cplx U[1 << (2 * ORC_MAXK)], Ud[1 << (2 * ORC_MAXK)], D[1 << (2 * ORC_MAXK)];

    memcpy(psi, psi0, sizeof(cplx) * len);
    orc_forward(n, B, psi, ngates, gates, params);
    orc_hpsi(n, B, psi, bar, nterms, coef, x, z);
    inner(n, B, psi, bar, res);
    for (long s = 0; s < B; ++s) energy[s] = creal(res[s]);
    memset(grad, 0, sizeof(double) * B * nparams);

    for (int t = ngates - 1; t >= 0; --t) {
        const orc_gate* g = &gates[t];
        double th = gate_theta(g, params);
        long d = orc_gate_matrix(g, th, U);
        conj_transpose(d, U, Ud);
        orc_apply_op(n, B, psi, prev, Ud, g->k, g->locs, g->nctrl, g->ctrls, g->cvals, 1);
        if (is_param_kind(g->kind) && g->param >= 0) {
            orc_gate_deriv(g, th, D);
            orc_apply_op(n, B, prev, dpsi, D, g->k, g->locs, g->nctrl, g->ctrls, g->cvals, 0);
            inner(n, B, bar, dpsi, res);
            for (long s = 0; s < B; ++s) grad[s * nparams + g->param] += 2.0 * creal(res[s]);
        }
        orc_apply(n, B, bar, Ud, g->k, g->locs, g->nctrl, g->ctrls, g->cvals);
        memcpy(psi, prev, sizeof(cplx) * len);
    }
    if (psi0_back) memcpy(psi0_back, psi, sizeof(cplx) * len);
    free(res); free(dpsi); free(bar); free(prev); free(psi);
}

/* ------------------------------------------------------------------------------------ */
/* Qubit management: focus! / relax! (Sec. "Active qubits and environment qubits").       */
/* ------------------------------------------------------------------------------------ */

/* out = the register with qubit q moved to position perm[q]: for every index i, the index i'
 * whose bit perm[q] is bit q of i receives in[i]. perm is a permutation of 0..n-1. */
void orc_permute_qubits(int n, long B, const cplx* in, cplx* out, const int* perm)
{
    const long N = 1L << n;
#pragma omp parallel for schedule(static) if ((1L << n) * B >= (1L << 14))
    for (long i = 0; i < N; ++i) {
        long ip = 0;
        for (int q = 0; q < n; ++q) ip |= ((i >> q) & 1L) << perm[q];
        for (long b = 0; b < B; ++b) out[ip * B + b] = in[i * B + b];
    }
}

/* ------------------------------------------------------------------------------------ */
/* Quantum Fourier transform on a set of qubits (Listing "QFT circuit", App. "Extending    */
/* QBIR: emulating QFT circuit").                                                          */
/* ------------------------------------------------------------------------------------ */

/* Bits of the locs of index i, locs[j] -> bit j. */
static long sub_index(long i, int k, const int* locs)
{
    long r = 0;
    for (int j = 0; j < k; ++j) r |= ((i >> locs[j]) & 1L) << j;
    return r;
}

static long with_sub_index(long i, int k, const int* locs, long s)
{
    for (int j = 0; j < k; ++j) {
        i &= ~(1L << locs[j]);
        i |= ((s >> j) & 1L) << locs[j];
    }
    return i;
}

static long reverse_bits(long x, int k)
{
    long r = 0;
    for (int j = 0; j < k; ++j) r |= ((x >> j) & 1L) << (k - 1 - j);
    return r;
}

/* The QFT on the k qubits locs as a matrix acting on the sub-index x = sum_j bit(locs[j]) 2^j:
 *   F[y][x] = 2^{-k/2} exp(+2 pi i rev(x) y / 2^k)     (the paper's circuit: the emulation
 * reverses the qubit order, then applies the unitary inverse DFT), and its inverse
 *   F^dagger[x][y] = 2^{-k/2} exp(-2 pi i rev(x) y / 2^k).
 * Output element idx[m] (every batch slot) is the sum over the sub-index of the row of F (or
 * F^dagger) for idx[m]'s own sub-index. out is [nidx][B]. The phase rev(x) y is reduced mod 2^k
 * in integers before the exponential. */
void orc_qft_at(int n, long B, const cplx* psi, int k, const int* locs, int inverse, long nidx, const long* idx,
                cplx* out)
{
    const long d = 1L << k;
    const double norm = 1.0 / sqrt((double)d);
    (void)n;
#pragma omp parallel for schedule(static) if ((1L << n) * B >= (1L << 14))
    for (long m = 0; m < nidx; ++m) {
        const long i = idx[m];
        const long r = sub_index(i, k, locs);
        for (long b = 0; b < B; ++b) {
            cplx acc = 0;
            for (long s = 0; s < d; ++s) {
                long ph;
                if (!inverse) ph = (reverse_bits(s, k) * r) & (d - 1);       /* F[r][s] */
                else ph = (d - ((reverse_bits(r, k) * s) & (d - 1))) & (d - 1);  /* F^dagger[r][s] */
                acc += cexp(I * 2.0 * M_PI * (double)ph / (double)d) * psi[with_sub_index(i, k, locs, s) * B + b];
            }
            out[m * B + b] = norm * acc;
        }
    }
}

/* ------------------------------------------------------------------------------------ */
/* Measurement (Listing "instruct! and measure": measure and measure!).                   */
/* ------------------------------------------------------------------------------------ */

/* probs[b][x] = sum over indices i whose locs bits read x of |psi[i][b]|^2, in index order. */
void orc_probs(int n, long B, const cplx* psi, int k, const int* locs, double* probs)
{
    const long N = 1L << n, d = 1L << k;
    memset(probs, 0, sizeof(double) * B * d);
    for (long i = 0; i < N; ++i) {
        const long x = sub_index(i, k, locs);
        for (long b = 0; b < B; ++b) {
            const cplx a = psi[i * B + b];
            probs[b * d + x] += creal(a) * creal(a) + cimag(a) * cimag(a);
        }
    }
}

/* measure(reg; nshots): outcome of shot s in slot b is the smallest x whose cumulative
 * probability cdf[x] = sum_{y <= x} p[y] (summed in order of y) exceeds u[b][s] * cdf[last],
 * for uniform numbers u in [0, 1) supplied by the caller (inverse-CDF sampling). */
void orc_sample(int n, long B, const cplx* psi, int k, const int* locs, long nshots, const double* u, long* out)
{
    const long d = 1L << k;
    double* p = malloc(sizeof(double) * B * d);
    double* cdf = malloc(sizeof(double) * d);
    orc_probs(n, B, psi, k, locs, p);
    for (long b = 0; b < B; ++b) {
        double run = 0;
        for (long x = 0; x < d; ++x) {
            run += p[b * d + x];
            cdf[x] = run;
        }
        for (long s = 0; s < nshots; ++s) {
            const double target = u[b * nshots + s] * cdf[d - 1];
            long lo = 0, hi = d - 1;  /* smallest x with cdf[x] > target; cdf[d-1] > target */
            while (lo < hi) {
                long mid = (lo + hi) / 2;
                if (cdf[mid] > target) hi = mid;
                else lo = mid + 1;
            }
            out[b * nshots + s] = lo;
        }
    }
    free(cdf);
    free(p);
}

/* measure!: project slot b onto the outcome x_b of the locs and renormalise:
 * psi[i][b] <- psi[i][b] / sqrt(p_b) where the locs bits of i read x_b, else 0. p_out[b]
 * receives p_b. */
void orc_collapse(int n, long B, cplx* psi, int k, const int* locs, const long* outcome, double* p_out)
{
    const long N = 1L << n, d = 1L << k;
    double* p = malloc(sizeof(double) * B * d);
    orc_probs(n, B, psi, k, locs, p);
    for (long i = 0; i < N; ++i) {
        const long x = sub_index(i, k, locs);
        for (long b = 0; b < B; ++b) {
            const double pb = p[b * d + outcome[b]];
            psi[i * B + b] = x == outcome[b] ? psi[i * B + b] / sqrt(pb) : 0;
        }
    }
    for (long b = 0; b < B; ++b) p_out[b] = p[b * d + outcome[b]];
    free(p);
}
