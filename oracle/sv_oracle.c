/*
 * CPU oracle for the sliced state-vector path.  TEST INFRASTRUCTURE ONLY.
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * load this library.  It shares no code with the GPU library: no headers, no
 * kernels, no helpers.  It is the plain definition of what the GPU path must
 * reproduce:
 *
 *     psi = U_L ... U_2 U_1 |0...0>,   then psi[x] for requested x and sum |psi|^2
 *
 * i.e. the Schroedinger approach of the paper (Sec. 2: evolve the full state
 * of a (sub)circuit by applying gates one at a time), with no gate
 * aggregation, no slicing and no index permutation.  Slicing (Sec. 2, "tensor
 * slicing"), aggregation into 2^k x 2^k blocks (Sec. 5) and diagonal
 * (hyperedge) folding (Sec. 2) all re-associate this same product exactly, so
 * the oracle does not implement any of them.
 *
 * Conventions: amplitude index little-endian (bit q of the index is qubit q);
 * a gate on qubits (q_0, ..., q_{k-1}) has matrix index c = sum_j b(q_j) 2^j.
 * Everything is complex128.  Parallelism (OpenMP) only splits independent
 * loop iterations; the arithmetic per amplitude is fixed.
 */
#include <complex.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double _Complex cplx;

#define ORC_MAXK 12

/* Thread count for the following calls (timing runs on one core). */
void orc_set_threads(int n)
{
#ifdef _OPENMP
    omp_set_num_threads(n > 0 ? n : 1);
#else
    (void)n;
#endif
}

int orc_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* psi <- e_0 (Sec. 2: every qubit starts in |0>). */
void orc_init_zero(cplx* psi, int n)
{
    const int64_t N = (int64_t)1 << n;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; ++i) psi[i] = 0.0;
    psi[0] = 1.0;
}

static int check_qubits(int n, int k, const int* q)
{
    if (n < 1 || n > 40 || k < 1 || k > ORC_MAXK || k > n) return -1;
    for (int j = 0; j < k; ++j) {
        if (q[j] < 0 || q[j] >= n) return -1;
        for (int l = 0; l < j; ++l)
            if (q[l] == q[j]) return -1;
    }
    return 0;
}

/*
 * Dense k-qubit gate (a 2^k x 2^k unitary acting on the listed qubits).
 * For every index i whose bits at the k qubits are zero, the 2^k amplitudes
 * x_c = psi[i + sum_j c_j 2^{q_j}] are replaced by y = M x.
 * M is row-major, M[r * 2^k + c].
 */
int orc_apply_dense(cplx* psi, int n, int k, const int* qubits, const cplx* m)
{
    if (check_qubits(n, k, qubits)) return -1;
    const int dim = 1 << k;
    int64_t off[1 << ORC_MAXK];
    for (int c = 0; c < dim; ++c) {
        int64_t o = 0;
        for (int j = 0; j < k; ++j)
            if ((c >> j) & 1) o += (int64_t)1 << qubits[j];
        off[c] = o;
    }
    /* qubit positions sorted ascending, to spread a group counter g over the
       n-k free bit positions */
    int sq[ORC_MAXK];
    for (int j = 0; j < k; ++j) sq[j] = qubits[j];
    for (int j = 1; j < k; ++j)
        for (int l = j; l > 0 && sq[l - 1] > sq[l]; --l) {
            int t = sq[l]; sq[l] = sq[l - 1]; sq[l - 1] = t;
        }
    const int64_t groups = (int64_t)1 << (n - k);
#pragma omp parallel
    {
        cplx* x = (cplx*)malloc(sizeof(cplx) * dim);
#pragma omp for schedule(static)
        for (int64_t g = 0; g < groups; ++g) {
            int64_t i = g;
            for (int j = 0; j < k; ++j) {          /* open a zero bit at sq[j] */
                int64_t low = i & (((int64_t)1 << sq[j]) - 1);
                i = ((i - low) << 1) | low;
            }
            for (int c = 0; c < dim; ++c) x[c] = psi[i + off[c]];
            for (int r = 0; r < dim; ++r) {
                cplx acc = 0.0;
                for (int c = 0; c < dim; ++c) acc += m[(int64_t)r * dim + c] * x[c];
                psi[i + off[r]] = acc;
            }
        }
        free(x);
    }
    return 0;
}

/*
 * Diagonal gate on m qubits (a hyperedge in the paper's hypergraph, Sec. 2):
 * psi[i] *= d[sum_j b_{q_j}(i) 2^j].
 */
int orc_apply_diag(cplx* psi, int n, int m, const int* qubits, const cplx* d)
{
    if (check_qubits(n, m, qubits)) return -1;
    const int64_t N = (int64_t)1 << n;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; ++i) {
        int idx = 0;
        for (int j = 0; j < m; ++j) idx |= (int)((i >> qubits[j]) & 1) << j;
        psi[i] *= d[idx];
    }
    return 0;
}

/*
 * Whole circuit: psi <- e_0, then every gate in list order.
 * arity[g] = number of qubits of gate g; qubits = all gates' qubit lists
 * concatenated; mats = all gates' matrices concatenated (row-major).
 */
int orc_simulate(cplx* psi, int n, int ngates, const int* arity, const int* qubits,
                 const cplx* mats)
{
    orc_init_zero(psi, n);
    int64_t qo = 0, mo = 0;
    for (int g = 0; g < ngates; ++g) {
        const int k = arity[g];
        if (orc_apply_dense(psi, n, k, qubits + qo, mats + mo)) return -1 - g;
        qo += k;
        mo += (int64_t)1 << (2 * k);
    }
    return 0;
}

/* Same, starting from the given state and applying gates [g0, g1). */
int orc_apply_gates(cplx* psi, int n, int g0, int g1, const int* arity, const int* qubits,
                    const cplx* mats)
{
    int64_t qo = 0, mo = 0;
    for (int g = 0; g < g1; ++g) {
        const int k = arity[g];
        if (g >= g0 && orc_apply_dense(psi, n, k, qubits + qo, mats + mo)) return -1 - g;
        qo += k;
        mo += (int64_t)1 << (2 * k);
    }
    return 0;
}

/* out[j] = psi[bits[j]] (bitstring bit q = qubit q). */
int orc_gather(const cplx* psi, int n, int64_t count, const uint64_t* bits, cplx* out)
{
    const uint64_t N = (uint64_t)1 << n;
    for (int64_t j = 0; j < count; ++j) {
        if (bits[j] >= N) return -1;
        out[j] = psi[bits[j]];
    }
    return 0;
}

/* Pairwise (recursive halving) sum of |psi|^2 over a power-of-two range. */
static double pairwise_norm(const cplx* a, int64_t len)
{
    if (len <= 8) {
        double s = 0.0;
        for (int64_t i = 0; i < len; ++i) s += creal(a[i]) * creal(a[i]) + cimag(a[i]) * cimag(a[i]);
        return s;
    }
    const int64_t h = len / 2;
    return pairwise_norm(a, h) + pairwise_norm(a + h, len - h);
}

double orc_norm(const cplx* psi, int n)
{
    const int64_t N = (int64_t)1 << n;
    const int64_t chunk = N < ((int64_t)1 << 16) ? N : ((int64_t)1 << 16);
    const int64_t nch = N / chunk;
    double* part = (double*)malloc(sizeof(double) * nch);
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < nch; ++c) part[c] = pairwise_norm(psi + c * chunk, chunk);
    /* pairwise over chunk sums: same tree as a single recursive sum */
    for (int64_t w = nch; w > 1; w /= 2)
        for (int64_t c = 0; c < w / 2; ++c) part[c] = part[2 * c] + part[2 * c + 1];
    const double s = part[0];
    free(part);
    return s;
}
