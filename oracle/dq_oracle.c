/*
 * dq_oracle.c -- TEST INFRASTRUCTURE, not part of the product.
 *
 * A plain, slow, complex128 state-vector simulator written from the paper's
 * definitions.  Only the tests, the smoke check and the bench's CPU-baseline
 * leg may load it.  It shares no code, header, table or helper with the HIP
 * library: the two meet only through the seeded inputs of the `workloads`
 * module.
 *
 * What it computes (paper section 4.1, "Background"):
 *   pure-state evolution  |psi_M> = U_M ... U_1 |psi_0>         (eq. of 4.1)
 *   expectation values    <psi_M| P |psi_M>  for Pauli strings P (4.2, API)
 * Conventions (readings of the paper; each is pinned by a test):
 *   - flat index j = sum_w b_w 2^(n-1-w): wire 0 is the most significant bit,
 *     the first factor of the ket (tensor form of section 7.1); pinned by the
 *     QFT listing equalling the unitary DFT;
 *   - RX/RY/RZ(t) = exp(-i t P/2), RZZ(t) = exp(-i t Z(x)Z/2), and likewise
 *     RXX(t) = exp(-i t X(x)X/2), RYY(t) = exp(-i t Y(x)Y/2);
 *   - CP(phi) = diag(1,1,1,e^{i phi}); CNOT flips the target where the control
 *     is 1; CZ negates |11>; SWAP exchanges the two wires;
 *   - U3(theta, phi, lambda) = [[cos(theta/2), -e^{i lambda} sin(theta/2)],
 *     [e^{i phi} sin(theta/2), e^{i (phi + lambda)} cos(theta/2)]] (the
 *     general one-qubit gate of the QResNet listing, section 4.3);
 *   - CRX/CRY/CRZ(theta) on (control, target) = |0><0| (x) I + |1><1| (x)
 *     R(theta) with R = RX/RY/RZ (the controlled rotations of the QCNN
 *     listing and the controlled encoding of the QResNet listing);
 *   - a k-qubit matrix acts on an ordered wire list whose first wire is the
 *     most significant bit of the matrix index.
 *
 * Every loop is the textbook one: for each index whose target bits are all
 * zero, gather the 2^k amplitudes, multiply by the matrix, scatter.
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

enum {
    ORC_H = 0, ORC_X, ORC_Y, ORC_Z, ORC_RX, ORC_RY, ORC_RZ,
    ORC_CNOT, ORC_CZ, ORC_SWAP, ORC_CP, ORC_RZZ, ORC_UNITARY, ORC_RXX, ORC_RYY,
    ORC_U3, ORC_CRX, ORC_CRY, ORC_CRZ
};

/* Matrix of a named gate at angle theta, row-major, into U (size dim*dim).
 * Returns the number of qubits (1 or 2), or -1 for an unknown op. */
int orc_gate_matrix(int op, double theta, double *U_interleaved)
{
    cplx U[16];
    int k;
    double c = cos(theta / 2.0), s = sin(theta / 2.0);
    for (int i = 0; i < 16; ++i) U[i] = 0.0;
    switch (op) {
    case ORC_H:
        k = 1;
        U[0] = 1.0 / sqrt(2.0); U[1] = 1.0 / sqrt(2.0);
        U[2] = 1.0 / sqrt(2.0); U[3] = -1.0 / sqrt(2.0);
        break;
    case ORC_X:
        k = 1; U[1] = 1.0; U[2] = 1.0;
        break;
    case ORC_Y:
        k = 1; U[1] = -I; U[2] = I;
        break;
    case ORC_Z:
        k = 1; U[0] = 1.0; U[3] = -1.0;
        break;
    case ORC_RX:   /* exp(-i theta X / 2) = c I - i s X */
        k = 1; U[0] = c; U[1] = -I * s; U[2] = -I * s; U[3] = c;
        break;
    case ORC_RY:   /* exp(-i theta Y / 2) = c I - i s Y */
        k = 1; U[0] = c; U[1] = -s; U[2] = s; U[3] = c;
        break;
    case ORC_RZ:   /* exp(-i theta Z / 2) */
        k = 1; U[0] = cexp(-I * theta / 2.0); U[3] = cexp(I * theta / 2.0);
        break;
    case ORC_CNOT: /* basis order |control target> */
        k = 2; U[0 * 4 + 0] = 1.0; U[1 * 4 + 1] = 1.0; U[2 * 4 + 3] = 1.0; U[3 * 4 + 2] = 1.0;
        break;
    case ORC_CZ:
        k = 2; U[0] = 1.0; U[5] = 1.0; U[10] = 1.0; U[15] = -1.0;
        break;
    case ORC_SWAP:
        k = 2; U[0 * 4 + 0] = 1.0; U[1 * 4 + 2] = 1.0; U[2 * 4 + 1] = 1.0; U[3 * 4 + 3] = 1.0;
        break;
    case ORC_CP:
        k = 2; U[0] = 1.0; U[5] = 1.0; U[10] = 1.0; U[15] = cexp(I * theta);
        break;
    case ORC_RZZ:  /* exp(-i theta Z(x)Z / 2): eigenvalue of ZZ is +1 on |00>,|11> */
        k = 2;
        U[0] = cexp(-I * theta / 2.0); U[5] = cexp(I * theta / 2.0);
        U[10] = cexp(I * theta / 2.0); U[15] = cexp(-I * theta / 2.0);
        break;
    case ORC_RXX:  /* c I - i s X(x)X: X(x)X exchanges |00>,|11> and |01>,|10> */
        k = 2;
        U[0] = c; U[5] = c; U[10] = c; U[15] = c;
        U[0 * 4 + 3] = -I * s; U[1 * 4 + 2] = -I * s; U[2 * 4 + 1] = -I * s; U[3 * 4 + 0] = -I * s;
        break;
    case ORC_RYY:  /* c I - i s Y(x)Y: Y(x)Y = -1 on the |00>,|11> corners, +1 on |01>,|10> */
        k = 2;
        U[0] = c; U[5] = c; U[10] = c; U[15] = c;
        U[0 * 4 + 3] = I * s; U[1 * 4 + 2] = -I * s; U[2 * 4 + 1] = -I * s; U[3 * 4 + 0] = I * s;
        break;
    case ORC_CRX: case ORC_CRY: case ORC_CRZ: {
        /* identity on the control-0 block, the rotation on the control-1 block */
        double R[8];
        orc_gate_matrix(op == ORC_CRX ? ORC_RX : (op == ORC_CRY ? ORC_RY : ORC_RZ), theta, R);
        k = 2;
        U[0 * 4 + 0] = 1.0;
        U[1 * 4 + 1] = 1.0;
        U[2 * 4 + 2] = R[0] + I * R[1];
        U[2 * 4 + 3] = R[2] + I * R[3];
        U[3 * 4 + 2] = R[4] + I * R[5];
        U[3 * 4 + 3] = R[6] + I * R[7];
        break;
    }
    default:
        return -1;
    }
    int dim = 1 << k;
    for (int i = 0; i < dim * dim; ++i) {
        U_interleaved[2 * i] = creal(U[i]);
        U_interleaved[2 * i + 1] = cimag(U[i]);
    }
    return k;
}

/* U3(theta, phi, lambda), row-major, into U (4 complex entries). */
void orc_u3_matrix(double theta, double phi, double lambda, double *U_interleaved)
{
    double ch = cos(theta / 2.0);
    double sh = sin(theta / 2.0);
    cplx U[4];
    U[0] = ch;
    U[1] = -cexp(I * lambda) * sh;
    U[2] = cexp(I * phi) * sh;
    U[3] = cexp(I * (phi + lambda)) * ch;
    for (int i = 0; i < 4; ++i) {
        U_interleaved[2 * i] = creal(U[i]);
        U_interleaved[2 * i + 1] = cimag(U[i]);
    }
}

/* Apply a k-qubit matrix U (dim x dim, row-major, interleaved re/im) to the
 * ordered wires[0..k-1] of an n-qubit state.  wires[0] is the most
 * significant bit of U's index; wire w sits at bit n-1-w of the flat index. */
void orc_apply(int n, double *psi_interleaved, int k, const int *wires, const double *U_interleaved)
{
    cplx *psi = (cplx *)psi_interleaved;
    const cplx *U = (const cplx *)U_interleaved;
    long long N = 1LL << n;
    int dim = 1 << k;
    long long target_mask = 0;
    long long *off = malloc(sizeof(long long) * dim);
    cplx *in = malloc(sizeof(cplx) * dim);
    cplx *out = malloc(sizeof(cplx) * dim);

    for (int t = 0; t < k; ++t)
        target_mask |= 1LL << (n - 1 - wires[t]);
    /* offset of sub-index a: bit (k-1-t) of a belongs to wires[t] */
    for (int a = 0; a < dim; ++a) {
        off[a] = 0;
        for (int t = 0; t < k; ++t)
            if ((a >> (k - 1 - t)) & 1)
                off[a] += 1LL << (n - 1 - wires[t]);
    }
    for (long long j = 0; j < N; ++j) {
        if (j & target_mask)
            continue;
        for (int a = 0; a < dim; ++a)
            in[a] = psi[j + off[a]];
        for (int r = 0; r < dim; ++r) {
            cplx acc = 0.0;
            for (int c = 0; c < dim; ++c)
                acc += U[r * dim + c] * in[c];
            out[r] = acc;
        }
        for (int a = 0; a < dim; ++a)
            psi[j + off[a]] = out[a];
    }
    free(off);
    free(in);
    free(out);
}

/* Run a gate list on psi (caller initialises psi, normally to |0...0>).
 * ops[g], nq[g], wires[5*g .. 5*g+nq-1], angles theta[3*g .. 3*g+2] (one
 * angle in theta[3*g] for every gate but U3, which takes theta, phi,
 * lambda); unitary gates consume their matrices from `dense` in order of
 * appearance.  Returns 0, or -1 on an unknown op. */
int orc_run(int n, double *psi, int ngates, const int *ops, const int *nq, const int *wires,
            const double *theta, const double *dense)
{
    double U[2 * 16];
    for (int g = 0; g < ngates; ++g) {
        if (ops[g] == ORC_UNITARY) {
            int dim = 1 << nq[g];
            orc_apply(n, psi, nq[g], wires + 5 * g, dense);
            dense += 2 * dim * dim;
            continue;
        }
        int k = 1;
        if (ops[g] == ORC_U3)
            orc_u3_matrix(theta[3 * g], theta[3 * g + 1], theta[3 * g + 2], U);
        else
            k = orc_gate_matrix(ops[g], theta[3 * g], U);
        if (k < 0 || k != nq[g])
            return -1;
        orc_apply(n, psi, k, wires + 5 * g, U);
    }
    return 0;
}

/* <psi| P |psi> for the Pauli string letters[0..n-1] over {I,X,Y,Z}
 * (letters[w] acts on wire w): copy psi, apply every letter as an ordinary
 * one-qubit gate, take the complex inner product.  The real part is
 * returned, the imaginary part stored in *imag (it must vanish: P is
 * Hermitian). */
double orc_pauli_expval(int n, const double *psi_interleaved, const char *letters, double *imag)
{
    long long N = 1LL << n;
    const cplx *psi = (const cplx *)psi_interleaved;
    cplx *phi = malloc(sizeof(cplx) * N);
    double M[8];
    memcpy(phi, psi, sizeof(cplx) * N);
    for (int w = 0; w < n; ++w) {
        int op;
        switch (letters[w]) {
        case 'I': continue;
        case 'X': op = ORC_X; break;
        case 'Y': op = ORC_Y; break;
        case 'Z': op = ORC_Z; break;
        default: free(phi); *imag = NAN; return NAN;
        }
        orc_gate_matrix(op, 0.0, M);
        orc_apply(n, (double *)phi, 1, &w, M);
    }
    cplx acc = 0.0;
    for (long long j = 0; j < N; ++j)
        acc += conj(psi[j]) * phi[j];
    free(phi);
    *imag = cimag(acc);
    return creal(acc);
}

/* Probability that wire `w` reads 0: sum of |psi_j|^2 over j with that bit
 * clear (the exact marginal behind measure(with_prob=True)). */
double orc_prob_zero(int n, const double *psi_interleaved, int w)
{
    const cplx *psi = (const cplx *)psi_interleaved;
    long long N = 1LL << n, bit = 1LL << (n - 1 - w);
    double p = 0.0;
    for (long long j = 0; j < N; ++j)
        if (!(j & bit))
            p += creal(psi[j]) * creal(psi[j]) + cimag(psi[j]) * cimag(psi[j]);
    return p;
}
