// dq_internal.h -- tables shared by the host runtime (runtime.cpp) and the
// gfx950 kernels (kernels.hip).  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dq {

// ---------------------------------------------------------------- gates
// Internal op codes equal the public dq_op values.
enum : int32_t {
    OP_H = 0, OP_X, OP_Y, OP_Z, OP_RX, OP_RY, OP_RZ, OP_CNOT, OP_CZ, OP_SWAP, OP_CP, OP_RZZ,
    OP_UNITARY
};
enum : int32_t { SRC_NONE = 0, SRC_PARAM = 1, SRC_DATA = 2 };

// Generator of a differentiable gate, as seen by the adjoint sweep:
//   GEN_X/Y/Z (one wire), GEN_ZZ (two wires) for exp(-i t G / 2)  -> dE/dt = Im<l|G|p>
//   GEN_P11 (|11><11| on two wires) for CP(t) = exp(i t P11)         -> dE/dt = -2 Im<l|P11|p>
enum : int32_t { GEN_NONE = 0, GEN_X = 1, GEN_Y = 2, GEN_Z = 3, GEN_ZZ = 4, GEN_P11 = 5 };

struct DGate {                 // device copy of one gate
    int32_t op, nq;
    int32_t bits[5];           // physical bit positions (n-1-wire); bits[0] = matrix MSB
    int32_t src;
    int64_t idx;
    double scale;
    int64_t mat_off;           // UNITARY: offset (complex) into the fixed-matrix table
};

// A matrix slot: the product F[nf-1] ... F[0] of gate matrices (F[0] acts
// first), optionally conjugate-transposed, formed in double per sample and
// rounded once into the per-sample matrix block at `off`.
enum : int32_t { SLOT_MAXF = 8 };
struct DSlot {
    int32_t dim;               // 2, 4, 8, 16 or 32
    int32_t nf;
    int32_t f[SLOT_MAXF];      // gate indices
    int32_t dagger;
    int32_t pad;
    int64_t off;               // complex offset inside one sample's matrix block
};

// A fused dense block: the product, in gate order, of nf one- and two-qubit
// gates (factor table entries foff..foff+nf-1) that act inside the K block
// bits bb[0..K-1] (bb[0] = most significant bit of the block index).
struct DBlock {
    int32_t k;
    int32_t nf;
    int32_t foff;
    int32_t bb[5];
    int64_t off;               // complex offset inside one sample's matrix block
};

// ---------------------------------------------------------------- tile passes
// Tile-local bit q: 0..5 = lane bits, 6..6+R-1 = register bits.  Lane bits 0..2
// are physical bits 0..2 in every pass (each group of 8 lanes reads 8
// consecutive amplitudes); lane bits 3..5 are physical lbits[0..2] and
// register bit q is physical rbits[q-6], chosen per pass.
enum : int32_t {
    TK_1Q = 0,      // dense 2x2 on q0
    TK_1QDIAG = 1,  // diagonal 2x2 on q0 (entries m00, m11 of the slot)
    TK_CNOT = 2,    // control q0, target q1
    TK_CZ = 3,      // q0, q1
    TK_2QDIAG = 4,  // diagonal 4x4 on (q0 = msb, q1) (entries 0, 5, 10, 15 of the slot)
    TK_SWAP = 5,    // exchange q0 and q1
    TK_1QREAL = 6,  // real 2x2 on q0 (real parts of the slot)
    TK_1QRX = 7     // [[c, i s], [i s, c]] on q0 (c = Re m00, s = Im m01)
};

struct TOp {
    int32_t kind;
    int32_t q0, q1;
    int32_t gen;       // adjoint: generator whose expectation is accumulated before un-applying
    int32_t slot;      // complex offset of the matrix inside one sample's block
    int32_t lslot;     // adjoint: accumulator index inside the pass, -1 none
};

enum : int32_t { MAX_TILE_R = 6, MAX_LSLOTS = 64 };

// One circuit's tile pass inside a multi-circuit launch.  Offsets: st_off in
// amplitudes from the packed state base; lam_off, mats_off, part_off in bytes
// from the workspace base.  unit_begin: first work unit of this entry (units:
// tiles in the forward, waves in the adjoint).
struct MultiEntry {
    int64_t st_off, lam_off, mats_off, part_off, unit_begin;
    const TOp *ops;
    const int32_t *lsg;
    int32_t n, nops, nls, wps, ngrad;
    int32_t rbits[MAX_TILE_R];
    int32_t lbits[3];
    int32_t tbits[MAX_TILE_R + 3];
};

// ---------------------------------------------------------------- observables
// Terms grouped by X mask (physical bits).  With w = coef * i^{nY} (complex,
// nY = number of Y letters) and S = sum_j (-1)^{|j & z|} conj(psi_{j^x}) psi_j,
// a term contributes Re(w S) = wr Re(S) - wi Im(S) to its observable.
struct DTerm {
    uint64_t zmask;
    double wr, wi;             // coef * i^{nY}
    int32_t obs;
    int32_t pad;
};
struct DGroup {
    uint64_t xmask;
    int32_t t0, t1;            // term range
};

}  // namespace dq

// ---------------------------------------------------------------- launchers
// Host-side entry points of kernels.hip, called by runtime.cpp.  `dbl`
// selects complex128 (1) or complex64 (0).  All launches are asynchronous
// on `stream`; they return the hipGetLastError() of the launch.
namespace dq {

struct TileArgs {
    void *st;                  // state [B][2^n]
    void *lam;                 // adjoint state (adjoint passes only)
    int32_t n, R;
    int32_t rbits[MAX_TILE_R]; // physical bits of the register bits
    int32_t lbits[3];          // physical bits of lane bits 3..5
    int32_t tbits[MAX_TILE_R + 3];  // lbits and rbits together, ascending
    int64_t batch;
    const TOp *ops;
    int32_t nops, nlslots;
    const void *mats;          // per-sample matrix blocks
    int64_t mstride;           // complex elements between samples' blocks (0 = shared)
    double *partial;           // adjoint: [B][wps][ngrad]
    const int32_t *lslot_gslot;// adjoint: global gradient index of each local slot
    int32_t wps, ngrad;
};

hipError_t launch_prepare(int dbl, const DGate *gates, const void *fixed, const DSlot *slots,
                          int32_t nslots, const double *params, int64_t pstride, const double *data,
                          int64_t dstride, void *mats, int64_t block, int64_t bm, hipStream_t s);
hipError_t launch_prepare_blocks(int dbl, const DGate *gates, const void *fixed, const DBlock *blocks,
                                 int32_t nblocks, const int32_t *factors, const double *params, int64_t pstride,
                                 const double *data, int64_t dstride, void *mats, int64_t block, int64_t bm,
                                 hipStream_t s);
hipError_t launch_init_zero(int dbl, void *st, int32_t n, int64_t batch, hipStream_t s);
hipError_t launch_init_copy(int dbl, void *st, const void *init, int32_t n, int64_t batch, hipStream_t s);
hipError_t launch_init_product(int dbl, void *st, int32_t n, int64_t batch, const void *mats,
                               int64_t mstride, const int64_t *fold_off, hipStream_t s);
hipError_t launch_copy(int dbl, void *dst, const void *src, int64_t count, hipStream_t s);
hipError_t launch_gate1(int dbl, void *st, int32_t n, int64_t batch, int32_t bit, const void *mats,
                        int64_t mstride, int64_t off, hipStream_t s);
hipError_t launch_cnot(int dbl, void *st, int32_t n, int64_t batch, int32_t cbit, int32_t tbit, hipStream_t s);
hipError_t launch_cz(int dbl, void *st, int32_t n, int64_t batch, int32_t abit, int32_t bbit, hipStream_t s);
hipError_t launch_gatek(int dbl, void *st, int32_t n, int64_t batch, int32_t k, const int32_t *bits,
                        const void *mats, int64_t mstride, int64_t off, hipStream_t s);
// dense 2^k x 2^k block (k = 4, 5) on the matrix cores; needs n >= k + 5
// (complex64) or n >= k + 4 (complex128)
hipError_t launch_dense(int dbl, void *st, int32_t n, int64_t batch, int32_t k, const int32_t *bits, const void *mats,
                        int64_t mstride, int64_t off, hipStream_t s);
hipError_t launch_tile_fwd(int dbl, const TileArgs &a, hipStream_t s);
hipError_t launch_tile_adj(int dbl, const TileArgs &a, hipStream_t s);
// resident single-wave workgroups of the adjoint tile kernel on the current device
int tile_adj_capacity(int dbl, int R);
// multi-circuit tile passes: entries describe one depth of every circuit
hipError_t launch_tile_fwd_multi(int dbl, int R, void *st, const void *ws, const MultiEntry *ents, int32_t nent,
                                 int64_t units, hipStream_t s);
hipError_t launch_tile_adj_multi(int dbl, int R, void *st, void *ws, const MultiEntry *ents, int32_t nent,
                                 int64_t units, int32_t max_nls, hipStream_t s);
hipError_t launch_grad_gate(int dbl, const void *psi, const void *lam, int32_t n, int64_t batch, int32_t gen,
                            int32_t bit0, int32_t bit1, double *partial, int32_t wps, int32_t ngrad,
                            int32_t gslot, hipStream_t s);
hipError_t launch_grad_final(const double *partial, int64_t batch, int32_t wps, int32_t ngrad,
                             const int64_t *csr_off, const int32_t *csr_g, const double *csr_f,
                             int64_t nout, int32_t per_sample, double *out, hipStream_t s);
hipError_t launch_expval(int dbl, const void *st, int32_t n, int64_t batch, const DGroup *groups,
                         int32_t ngroups, const DTerm *terms, int32_t nterms, int32_t nobs,
                         double *partial, int32_t eb, double *out, hipStream_t s);
hipError_t launch_lambda(int dbl, const void *psi, void *lam, int32_t n, int64_t batch, const DGroup *groups,
                         int32_t ngroups, const DTerm *terms, const double *grad_out, int32_t nobs,
                         hipStream_t s);

}  // namespace dq
