// dq_internal.h -- tables shared by the host runtime (runtime.cpp) and the
// gfx950 kernels (kernels.hip).  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "tile_dev.h"

namespace dq {

// ---------------------------------------------------------------- gates
// Internal op codes equal the public dq_op values.
enum : int32_t {
    OP_H = 0, OP_X, OP_Y, OP_Z, OP_RX, OP_RY, OP_RZ, OP_CNOT, OP_CZ, OP_SWAP, OP_CP, OP_RZZ,
    OP_UNITARY,
    OP_RXX, OP_RYY,  // plan input only: expanded into basis changes around an RZZ
    OP_U3,           // plan input only: phase(lambda), RY(theta), phase(phi)
    OP_CRX, OP_CRY, OP_CRZ,   // plan input only: two half-angle rotations around two CNOT / CZ
    OP_PHASE = 32    // internal: diag(1, e^{i t}) = e^{i t/2} RZ(t); the angle of U3's phi and lambda
};
enum : int32_t { SRC_NONE = 0, SRC_PARAM = 1, SRC_DATA = 2 };

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

// One circuit's tile pass inside a multi-circuit launch.  Offsets: st_off in
// amplitudes from the packed state base; lam_off, mats_off, part_off in bytes
// from the workspace base.  unit_begin: first work unit of this entry (units:
// tiles in the forward, waves in the adjoint).
struct MultiEntry {
    int64_t st_off, lam_off, mats_off, part_off, unit_begin;
    const TOp *ops;
    const int32_t *lsg;
    int32_t n, nops, nls, wps, ngrad;
    int32_t nt;                // 1: non-temporal loads and stores (see TileArgs)
    int32_t rbits[MAX_TILE_R];
    int32_t lbits[3];
    int32_t tbits[MAX_TILE_R + 3];
};

// The per-circuit steps of an uneven batch that surround the tile passes,
// one launch each over all circuits: matrix preparation, start states,
// expectations, the adjoint seed and the final gradient sums.  Offsets:
// st_off in amplitudes from the packed state base, *_off in bytes from the
// workspace base except par_off / out_off (elements of the packed
// parameter / output arrays).
struct DGroup;
struct DTerm;
struct MPrep {
    const DGate *gates;
    const double2 *fixed;
    const DSlot *slots;        // the program's slot range
    int32_t nslots, pad;
    int64_t par_off, mats_off;
};
struct MInit {
    int64_t st_off, mats_off;
    const int64_t *fold;       // per physical bit: folded slot offset, -1 none
    int32_t n, has_fold;
};
struct MExp {
    int64_t st_off, lam_off, part_off;
    int64_t unit_begin;        // first expectation block of this circuit
    int64_t amp_begin;         // first amplitude of this circuit in the adjoint-seed range
    int64_t out_off;
    const DGroup *groups;
    const DTerm *terms;
    int32_t n, ngroups, nterms, nobs, eb, pad;
};
struct MGrad {
    int64_t part_off, par_off, unit_begin;
    const int64_t *poff;       // parameter -> gradient slots (CSR) with chain factors
    const int32_t *pg;
    const double *pf;
    int32_t wps, ngrad;
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
// Terms whose X mask is one bit, taken in register tiles of 2048 amplitudes:
// lane l = physical bits 0..5, register k = the five bits rb (ascending, all
// >= 6); one read of the state serves every such term whose X bit is a tile
// bit.  pos: the X bit's place in the tile (0..5 lane bit, 6 + r register
// bit r).
constexpr int XT_MAX = 12;     // terms per tile set
struct XSet {
    int32_t rb[5];
    int32_t x0, x1;            // XTerm range (at most XT_MAX)
};
struct XTerm {
    int32_t t, pos;
};

}  // namespace dq

// ---------------------------------------------------------------- launchers
// Host-side entry points of kernels.hip, called by runtime.cpp.  `dbl`
// selects complex128 (1) or complex64 (0).  All launches are asynchronous
// on `stream`; they return the hipGetLastError() of the launch.
namespace dq {

hipError_t launch_prepare(int dbl, const DGate *gates, const void *fixed, const DSlot *slots,
                          int32_t nslots, const double *params, int64_t pstride, const double *data,
                          int64_t dstride, void *mats, int64_t block, int64_t bm, hipStream_t s);
hipError_t launch_prepare_blocks(int dbl, const DGate *gates, const void *fixed, const DBlock *blocks,
                                 int32_t nblocks, const int32_t *factors, const double *params, int64_t pstride,
                                 const double *data, int64_t dstride, void *mats, int64_t block, int64_t bm,
                                 hipStream_t s);
hipError_t launch_init_zero(int dbl, void *st, int32_t n, int64_t batch, hipStream_t s);
hipError_t launch_init_copy(int dbl, void *st, const void *init, int32_t n, int64_t batch, hipStream_t s);
// mdbl: the folded matrices are complex128 (complex128 states, or complex64
// states of a plan with float64 arithmetic)
hipError_t launch_init_product(int dbl, int mdbl, void *st, int32_t n, int64_t batch, const void *mats,
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
// per-precision entry points of the interpreted tile passes (tiles.hip)
hipError_t tile_fwd_f32(const TileArgs &a, hipStream_t s);
hipError_t tile_fwd_f64(const TileArgs &a, hipStream_t s);
hipError_t tile_adj_f32(const TileArgs &a, hipStream_t s);
hipError_t tile_adj_f64(const TileArgs &a, hipStream_t s);
int tile_adj_capacity_f32(int R);
int tile_adj_capacity_f64(int R);
hipError_t tile_fwd_multi_f32(int R, void *st, const void *ws, const MultiEntry *e, int32_t n, int64_t units,
                              hipStream_t s);
hipError_t tile_fwd_multi_f64(int R, void *st, const void *ws, const MultiEntry *e, int32_t n, int64_t units,
                              hipStream_t s);
hipError_t tile_adj_multi_f32(int R, void *st, void *ws, const MultiEntry *e, int32_t n, int64_t units, size_t lds,
                              hipStream_t s);
hipError_t tile_adj_multi_f64(int R, void *st, void *ws, const MultiEntry *e, int32_t n, int64_t units, size_t lds,
                              hipStream_t s);
// passes compiled at plan time (jit.cpp): jit_key names the kernel of a
// source body (a hash that also covers tile_dev.h and the compiler options);
// jit_load returns, for the current device, the kernels of the given names
// and full sources, compiling what neither the process nor the disk cache
// holds; jit_launch runs one on a tile argument block.
std::string jit_key(const std::string &body);
bool jit_load(const std::vector<std::string> &names, const std::vector<std::string> &srcs,
              std::vector<hipFunction_t> &out, std::string &err);
hipError_t jit_launch(hipFunction_t f, const std::string &name, const TileArgs &a, bool adj, hipStream_t s);
// resident single-wave workgroups of a compiled pass with `lds` bytes of
// dynamic LDS on the current device (0 if unknown)
int jit_resident(hipFunction_t f, size_t lds);
hipError_t launch_tile_fwd(int dbl, const TileArgs &a, hipStream_t s);
hipError_t launch_tile_adj(int dbl, const TileArgs &a, hipStream_t s);
// resident single-wave workgroups of the adjoint tile kernel on the current device
int tile_adj_capacity(int dbl, int R);
// multi-circuit tile passes: entries describe one depth of every circuit
// tile shapes the multi-circuit kernels are instantiated for (tiles.hip)
inline bool multi_fwd_has(int dbl, int R) { return R == 3 || R == 4 || (R == 5 && !dbl); }
inline bool multi_adj_has(int dbl, int R) { return R == 3 || (R == 4 && !dbl); }
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
// uneven batches (kernels.hip): one launch per step over all circuits
hipError_t launch_prepare_multi(int dbl, const MPrep *ents, int32_t nent, int32_t max_slots, const double *params,
                                void *ws, hipStream_t s);
hipError_t launch_init_multi(int dbl, void *st, const void *ws, const MInit *ents, int32_t nent, int32_t max_n,
                             hipStream_t s);
// units: sum of the entries' eb; writes out[out_off + o] for every circuit
// max_group: the most terms any X-mask group of the batched circuits holds
hipError_t launch_expval_multi(int dbl, const void *st, void *ws, const MExp *ents, int32_t nent, int64_t units,
                               int32_t max_group, double *out, hipStream_t s);
// total: sum of the circuits' amplitudes (amp_begin ranges)
hipError_t launch_lambda_multi(int dbl, const void *st, void *ws, const MExp *ents, int32_t nent, int64_t total,
                               const double *gout, hipStream_t s);
// total: sum of the circuits' parameter counts (unit ranges)
hipError_t launch_grad_final_multi(const void *ws, const MGrad *ents, int32_t nent, int64_t total, double *out,
                                   hipStream_t s);
// Hessian by shifted adjoints (kernels.hip): angle rows of 2 mc shifted
// circuits, the observable weights broadcast to every row, and the
// deterministic accumulation of H[P][P] from the rows' gradients (the first
// chunk, c0 = 0, overwrites H)
hipError_t launch_hess_rows(const double *params, const int32_t *occ_param, const double *occ_scale, int64_t K,
                            int64_t c0, int64_t mc, double *rows, hipStream_t s);
hipError_t launch_bcast_rows(const double *w, int32_t nobs, int64_t rows, double *out, hipStream_t s);
hipError_t launch_hess_accum(const double *G, int64_t K, int64_t c0, int64_t mc, const int64_t *poff,
                             const int32_t *pocc, const double *occ_scale, int64_t P, double *H, hipStream_t s);
// observables at most the diagonal expectation kernel sums at once
constexpr int ZD_MAXOBS = 8;
// blocks of the diagonal expectation kernel per sample (4 waves of
// 2048-amplitude tiles each), for n >= 11
inline int zdiag_blocks(int n) {
    if (n < 11) return 1;
    const int64_t q = (int64_t(1) << (n - 11)) / 4;
    return (int)(q < 1 ? 1 : (q < 1024 ? q : 1024));
}
// expectations; terms dt0..dt1 (group 0, X-free) go through the diagonal
// kernel into dpart ([batch][blocks][nobs] doubles) when dt0 < dt1
// marginal probabilities (kernels.hip): measured wires' physical bits in
// wire order (pb) and ascending (asc)
constexpr int PROB_MAXW = 12;
struct ProbArgs {
    int32_t n, k;
    int32_t pb[PROB_MAXW];
    int32_t asc[PROB_MAXW];
};
// amplitudes one block of k_probs_part sums (256 threads x 16)
constexpr int64_t PROB_CHUNK = 4096;
hipError_t launch_probs(int dbl, const void *st, int64_t batch, const ProbArgs &a, double *partial, int64_t bpo,
                        double *out, hipStream_t s);
hipError_t launch_sample(const double *p, int64_t batch, int32_t nout, const double *u, int32_t shots, int64_t *out,
                         hipStream_t s);
// Groups [0, ngroups) by the pair kernels (the X-free group 0 by k_zdiag
// when dt0 < dt1); the one-bit-X terms of the nxs tile sets (host array xs,
// term lists at device xt) by the tile kernels (complex64 only).
hipError_t launch_expval(int dbl, const void *st, int32_t n, int64_t batch, const DGroup *groups, int32_t ngroups,
                         const DTerm *terms, int32_t nterms, int32_t nobs, double *partial, int32_t eb, double *out,
                         int32_t dt0, int32_t dt1, double *dpart, const XSet *xs, int32_t nxs, const XTerm *xt,
                         hipStream_t s);
hipError_t launch_lambda(int dbl, const void *psi, void *lam, int32_t n, int64_t batch, const DGroup *groups,
                         int32_t ngroups, const DTerm *terms, const double *grad_out, int32_t nobs, int32_t dt0, int32_t dt1,
                         const XSet *xs, int32_t nxs, const XTerm *xt, hipStream_t s);

}  // namespace dq
