// kernels.hip -- gfx950 (CDNA4) kernels of libdq.
//
// State vectors are [batch][2^n] interleaved complex (float2 / double2);
// physical bit s of the flat index belongs to wire n-1-s (wire 0 = MSB).
//
// Kernel families
//   prepare      gate matrices per sample: sincos of the angle in double,
//                products of fused one-qubit factors, daggers; rounded once
//   init_*       |0..0>, broadcast copy, or a product state (leading one-qubit
//                gates of every wire folded into the first write)
//   gate1/cnot/cz/gatek   one launch per gate: the plain path
//   tile_fwd     register tiles: one wave64 owns 2^(6+R) amplitudes, lanes span
//                physical bits 0..5 (every load/store instruction moves 64
//                consecutive amplitudes), R register-resident bits are chosen
//                per pass; gates on register bits are in-register butterflies,
//                gates on lane bits use cross-lane shuffles.  Many gates per
//                HBM round trip.
//   tile_adj     the same tiles over (psi, lambda) for the adjoint sweep,
//                accumulating Im<lambda|G|psi> per differentiable gate
//   expval/lambda/grad_*   Pauli-sum reductions, H psi for the adjoint seed,
//                per-gate gradient reductions and the deterministic final sum
#include "dq_internal.h"

#include <type_traits>
#include <utility>

namespace dq {
namespace {


inline unsigned grid_for(int64_t work, int block, int64_t cap = 1 << 16) {
    int64_t g = (work + block - 1) / block;
    if (g > cap) g = cap;
    if (g < 1) g = 1;
    return (unsigned)g;
}

// ============================================================ prepare
__device__ void gate_matrix(const DGate &g, double th, const double2 *fixed, double2 *U) {
    const int dim = 1 << g.nq;
    for (int i = 0; i < dim * dim; ++i) U[i] = double2{0.0, 0.0};
    double s, c;
    sincos(0.5 * th, &s, &c);
    switch (g.op) {
    case OP_H: {
        const double r = 0.70710678118654752440;
        U[0] = {r, 0}; U[1] = {r, 0}; U[2] = {r, 0}; U[3] = {-r, 0};
        break;
    }
    case OP_X: U[1] = {1, 0}; U[2] = {1, 0}; break;
    case OP_Y: U[1] = {0, -1}; U[2] = {0, 1}; break;
    case OP_Z: U[0] = {1, 0}; U[3] = {-1, 0}; break;
    case OP_RX: U[0] = {c, 0}; U[1] = {0, -s}; U[2] = {0, -s}; U[3] = {c, 0}; break;
    case OP_RY: U[0] = {c, 0}; U[1] = {-s, 0}; U[2] = {s, 0}; U[3] = {c, 0}; break;
    case OP_RZ: U[0] = {c, -s}; U[3] = {c, s}; break;
    case OP_PHASE: {
        double sp, cp;
        sincos(th, &sp, &cp);
        U[0] = {1, 0}; U[3] = {cp, sp};
        break;
    }
    case OP_CNOT: U[0] = {1, 0}; U[5] = {1, 0}; U[11] = {1, 0}; U[14] = {1, 0}; break;
    case OP_CZ: U[0] = {1, 0}; U[5] = {1, 0}; U[10] = {1, 0}; U[15] = {-1, 0}; break;
    case OP_SWAP: U[0] = {1, 0}; U[6] = {1, 0}; U[9] = {1, 0}; U[15] = {1, 0}; break;
    case OP_CP: {
        double sp, cp;
        sincos(th, &sp, &cp);
        U[0] = {1, 0}; U[5] = {1, 0}; U[10] = {1, 0}; U[15] = {cp, sp};
        break;
    }
    case OP_RZZ: U[0] = {c, -s}; U[5] = {c, s}; U[10] = {c, s}; U[15] = {c, -s}; break;
    case OP_UNITARY:
        for (int i = 0; i < dim * dim; ++i) U[i] = fixed[g.mat_off + i];
        break;
    }
}

// One matrix slot of one sample: the product of its factor gates (angles
// from the sample's params / data rows), formed in double, rounded once.
template <typename T>
__device__ void prepare_slot(const DGate *gates, const double2 *fixed, const DSlot &sl, const double *prow,
                             const double *drow, cx<T> *out) {
    const int dim = sl.dim;
    if (dim > 4) {  // a single dense factor of 3..5 qubits
        const DGate g = gates[sl.f[0]];
        for (int r = 0; r < dim; ++r)
            for (int c = 0; c < dim; ++c) {
                double2 e = sl.dagger ? fixed[g.mat_off + c * dim + r] : fixed[g.mat_off + r * dim + c];
                if (sl.dagger) e.y = -e.y;
                out[r * dim + c] = cx<T>{(T)e.x, (T)e.y};
            }
        return;
    }
    double2 M[16], F[16], P[16];
    for (int i = 0; i < dim * dim; ++i) M[i] = double2{(i % (dim + 1)) == 0 ? 1.0 : 0.0, 0.0};
    for (int f = 0; f < sl.nf; ++f) {
        const DGate g = gates[sl.f[f]];
        double v = 1.0;
        if (g.src == SRC_PARAM) v = prow[g.idx];
        else if (g.src == SRC_DATA) v = drow[g.idx];
        gate_matrix(g, g.scale * v, fixed, F);
        for (int r = 0; r < dim; ++r)          // P = F * M  (F acts after M)
            for (int c = 0; c < dim; ++c) {
                double2 acc{0.0, 0.0};
                for (int k = 0; k < dim; ++k) {
                    const double2 x = F[r * dim + k], y = M[k * dim + c];
                    acc.x += x.x * y.x - x.y * y.y;
                    acc.y += x.x * y.y + x.y * y.x;
                }
                P[r * dim + c] = acc;
            }
        for (int i = 0; i < dim * dim; ++i) M[i] = P[i];
    }
    for (int r = 0; r < dim; ++r)
        for (int c = 0; c < dim; ++c) {
            double2 e = sl.dagger ? M[c * dim + r] : M[r * dim + c];
            if (sl.dagger) e.y = -e.y;
            out[r * dim + c] = cx<T>{(T)e.x, (T)e.y};
        }
}

template <typename T>
__global__ void k_prepare(const DGate *gates, const double2 *fixed, const DSlot *slots, int nslots,
                          const double *params, int64_t pstride, const double *data, int64_t dstride,
                          cx<T> *mats, int64_t block) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t b = blockIdx.y;
    if (s >= nslots) return;
    const DSlot sl = slots[s];
    prepare_slot<T>(gates, fixed, sl, params ? params + b * pstride : nullptr, data ? data + b * dstride : nullptr,
                    mats + b * block + sl.off);
}

// Uneven batches: the slots of every circuit in one launch (blockIdx.y =
// circuit entry); matrices at ws + mats_off, parameters at params + par_off.
template <typename T>
__global__ void k_prepare_multi(const MPrep *ents, const double *params, char *ws) {
    const MPrep E = ents[blockIdx.y];
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= E.nslots) return;
    const DSlot sl = E.slots[s];
    prepare_slot<T>(E.gates, E.fixed, sl, params ? params + E.par_off : nullptr, nullptr,
                    (cx<T> *)(ws + E.mats_off) + sl.off);
}

// One dense block per workgroup, one column per thread: the column starts
// as a unit vector and every factor gate is applied to it as to a K-qubit
// state (double precision), then the column is rounded once into the block.
template <typename T>
__global__ void k_prepare_block(const DGate *gates, const double2 *fixed, const DBlock *blocks, const int32_t *factors,
                                const double *params, int64_t pstride, const double *data, int64_t dstride,
                                cx<T> *mats, int64_t block) {
    const DBlock bl = blocks[blockIdx.x];
    const int64_t b = blockIdx.y;
    const int D = 1 << bl.k, c = threadIdx.x;
    if (c >= D) return;
    double2 col[32];
    for (int r = 0; r < D; ++r) col[r] = double2{r == c ? 1.0 : 0.0, 0.0};
    double2 F[16];
    for (int f = 0; f < bl.nf; ++f) {
        const DGate g = gates[factors[bl.foff + f]];
        double v = 1.0;
        if (g.src == SRC_PARAM) v = params[b * pstride + g.idx];
        else if (g.src == SRC_DATA) v = data[b * dstride + g.idx];
        gate_matrix(g, g.scale * v, fixed, F);
        // block index bit of each gate bit: bb[t] sits at bit (k-1-t) of the block index
        int pos[2] = {0, 0};
        for (int q = 0; q < g.nq; ++q)
            for (int t = 0; t < bl.k; ++t)
                if (bl.bb[t] == g.bits[q]) pos[q] = bl.k - 1 - t;
        if (g.nq == 1) {
            const int m = 1 << pos[0];
            for (int r = 0; r < D; ++r) {
                if (r & m) continue;
                const double2 a0 = col[r], a1 = col[r | m];
                col[r] = double2{F[0].x * a0.x - F[0].y * a0.y + F[1].x * a1.x - F[1].y * a1.y,
                                 F[0].x * a0.y + F[0].y * a0.x + F[1].x * a1.y + F[1].y * a1.x};
                col[r | m] = double2{F[2].x * a0.x - F[2].y * a0.y + F[3].x * a1.x - F[3].y * a1.y,
                                     F[2].x * a0.y + F[2].y * a0.x + F[3].x * a1.y + F[3].y * a1.x};
            }
        } else {
            const int m0 = 1 << pos[0], m1 = 1 << pos[1];   // gate bits[0] is the MSB of F's index
            for (int r = 0; r < D; ++r) {
                if (r & (m0 | m1)) continue;
                const int idx[4] = {r, r | m1, r | m0, r | m0 | m1};
                double2 a[4], o[4];
                for (int q = 0; q < 4; ++q) a[q] = col[idx[q]];
                for (int x = 0; x < 4; ++x) {
                    double re = 0, im = 0;
                    for (int q = 0; q < 4; ++q) {
                        re += F[x * 4 + q].x * a[q].x - F[x * 4 + q].y * a[q].y;
                        im += F[x * 4 + q].x * a[q].y + F[x * 4 + q].y * a[q].x;
                    }
                    o[x] = double2{re, im};
                }
                for (int q = 0; q < 4; ++q) col[idx[q]] = o[q];
            }
        }
    }
    cx<T> *out = mats + b * block + bl.off;
    for (int r = 0; r < D; ++r) out[r * D + c] = cx<T>{(T)col[r].x, (T)col[r].y};
}

// ============================================================ init
template <typename T>
__global__ void k_init_zero(cx<T> *st, int n, int64_t total) {
    const int64_t mask = (int64_t(1) << n) - 1;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x)
        st[i] = cx<T>{(i & mask) == 0 ? T(1) : T(0), T(0)};
}

template <typename T>
__global__ void k_init_copy(cx<T> *st, const cx<T> *init, int n, int64_t total) {
    const int64_t mask = (int64_t(1) << n) - 1;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x)
        st[i] = init[i & mask];
}

template <typename T>
__global__ void k_copy(cx<T> *dst, const cx<T> *src, int64_t count) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

// amp_j = prod_s u_s[bit_s(j)], u_s = first column of the folded one-qubit
// product on physical bit s (identity column (1, 0) where nothing is folded).
template <typename T, typename M>
__global__ __launch_bounds__(256) void k_init_product(cx<T> *st, int n, const cx<M> *mats, int64_t mstride,
                                                      const int64_t *fold_off) {
    __shared__ double2 u[64][2];
    const int64_t b = blockIdx.y;
    if (threadIdx.x < n) {
        const int64_t off = fold_off[threadIdx.x];
        if (off < 0) {
            u[threadIdx.x][0] = double2{1.0, 0.0};
            u[threadIdx.x][1] = double2{0.0, 0.0};
        } else {
            const cx<M> *m = mats + b * mstride + off;
            u[threadIdx.x][0] = double2{(double)m[0].x, (double)m[0].y};
            u[threadIdx.x][1] = double2{(double)m[2].x, (double)m[2].y};
        }
    }
    __syncthreads();
    const int64_t N = int64_t(1) << n;
    cx<T> *p = st + b * N;
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < N; j += (int64_t)gridDim.x * blockDim.x) {
        double2 acc{1.0, 0.0};
        for (int s = 0; s < n; ++s) {
            const double2 f = u[s][(j >> s) & 1];
            acc = double2{acc.x * f.x - acc.y * f.y, acc.x * f.y + acc.y * f.x};
        }
        p[j] = cx<T>{(T)acc.x, (T)acc.y};
    }
}

// The same state for n >= 16: a block writes 2^16 consecutive amplitudes whose
// bits 16.. are fixed (one product per block), bits 8..15 index a 256-entry
// product table in LDS and bits 0..7 are this thread's (one product per
// thread), so each amplitude costs one complex multiply.
template <typename T, typename M>
__global__ __launch_bounds__(256) void k_init_product_tab(cx<T> *st, int n, const cx<M> *mats, int64_t mstride,
                                                          const int64_t *fold_off) {
    __shared__ double2 u[64][2];
    __shared__ double2 tab[256];
    const int64_t b = blockIdx.y;
    const int t = threadIdx.x;
    if (t < n) {
        const int64_t off = fold_off[t];
        if (off < 0) {
            u[t][0] = double2{1.0, 0.0};
            u[t][1] = double2{0.0, 0.0};
        } else {
            const cx<M> *m = mats + b * mstride + off;
            u[t][0] = double2{(double)m[0].x, (double)m[0].y};
            u[t][1] = double2{(double)m[2].x, (double)m[2].y};
        }
    }
    __syncthreads();
    auto mul = [](double2 a, double2 c) { return double2{a.x * c.x - a.y * c.y, a.x * c.y + a.y * c.x}; };
    {
        double2 f{1.0, 0.0};
        for (int k = 0; k < 8; ++k) f = mul(f, u[8 + k][(t >> k) & 1]);
        tab[t] = f;
    }
    double2 lo{1.0, 0.0};
    for (int k = 0; k < 8; ++k) lo = mul(lo, u[k][(t >> k) & 1]);
    __syncthreads();
    const int64_t nblk = int64_t(1) << (n - 16);
    cx<T> *p = st + (b << n);
    for (int64_t blk = blockIdx.x; blk < nblk; blk += gridDim.x) {
        double2 q = lo;
        for (int k = 16; k < n; ++k) q = mul(q, u[k][(blk >> (k - 16)) & 1]);
        cx<T> *pb = p + (blk << 16);
        for (int r = 0; r < 256; ++r) {
            const double2 a = mul(q, tab[r]);
            pb[(r << 8) + t] = cx<T>{(T)a.x, (T)a.y};
        }
    }
}

// Uneven batches: every circuit's start state in one launch (blockIdx.y =
// circuit entry): the folded product state (as k_init_product) or |0..0>.
template <typename T>
__global__ __launch_bounds__(256) void k_init_multi(cx<T> *st, const char *ws, const MInit *ents) {
    __shared__ double2 u[64][2];
    const MInit E = ents[blockIdx.y];
    const int n = E.n;
    const int64_t N = int64_t(1) << n;
    if (blockIdx.x * (int64_t)blockDim.x >= N) return;   // block-uniform
    if (threadIdx.x < n) {
        const int64_t off = E.has_fold ? E.fold[threadIdx.x] : -1;
        if (off < 0) {
            u[threadIdx.x][0] = double2{1.0, 0.0};
            u[threadIdx.x][1] = double2{0.0, 0.0};
        } else {
            const cx<T> *m = (const cx<T> *)(ws + E.mats_off) + off;
            u[threadIdx.x][0] = double2{(double)m[0].x, (double)m[0].y};
            u[threadIdx.x][1] = double2{(double)m[2].x, (double)m[2].y};
        }
    }
    __syncthreads();
    cx<T> *p = st + E.st_off;
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < N; j += (int64_t)gridDim.x * blockDim.x) {
        double2 acc{1.0, 0.0};
        for (int k = 0; k < n; ++k) {
            const double2 f = u[k][(j >> k) & 1];
            acc = double2{acc.x * f.x - acc.y * f.y, acc.x * f.y + acc.y * f.x};
        }
        p[j] = cx<T>{(T)acc.x, (T)acc.y};
    }
}

// ============================================================ plain per-gate sweeps
// Each thread keeps SWEEP_U pairs in flight: all loads are issued before the
// first update, so a wave has 2 x SWEEP_U independent 512-byte (complex64)
// requests outstanding.
constexpr int SWEEP_U = 4;

template <typename T>
__global__ __launch_bounds__(256) void k_gate1(cx<T> *st, int n, int64_t total, int bit, const cx<T> *mats,
                                               int64_t mstride, int64_t off) {
    const int64_t halfmask = (int64_t(1) << (n - 1)) - 1;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i0 = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i0 < total; i0 += stride * SWEEP_U) {
        cx<T> a0[SWEEP_U], a1[SWEEP_U];
        int64_t j0[SWEEP_U];
#pragma unroll
        for (int u = 0; u < SWEEP_U; ++u) {
            const int64_t i = i0 + u * stride;
            if (i < total) {
                const int64_t b = i >> (n - 1), k = i & halfmask;
                j0[u] = (b << n) + insert_zero(k, bit);
                a0[u] = st[j0[u]];
                a1[u] = st[j0[u] + (int64_t(1) << bit)];
            }
        }
#pragma unroll
        for (int u = 0; u < SWEEP_U; ++u) {
            const int64_t i = i0 + u * stride;
            if (i < total) {
                const cx<T> *m = mats + (i >> (n - 1)) * mstride + off;
                st[j0[u]] = cmac(m[0], a0[u], cmul(m[1], a1[u]));
                st[j0[u] + (int64_t(1) << bit)] = cmac(m[2], a0[u], cmul(m[3], a1[u]));
            }
        }
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_cnot(cx<T> *st, int n, int64_t total, int cbit, int tbit) {
    const int lo = cbit < tbit ? cbit : tbit, hi = cbit < tbit ? tbit : cbit;
    const int64_t qmask = (int64_t(1) << (n - 2)) - 1;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t b = i >> (n - 2), k = i & qmask;
        const int64_t j0 = insert_zero(insert_zero(k, lo), hi) | (int64_t(1) << cbit);
        const int64_t j1 = j0 | (int64_t(1) << tbit);
        cx<T> *p = st + (b << n);
        const cx<T> a0 = p[j0], a1 = p[j1];
        p[j0] = a1;
        p[j1] = a0;
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_cz(cx<T> *st, int n, int64_t total, int abit, int bbit) {
    const int lo = abit < bbit ? abit : bbit, hi = abit < bbit ? bbit : abit;
    const int64_t qmask = (int64_t(1) << (n - 2)) - 1;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t b = i >> (n - 2), k = i & qmask;
        const int64_t j = insert_zero(insert_zero(k, lo), hi) | (int64_t(1) << abit) | (int64_t(1) << bbit);
        cx<T> *p = st + (b << n);
        p[j] = cneg(p[j]);
    }
}

struct KBits {
    int32_t bits[5];     // bits[0] = MSB of the matrix index
    int32_t sorted[5];   // ascending
};

template <typename T, int K>
__global__ __launch_bounds__(256) void k_gatek(cx<T> *st, int n, int64_t total, KBits kb, const cx<T> *mats,
                                               int64_t mstride, int64_t off) {
    constexpr int D = 1 << K;
    const int64_t gmask = (int64_t(1) << (n - K)) - 1;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t b = i >> (n - K);
        int64_t j = i & gmask;
#pragma unroll
        for (int t = 0; t < K; ++t) j = insert_zero(j, kb.sorted[t]);
        cx<T> *p = st + (b << n) + j;
        const cx<T> *m = mats + b * mstride + off;
        cx<T> a[D], o[D];
#pragma unroll
        for (int x = 0; x < D; ++x) {
            int64_t of = 0;
#pragma unroll
            for (int t = 0; t < K; ++t)
                if ((x >> (K - 1 - t)) & 1) of += int64_t(1) << kb.bits[t];
            a[x] = p[of];
        }
#pragma unroll
        for (int r = 0; r < D; ++r) {
            cx<T> acc{0, 0};
#pragma unroll
            for (int c = 0; c < D; ++c) acc = cmac(m[r * D + c], a[c], acc);
            o[r] = acc;
        }
#pragma unroll
        for (int x = 0; x < D; ++x) {
            int64_t of = 0;
#pragma unroll
            for (int t = 0; t < K; ++t)
                if ((x >> (K - 1 - t)) & 1) of += int64_t(1) << kb.bits[t];
            p[of] = o[x];
        }
    }
}

// ============================================================ matrix-core dense blocks
// y = U x for a dense 2^K x 2^K complex U on K target bits (K = 4, 5), as the
// real product [[Re U, -Im U], [Im U, Re U]] (2D x 2D, D = 2^K) times
// [Re x; Im x] (2D x columns).  Columns are the 2^(n-K) index values of the
// other bits; a wave owns 32 consecutive columns (complex64) or 16 (complex128),
// so with no target bit among the lowest 5 (4) physical bits each row is one
// contiguous run.  complex64: v_mfma_f32_32x32x2_f32, lane l supplies
// B[k = l/32][n = l%32] and A[m = l%32][k = l/32], and receives
// D[8 (v/4) + 4 (l/32) + v%4][l%32] in accumulator v.  complex128:
// v_mfma_f64_16x16x4_f64, B[k = l/16][n = l%16], A[m = l%16][k = l/16],
// D[l/16 + 4 v][l%16] (lane layout checked on the device).
struct DenseBits {
    int32_t bits[5];     // physical bits, bits[0] = MSB of U's index
    int32_t sorted[5];   // ascending
};

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

template <int K>
__device__ __forceinline__ int64_t dense_row_off(int r, const DenseBits &db) {
    int64_t o = 0;
#pragma unroll
    for (int t = 0; t < K; ++t)
        if ((r >> (K - 1 - t)) & 1) o += int64_t(1) << db.bits[t];
    return o;
}

// entry (m, c) of the real 2D x 2D form of U (row-major complex, dimension D)
template <int D, typename T>
__device__ __forceinline__ T real_form(cptr<cx<T>> U, int m, int c) {
    const int mr = m & (D - 1), cr = c & (D - 1);
    const bool im_row = m >= D, im_col = c >= D;
    const T re = U[mr * D + cr].x, im = U[mr * D + cr].y;
    return im_row ? (im_col ? re : im) : (im_col ? -im : re);
}

template <int K>
__global__ __launch_bounds__(256) void k_dense_f32(C64 *st, int n, int64_t groups, DenseBits db, const C64 *mats,
                                                   int64_t mstride, int64_t off) {
    constexpr int D = 1 << K, MB = 2 * D / 32, KK = D, XR = D / 2;
    const int lane = threadIdx.x & 63, kq = lane >> 5, nn = lane & 31;
    const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = (gridDim.x * (int64_t)blockDim.x) >> 6;
    const int gshift = n - K - 5;
    // K = 5 keeps only [Re U | Im U] (32 x 64, one register per k-step) and
    // moves the sign and the real/imaginary swap of the real form onto the
    // amplitudes:  Re y = [Re U | Im U] [Re x; -Im x],
    //              Im y = [Re U | Im U] [Im x;  Re x].
    // Half the matrix registers of the full real form, the same products.
    constexpr int MA = K == 5 ? 1 : MB;
    float A[MA][KK];
    int64_t cur = -1;
    for (int64_t g = wave; g < groups; g += nwaves) {
        const int64_t b = g >> gshift;
        if (b != cur) {
            const cptr<C64> U = to_const(mats + b * mstride + off);
            if constexpr (K == 5) {
#pragma unroll
                for (int kk = 0; kk < KK; ++kk) {
                    const int c = 2 * kk + kq;
                    A[0][kk] = c < D ? U[nn * D + c].x : U[nn * D + c - D].y;
                }
            } else {
#pragma unroll
                for (int mb = 0; mb < MB; ++mb)
#pragma unroll
                    for (int kk = 0; kk < KK; ++kk) A[mb][kk] = real_form<D, float>(U, 32 * mb + nn, 2 * kk + kq);
            }
            cur = b;
        }
        int64_t col = ((g & ((int64_t(1) << gshift) - 1)) << 5) | nn;
#pragma unroll
        for (int t = 0; t < K; ++t) col = insert_zero(col, db.sorted[t]);
        C64 *p = st + (b << n) + col;
        C64 x[XR];
#pragma unroll
        for (int k2 = 0; k2 < XR; ++k2) x[k2] = p[dense_row_off<K>(2 * k2 + kq, db)];
        f32x16 acc[MB];
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) acc[mb] = f32x16{};
        if constexpr (K == 5) {
#pragma unroll
            for (int kk = 0; kk < KK; ++kk) {
                const float br = kk < XR ? x[kk].x : -x[kk - XR].y;
                const float bi = kk < XR ? x[kk].y : x[kk - XR].x;
                acc[0] = __builtin_amdgcn_mfma_f32_32x32x2f32(A[0][kk], br, acc[0], 0, 0, 0);
                acc[1] = __builtin_amdgcn_mfma_f32_32x32x2f32(A[0][kk], bi, acc[1], 0, 0, 0);
            }
        } else {
#pragma unroll
            for (int kk = 0; kk < KK; ++kk) {
                const float bv = kk < XR ? x[kk].x : x[kk - XR].y;
#pragma unroll
                for (int mb = 0; mb < MB; ++mb) acc[mb] = __builtin_amdgcn_mfma_f32_32x32x2f32(A[mb][kk], bv, acc[mb], 0, 0, 0);
            }
        }
        if constexpr (MB == 2) {
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int r = 8 * (v >> 2) + 4 * kq + (v & 3);
                p[dense_row_off<K>(r, db)] = C64{acc[0][v], acc[1][v]};
            }
        } else {
#pragma unroll
            for (int v = 0; v < 8; ++v) {
                const int r = 8 * (v >> 2) + 4 * kq + (v & 3);   // rows < 16: real parts; row + 16: imaginary
                p[dense_row_off<K>(r, db)] = C64{acc[0][v], acc[0][v + 8]};
            }
        }
    }
}

// Dense block through LDS: the wave reads and writes its group (32 columns x
// 2^K rows) with 16-byte coalesced accesses and transposes it through LDS
// into the matrix cores' column layout.  Two cases:
//  * CONTIG: every block bit lies below K + 5, so a group is one contiguous
//    run of 2^(K+5) amplitudes, indexed in LDS by its offset j.  Reading the
//    rows straight from memory would give every lane its own 2^K-amplitude
//    stride: each load touches 32 cache lines for 8 useful bytes apiece.
//  * otherwise physical bit 0 is a column bit: amplitude pairs (2c, 2c + 1)
//    of a row are adjacent in memory, and LDS is indexed by j = c + 32 r.
// LDS index of j: j with its low five bits XORed with the next five, so the
// 32 lanes of a half-wave reading one row of 32 columns hit distinct banks
// (in the CONTIG case when the column bits fall in distinct positions mod 5,
// as in every contiguous block).  One wave per block; the products are the
// same as k_dense_f32's.
typedef float f32x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ int lds_swz(int j) { return j ^ ((j >> 5) & 31); }

template <int K, bool CONTIG>
__global__ __launch_bounds__(64) void k_dense_f32_lds(C64 *st, int n, int64_t groups, DenseBits db, const C64 *mats,
                                                      int64_t mstride, int64_t off) {
    constexpr int D = 1 << K, MB = 2 * D / 32, KK = D, XR = D / 2, GA = 32 * D, NL = GA / 128;
    constexpr int MA = K == 5 ? 1 : MB;
    __shared__ f32x4 lds4[GA / 2];
    C64 *lds = reinterpret_cast<C64 *>(lds4);
    const int lane = threadIdx.x, kq = lane >> 5, nn = lane & 31;
    const int gshift = n - K - 5;
    // physical offset of column c inside a group: c spread over the lowest
    // non-block bits
    auto colpos = [&](int64_t c) {
#pragma unroll
        for (int t = 0; t < K; ++t) c = insert_zero(c, db.sorted[t]);
        return c;
    };
    // LDS slot of this lane's column in row r
    const int64_t mycol = colpos(nn);
    auto slot = [&](int r) {
        return CONTIG ? lds_swz((int)(mycol + dense_row_off<K>(r, db))) : lds_swz(nn + 32 * r);
    };
    // physical offset (inside the group) of the amplitude pair a lane moves
    // in coalesced access i: pair index j = 2 (lane + 64 i)
    const int64_t pcol = CONTIG ? 0 : colpos(2 * (lane & 15));
    auto pair_off = [&](int i) -> int64_t {
        const int j = 2 * (lane + 64 * i);
        return CONTIG ? j : pcol + dense_row_off<K>(j >> 5, db);
    };
    float A[MA][KK];
    int64_t cur = -1;
    for (int64_t g = blockIdx.x; g < groups; g += gridDim.x) {
        const int64_t b = g >> gshift;
        if (b != cur) {
            const cptr<C64> U = to_const(mats + b * mstride + off);
            if constexpr (K == 5) {
#pragma unroll
                for (int kk = 0; kk < KK; ++kk) {
                    const int c = 2 * kk + kq;
                    A[0][kk] = c < D ? U[nn * D + c].x : U[nn * D + c - D].y;
                }
            } else {
#pragma unroll
                for (int mb = 0; mb < MB; ++mb)
#pragma unroll
                    for (int kk = 0; kk < KK; ++kk) A[mb][kk] = real_form<D, float>(U, 32 * mb + nn, 2 * kk + kq);
            }
            cur = b;
        }
        C64 *gb = CONTIG ? st + (g << (K + 5))
                         : st + (b << n) + colpos((g & ((int64_t(1) << gshift) - 1)) << 5);
        f32x4 w[NL];
#pragma unroll
        for (int i = 0; i < NL; ++i) w[i] = __builtin_nontemporal_load(reinterpret_cast<const f32x4 *>(gb + pair_off(i)));
#pragma unroll
        for (int i = 0; i < NL; ++i) {
            const int q = lds_swz(2 * (lane + 64 * i));   // q ^ 1 is the slot of the pair's second amplitude
            lds4[q >> 1] = (q & 1) ? f32x4{w[i].z, w[i].w, w[i].x, w[i].y} : w[i];
        }
        __syncthreads();
        C64 x[XR];
#pragma unroll
        for (int k2 = 0; k2 < XR; ++k2) x[k2] = lds[slot(2 * k2 + kq)];
        f32x16 acc[MB];
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) acc[mb] = f32x16{};
        if constexpr (K == 5) {
#pragma unroll
            for (int kk = 0; kk < KK; ++kk) {
                const float br = kk < XR ? x[kk].x : -x[kk - XR].y;
                const float bi = kk < XR ? x[kk].y : x[kk - XR].x;
                acc[0] = __builtin_amdgcn_mfma_f32_32x32x2f32(A[0][kk], br, acc[0], 0, 0, 0);
                acc[1] = __builtin_amdgcn_mfma_f32_32x32x2f32(A[0][kk], bi, acc[1], 0, 0, 0);
            }
        } else {
#pragma unroll
            for (int kk = 0; kk < KK; ++kk) {
                const float bv = kk < XR ? x[kk].x : x[kk - XR].y;
#pragma unroll
                for (int mb = 0; mb < MB; ++mb) acc[mb] = __builtin_amdgcn_mfma_f32_32x32x2f32(A[mb][kk], bv, acc[mb], 0, 0, 0);
            }
        }
        __syncthreads();   // every lane has read its column before it is overwritten
        if constexpr (MB == 2) {
#pragma unroll
            for (int v = 0; v < 16; ++v) lds[slot(8 * (v >> 2) + 4 * kq + (v & 3))] = C64{acc[0][v], acc[1][v]};
        } else {
#pragma unroll
            for (int v = 0; v < 8; ++v)   // rows < 16: real parts; row + 16: imaginary
                lds[slot(8 * (v >> 2) + 4 * kq + (v & 3))] = C64{acc[0][v], acc[0][v + 8]};
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < NL; ++i) {
            const int q = lds_swz(2 * (lane + 64 * i));
            const f32x4 y = lds4[q >> 1];
            __builtin_nontemporal_store((q & 1) ? f32x4{y.z, y.w, y.x, y.y} : y,
                                        reinterpret_cast<f32x4 *>(gb + pair_off(i)));
        }
        __syncthreads();   // the next group's writes to LDS come after every lane's read
    }
}

template <int K>
__global__ __launch_bounds__(256) void k_dense_f64(C128 *st, int n, int64_t groups, DenseBits db, const C128 *mats,
                                                   int64_t mstride, int64_t off) {
    constexpr int D = 1 << K, MB = 2 * D / 16, KK = 2 * D / 4, XR = D / 4;
    const int lane = threadIdx.x & 63, kq = lane >> 4, nn = lane & 15;
    const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = (gridDim.x * (int64_t)blockDim.x) >> 6;
    const int gshift = n - K - 4;
    double A[MB][KK];
    int64_t cur = -1;
    for (int64_t g = wave; g < groups; g += nwaves) {
        const int64_t b = g >> gshift;
        if (b != cur) {
            const cptr<C128> U = to_const(mats + b * mstride + off);
#pragma unroll
            for (int mb = 0; mb < MB; ++mb)
#pragma unroll
                for (int kk = 0; kk < KK; ++kk) A[mb][kk] = real_form<D, double>(U, 16 * mb + nn, 4 * kk + kq);
            cur = b;
        }
        int64_t col = ((g & ((int64_t(1) << gshift) - 1)) << 4) | nn;
#pragma unroll
        for (int t = 0; t < K; ++t) col = insert_zero(col, db.sorted[t]);
        C128 *p = st + (b << n) + col;
        C128 x[XR];     // rows r = 4 k2 + kq
#pragma unroll
        for (int k2 = 0; k2 < XR; ++k2) x[k2] = p[dense_row_off<K>(4 * k2 + kq, db)];
        f64x4 acc[MB];
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) acc[mb] = f64x4{};
#pragma unroll
        for (int kk = 0; kk < KK; ++kk) {
            // B[k][n] = X[4 kk + k][n]: real rows 0..D-1, imaginary rows D..2D-1
            const double bv = kk < XR ? x[kk].x : x[kk - XR].y;
#pragma unroll
            for (int mb = 0; mb < MB; ++mb) acc[mb] = __builtin_amdgcn_mfma_f64_16x16x4f64(A[mb][kk], bv, acc[mb], 0, 0, 0);
        }
        // block mb covers rows 16 mb .. 16 mb + 15; real parts in the first MB/2 blocks;
        // accumulator v of lane l holds row 16 mb + l/16 + 4 v, column l % 16
#pragma unroll
        for (int mb = 0; mb < MB / 2; ++mb)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int r = 16 * mb + kq + 4 * v;
                p[dense_row_off<K>(r, db)] = C128{acc[mb][v], acc[mb + MB / 2][v]};
            }
    }
}

// ============================================================ reductions
__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
    return x;
}

// Im<lambda|G|psi> of one differentiable gate over every amplitude of a sample.
template <typename T>
__global__ __launch_bounds__(256) void k_grad_gate(const cx<T> *psi, const cx<T> *lam, int n, int gen, int bit0,
                                                   int bit1, double *partial, int wps, int ngrad, int gslot) {
    __shared__ double red[4];
    const int64_t b = blockIdx.y;
    const int64_t N = int64_t(1) << n;
    const cx<T> *p = psi + b * N, *q = lam + b * N;
    double s = 0.0;
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < N; j += (int64_t)wps * blockDim.x) {
        const cx<T> l = q[j];
        const bool b0 = (j >> bit0) & 1;
        cx<T> o;
        bool neg = false, zero = false;
        switch (gen) {
        case GEN_X: o = p[j ^ (int64_t(1) << bit0)]; break;
        case GEN_Y: {
            const cx<T> t = p[j ^ (int64_t(1) << bit0)];
            o = b0 ? cx<T>{-t.y, t.x} : cx<T>{t.y, -t.x};
            break;
        }
        case GEN_Z: o = p[j]; neg = b0; break;
        case GEN_ZZ: o = p[j]; neg = b0 != (bool)((j >> bit1) & 1); break;
        default: o = p[j]; zero = !(b0 && ((j >> bit1) & 1)); break;   // GEN_P11
        }
        const double t = (double)(l.x * o.y - l.y * o.x);
        s += zero ? 0.0 : (neg ? -t : t);
    }
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0)
        partial[(b * wps + blockIdx.x) * (int64_t)ngrad + gslot] = (red[0] + red[1]) + (red[2] + red[3]);
}

__global__ void k_grad_final(const double *partial, int64_t batch, int wps, int ngrad, const int64_t *csr_off,
                             const int32_t *csr_g, const double *csr_f, int64_t nout, int per_sample,
                             double *out) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t total = per_sample ? batch * nout : nout;
    if (i >= total) return;
    const int64_t p = per_sample ? i % nout : i;
    const int64_t b0 = per_sample ? i / nout : 0, b1 = per_sample ? b0 + 1 : batch;
    double sum = 0.0;
    for (int64_t e = csr_off[p]; e < csr_off[p + 1]; ++e) {
        const int g = csr_g[e];
        double s = 0.0;
        for (int64_t b = b0; b < b1; ++b)
            for (int w = 0; w < wps; ++w) s += partial[(b * wps + w) * (int64_t)ngrad + g];
        sum += csr_f[e] * s;
    }
    out[i] = sum;
}

// ============================================================ Hessian
// Angle rows of the shifted circuits: occurrence a (a gate angle that reads
// parameter occ_param[a] with chain factor occ_scale[a]) gets angle
// occ_scale[a] * params[occ_param[a]] in every row; rows 2r and 2r+1 shift
// occurrence c0 + r by +pi/2 and -pi/2.
__global__ void k_hess_rows(const double *params, const int32_t *occ_param, const double *occ_scale, int64_t K,
                            int64_t c0, int64_t mc, double *rows) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= 2 * mc * K) return;
    const int64_t row = i / K, a = i % K;
    double v = occ_scale[a] * params[occ_param[a]];
    if (a == c0 + row / 2) v += (row & 1) ? -0.5 * M_PI : 0.5 * M_PI;
    rows[i] = v;
}

// rows x nobs copies of the observable weights (the adjoint seed of every
// shifted circuit)
__global__ void k_bcast_rows(const double *w, int32_t nobs, int64_t rows, double *out) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < rows * nobs) out[i] = w[i % nobs];
}

// H[p][q] += sum over occurrences b of parameter q inside this chunk
// [c0, c0+mc) of s_b sum over occurrences a of parameter p of
// s_a (G[2(b-c0)][a] - G[2(b-c0)+1][a]) / 2, where G[row][a] is the
// gradient of the shifted circuit `row` with respect to angle a.  One thread
// per (p, q), sums in a fixed order: deterministic.
__global__ void k_hess_accum(const double *G, int64_t K, int64_t c0, int64_t mc, const int64_t *poff,
                             const int32_t *pocc, const double *occ_scale, int64_t P, double *H) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= P * P) return;
    const int64_t p = i / P, q = i % P;
    double acc = 0.0;
    for (int64_t eb = poff[q]; eb < poff[q + 1]; ++eb) {
        const int64_t b = pocc[eb];
        if (b < c0 || b >= c0 + mc) continue;
        const double *gp = G + 2 * (b - c0) * K, *gm = gp + K;
        double s = 0.0;
        for (int64_t ea = poff[p]; ea < poff[p + 1]; ++ea) {
            const int64_t a = pocc[ea];
            s += occ_scale[a] * 0.5 * (gp[a] - gm[a]);
        }
        acc += occ_scale[b] * s;
    }
    H[i] = (c0 == 0 ? 0.0 : H[i]) + acc;
}

constexpr int EXP_TM = 32;

// Partial sums S_t = sum_j (-1)^{|j & z_t|} conj(psi_{j^x}) psi_j over this
// block's share of the amplitudes, for up to TM (<= EXP_TM) terms of one
// X-mask group.  DIAG (x = 0): the product is |psi_j|^2, real.  Otherwise the
// indices pair up as (j, j^x) with bit h (the highest of x) clear in j: the
// summand at j^x is the conjugate of the one at j times
// sigma = (-1)^{|x & z_t|}, so a pair adds 2 s_j Re(c) when sigma = +1 and
// 2 i s_j Im(c) when sigma = -1 (c = conj(psi_{j^x}) psi_j), and each
// amplitude is loaded once per group.
template <typename T, bool DIAG, int TM = EXP_TM>
__device__ __forceinline__ void expval_chunk(const cx<T> *p, int64_t N, uint64_t x, cptr<DTerm> terms, int c0,
                                             int nt, double *row, int eb, double (*red)[2 * EXP_TM], int64_t blk) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    uint64_t z[TM];
    double ar[TM], ai[TM];
#pragma unroll
    for (int t = 0; t < TM; ++t) {
        z[t] = t < nt ? terms[c0 + t].zmask : 0;
        ar[t] = 0.0;
        ai[t] = 0.0;
    }
    if (DIAG) {
        for (int64_t j = blk * blockDim.x + threadIdx.x; j < N; j += (int64_t)eb * blockDim.x) {
            const cx<T> a = p[j];
            const double pr = (double)(a.x * a.x + a.y * a.y);
#pragma unroll
            for (int t = 0; t < TM; ++t) {
                if (t < nt) {
                    const bool neg = __popcll((uint64_t)j & z[t]) & 1;
                    ar[t] += neg ? -pr : pr;
                }
            }
        }
    } else {
        const int h = 63 - __clzll((long long)x);   // x != 0
        const int64_t lo = (int64_t(1) << h) - 1;
        bool odd[TM];
#pragma unroll
        for (int t = 0; t < TM; ++t) odd[t] = t < nt && (__popcll(x & z[t]) & 1);
        for (int64_t k = blk * blockDim.x + threadIdx.x; k < (N >> 1); k += (int64_t)eb * blockDim.x) {
            const int64_t j = ((k & ~lo) << 1) | (k & lo);
            const cx<T> a = p[j];
            const cx<T> o = p[j ^ (int64_t)x];
            const double pr = (double)(o.x * a.x + o.y * a.y);
            const double pi = (double)(o.x * a.y - o.y * a.x);
#pragma unroll
            for (int t = 0; t < TM; ++t) {
                if (t < nt) {
                    const bool neg = __popcll((uint64_t)j & z[t]) & 1;
                    if (odd[t]) ai[t] += neg ? -pi : pi;
                    else ar[t] += neg ? -pr : pr;
                }
            }
        }
    }
#pragma unroll
    for (int t = 0; t < TM; ++t) {
        if (t < nt) {
            const double xr = DIAG ? wave_sum(ar[t]) : 2.0 * wave_sum(ar[t]);
            const double xi = DIAG ? 0.0 : 2.0 * wave_sum(ai[t]);
            if (lane == 0) {
                red[wv][2 * t] = xr;
                red[wv][2 * t + 1] = xi;
            }
        }
    }
    __syncthreads();
    if (threadIdx.x < 2 * nt)
        row[c0 * 2 + threadIdx.x] =
            (red[0][threadIdx.x] + red[1][threadIdx.x]) + (red[2][threadIdx.x] + red[3][threadIdx.x]);
    __syncthreads();
}

template <typename T>
__global__ __launch_bounds__(256) void k_expval_part(const cx<T> *st, int n, const DGroup *groups, int g0, int ngroups,
                                                     const DTerm *terms, int nterms, double *partial, int eb) {
    __shared__ double red[4][2 * EXP_TM];
    const int64_t b = blockIdx.y;
    const int64_t N = int64_t(1) << n;
    const cx<T> *p = st + b * N;
    const cptr<DGroup> gp = to_const(groups);
    const cptr<DTerm> tp = to_const(terms);
    double *row = partial + (b * eb + blockIdx.x) * (int64_t)nterms * 2;   // this block's [nterms][2]
    for (int g = g0; g < ngroups; ++g) {
        const uint64_t x = gp[g].xmask;
        const int t0 = gp[g].t0, t1 = gp[g].t1;
        for (int c0 = t0; c0 < t1; c0 += EXP_TM) {
            const int nt = (t1 - c0) < EXP_TM ? (t1 - c0) : EXP_TM;
            if (x == 0) expval_chunk<T, true>(p, N, x, tp, c0, nt, row, eb, red, blockIdx.x);
            else expval_chunk<T, false>(p, N, x, tp, c0, nt, row, eb, red, blockIdx.x);
        }
    }
}

// multi-plan entries: work unit u belongs to the entry e with
// unit_begin[e] <= u < unit_begin[e + 1] (binary search; entries ascending)
template <typename E>
__device__ __forceinline__ int find_unit(const E *ents, int nent, int64_t u) {
    int lo = 0, hi = nent - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (ents[mid].unit_begin <= u) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Uneven batches: the expectation partial sums of every circuit in one
// launch, block u doing chunk u - unit_begin of its circuit's eb chunks,
// every X-mask group of the circuit (as k_expval_part), TM terms of a group
// per sweep over the amplitudes.  TM = 4 serves observables whose groups
// hold at most four terms (a product of random Pauli strings has one term
// per X mask) with a quarter of the registers of TM = EXP_TM, so more waves
// stay resident to hide the loads' latency.
template <typename T, int TM>
__global__ __launch_bounds__(256) void k_expval_multi(const cx<T> *st, char *ws, const MExp *ents, int nent) {
    __shared__ double red[4][2 * EXP_TM];
    const int e = find_unit(ents, nent, blockIdx.x);
    const MExp E = ents[e];
    const int64_t blk = blockIdx.x - E.unit_begin;
    const int64_t N = int64_t(1) << E.n;
    const cx<T> *p = st + E.st_off;
    const cptr<DGroup> gp = to_const(E.groups);
    const cptr<DTerm> tp = to_const(E.terms);
    double *row = (double *)(ws + E.part_off) + blk * (int64_t)E.nterms * 2;
    for (int g = 0; g < E.ngroups; ++g) {
        const uint64_t x = gp[g].xmask;
        const int t0 = gp[g].t0, t1 = gp[g].t1;
        for (int c0 = t0; c0 < t1; c0 += TM) {
            const int nt = (t1 - c0) < TM ? (t1 - c0) : TM;
            if (x == 0) expval_chunk<T, true, TM>(p, N, x, tp, c0, nt, row, E.eb, red, blk);
            else expval_chunk<T, false, TM>(p, N, x, tp, c0, nt, row, E.eb, red, blk);
        }
    }
}

// out[out_off + o] = sum over the terms of observable o of Re(w_t S_t): one
// wave per circuit, its lanes adding the chunks k = lane, lane + 64, ... in
// order, then a fixed shuffle tree (deterministic).
__global__ __launch_bounds__(64) void k_expval_final_multi(const char *ws, const MExp *ents, double *out) {
    const cptr<MExp> ep = to_const(ents);
    const int e = blockIdx.x, lane = threadIdx.x;
    const double *part = (const double *)(ws + ep[e].part_off);
    const cptr<DTerm> tp = to_const(ep[e].terms);
    const int nterms = ep[e].nterms, nobs = ep[e].nobs, eb = ep[e].eb;
    for (int o = 0; o < nobs; ++o) {
        double v = 0.0;
        for (int t = 0; t < nterms; ++t) {
            if (tp[t].obs != o) continue;
            double sr = 0.0, si = 0.0;
            for (int k = lane; k < eb; k += 64) {
                sr += part[((int64_t)k * nterms + t) * 2];
                si += part[((int64_t)k * nterms + t) * 2 + 1];
            }
            sr = wave_sum(sr);
            si = wave_sum(si);
            v += tp[t].wr * sr - tp[t].wi * si;
        }
        if (lane == 0) out[ep[e].out_off + o] = v;
    }
}

// The X-free group (diagonal observables) for n >= 11: per amplitude j the
// weight d_o(j) = sum_{t in o} w_t (-1)^{|j & z_t|} (w_t real: no Y without X).
// A wave owns tiles of 2048 consecutive amplitudes, lane l holding
// j = 2048 tile + 64 i + l for registers i = 0..31 (each load instruction
// reads 512 contiguous bytes).  A term's sign is the product of a tile part
// (uniform), a lane part and a register part (bits 6..10 of j); the first two
// are taken once per tile and term, and terms whose mask misses bits 6..10
// weigh all 32 registers alike.  Terms are ordered by observable.
//   EXPVAL: partial[b][block][o] = sum_j d_o(j) |psi_j|^2 over the block's tiles
//   LAMBDA: lam_j = (sum_o g[b,o] d_o(j)) psi_j
template <typename T, bool LAMBDA>
__global__ __launch_bounds__(256) void k_zdiag(const cx<T> *psi, cx<T> *lam, int n, const DTerm *terms, int t0, int t1,
                                              const double *gout, int nobs, double *partial) {
    __shared__ double red[4][ZD_MAXOBS];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t b = blockIdx.y;
    const cptr<DTerm> tp = to_const(terms);
    const cx<T> *p = psi + (b << n);
    double acc[ZD_MAXOBS];
    for (int o = 0; o < ZD_MAXOBS; ++o) acc[o] = 0.0;
    const int64_t ntiles = int64_t(1) << (n - 11);
    for (int64_t tile = (int64_t)blockIdx.x * 4 + wv; tile < ntiles; tile += (int64_t)gridDim.x * 4) {
        const uint64_t base = (uint64_t)tile << 11;
        cx<T> v[32];
        DQ_SF(32, { v[i] = p[base + 64 * i + lane]; });
        T d[32];
        DQ_SF(32, { d[i] = T(0); });
        int t = t0;
        while (t < t1) {
            const int o = tp[t].obs;
            T e[32];
            DQ_SF(32, { e[i] = T(0); });
            T ec = 0;   // terms that weigh every register alike
            for (; t < t1 && tp[t].obs == o; ++t) {
                const uint64_t z = tp[t].zmask;
                const int hs = __popcll(base & z) & 1, ls = __popc((unsigned)lane & (unsigned)z) & 1;
                const T c = ((hs ^ ls) ? T(-1) : T(1)) * (T)tp[t].wr;
                const unsigned zr = (unsigned)(z >> 6) & 31u;
                if (zr == 0) {
                    ec += c;
                } else {
                    DQ_SF(32, { e[i] += (__popc((unsigned)i & zr) & 1) ? -c : c; });
                }
            }
            if (LAMBDA) {
                const T g = (T)gout[b * nobs + o];
                DQ_SF(32, { d[i] += g * (e[i] + ec); });
            } else if (o < ZD_MAXOBS) {
                T s = 0;
                DQ_SF(32, { s += (e[i] + ec) * (v[i].x * v[i].x + v[i].y * v[i].y); });
                acc[o] += (double)s;
            }
        }
        if (LAMBDA) {
            cx<T> *q = lam + (b << n);
            DQ_SF(32, { q[base + 64 * i + lane] = cx<T>{d[i] * v[i].x, d[i] * v[i].y}; });
        }
    }
    if (!LAMBDA) {
        for (int o = 0; o < nobs && o < ZD_MAXOBS; ++o) {
            const double x = wave_sum(acc[o]);
            if (lane == 0) red[wv][o] = x;
        }
        __syncthreads();
        if (threadIdx.x < nobs && threadIdx.x < ZD_MAXOBS)
            partial[(b * gridDim.x + blockIdx.x) * nobs + threadIdx.x] =
                (red[0][threadIdx.x] + red[1][threadIdx.x]) + (red[2][threadIdx.x] + red[3][threadIdx.x]);
    }
}

__global__ void k_expval_final(const double *partial, int64_t batch, int eb, const DTerm *terms, int nterms,
                               int nobs, double *out, int skip0, int skip1, const double *dpart, int deb) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= batch * nobs) return;
    const int64_t b = i / nobs;
    const int o = (int)(i % nobs);
    double e = 0.0;
    if (dpart)   // the X-free group, summed by k_zdiag
        for (int k = 0; k < deb; ++k) e += dpart[(b * deb + k) * nobs + o];
    for (int t = 0; t < nterms; ++t) {
        const DTerm tm = terms[t];
        if (tm.obs != o || (t >= skip0 && t < skip1)) continue;
        double sr = 0.0, si = 0.0;
        for (int k = 0; k < eb; ++k) {
            sr += partial[((b * eb + k) * (int64_t)nterms + t) * 2];
            si += partial[((b * eb + k) * (int64_t)nterms + t) * 2 + 1];
        }
        e += tm.wr * sr - tm.wi * si;
    }
    out[i] = e;
}

// ---------------------------------------------------------------- one-bit X terms in tiles
// A wave owns tiles of 2048 amplitudes: lane l holds physical bits 0..5,
// register k the five bits S.rb, so tile t starts at t << 6 with zeros
// inserted at S.rb and every load reads 512 contiguous bytes.  A term X_h
// (times a Z string) pairs amplitudes inside the tile: across lanes when h
// is a lane bit (one backwards permute per register), across registers when
// h is one of S.rb.  The sign (-1)^{|j & z|} splits into the tile base
// (uniform), the lane and the register parts.
__device__ __forceinline__ int64_t xtile_base(int64_t t, const XSet &S) {
    int64_t b = t << 6;
#pragma unroll
    for (int r = 0; r < 5; ++r) b = insert_zero(b, S.rb[r]);
    return b;
}
__device__ __forceinline__ int64_t xtile_reg(int k, const XSet &S) {
    int64_t o = 0;
#pragma unroll
    for (int r = 0; r < 5; ++r)
        if ((k >> r) & 1) o += int64_t(1) << S.rb[r];
    return o;
}
// the register part of a Z mask: bit r set when z holds S.rb[r]
__device__ __forceinline__ int xtile_zr(uint64_t z, const XSet &S) {
    int m = 0;
#pragma unroll
    for (int r = 0; r < 5; ++r) m |= (int)((z >> S.rb[r]) & 1) << r;
    return m;
}
__device__ __forceinline__ C64 bperm_c64(C64 a, int addr) {
    return C64{__int_as_float(__builtin_amdgcn_ds_bpermute(addr, __float_as_int(a.x))),
               __int_as_float(__builtin_amdgcn_ds_bpermute(addr, __float_as_int(a.y)))};
}

// Partial sums S_t = sum_j (-1)^{|j & z_t|} conj(psi_{j^x}) psi_j of the
// set's terms (as expval_chunk: over the pair members j whose X bit is 0,
// doubled), one row per block: partial[b][block][t][2].  Per tile and term
// the wave's sum goes to a per-wave accumulator in LDS.
__global__ __launch_bounds__(256) void k_xtile_expval(const C64 *st, int n, XSet S, const XTerm *xts, const DTerm *terms,
                                                      int nterms, double *partial, int eb) {
    __shared__ double acc[4][2 * XT_MAX];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t b = blockIdx.y, N = int64_t(1) << n;
    const C64 *p = st + b * N;
    const int nx = S.x1 - S.x0;
    if (lane < 2 * XT_MAX) acc[wv][lane] = 0.0;
    const int64_t ntiles = N >> 11;
    for (int64_t t = blockIdx.x * 4 + wv; t < ntiles; t += (int64_t)eb * 4) {
        const int64_t base = xtile_base(t, S);
        C64 v[32];
#pragma unroll
        for (int k = 0; k < 32; ++k) v[k] = p[base + xtile_reg(k, S) + lane];
        for (int i = 0; i < nx; ++i) {
            const XTerm x = xts[S.x0 + i];
            const uint64_t z = terms[x.t].zmask;
            const int h = x.pos < 6 ? x.pos : S.rb[x.pos - 6];
            const bool odd = (z >> h) & 1;
            const int zr = xtile_zr(z, S);
            const int s0 = (__popcll((uint64_t)base & z) & 1) ^ (__popcll((uint64_t)lane & z) & 1);
            double sr = 0.0;
            if (x.pos < 6) {
                const int addr = (lane ^ (1 << x.pos)) << 2;
                const bool mine = !((lane >> x.pos) & 1);
#pragma unroll
                for (int k = 0; k < 32; ++k) {
                    const C64 o = bperm_c64(v[k], addr), a = v[k];
                    const double c = odd ? (double)(o.x * a.y - o.y * a.x) : (double)(o.x * a.x + o.y * a.y);
                    const bool neg = (s0 ^ __popc(k & zr)) & 1;
                    sr += neg ? -c : c;
                }
                if (!mine) sr = 0.0;
            } else {
#pragma unroll
                for (int r = 0; r < 5; ++r) {
                    if (x.pos != 6 + r) continue;
#pragma unroll
                    for (int k = 0; k < 32; ++k) {
                        if ((k >> r) & 1) continue;
                        const C64 a = v[k], o = v[k | (1 << r)];
                        const double c = odd ? (double)(o.x * a.y - o.y * a.x) : (double)(o.x * a.x + o.y * a.y);
                        const bool neg = (s0 ^ __popc(k & zr)) & 1;
                        sr += neg ? -c : c;
                    }
                }
            }
            sr = wave_sum(sr);
            if (lane == 0) acc[wv][2 * i + (odd ? 1 : 0)] += sr;
        }
    }
    __syncthreads();
    if (threadIdx.x < 2 * nx) {
        const int ti = xts[S.x0 + (threadIdx.x >> 1)].t;
        partial[((b * eb + blockIdx.x) * (int64_t)nterms + ti) * 2 + (threadIdx.x & 1)] =
            2.0 * ((acc[0][threadIdx.x] + acc[1][threadIdx.x]) + (acc[2][threadIdx.x] + acc[3][threadIdx.x]));
    }
}

// lambda_j (+)= sum over the set's terms of gout[b, obs_t] w_t
// (-1)^{|(j ^ x_t) & z_t|} psi_{j ^ x_t}; one tile per wave at a time.
__global__ __launch_bounds__(256) void k_xtile_lambda(const C64 *psi, C64 *lam, int n, int64_t batch, XSet S,
                                                      const XTerm *xts, const DTerm *terms, const double *gout, int nobs,
                                                      bool add) {
    const int lane = threadIdx.x & 63;
    const int nx = S.x1 - S.x0;
    const int64_t ntiles = batch << (n - 11);
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t t = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; t < ntiles; t += nw) {
        const int64_t b = t >> (n - 11);
        const int64_t base = (b << n) + xtile_base(t & ((int64_t(1) << (n - 11)) - 1), S);
        C64 v[32], l[32];
#pragma unroll
        for (int k = 0; k < 32; ++k) {
            v[k] = psi[base + xtile_reg(k, S) + lane];
            l[k] = add ? lam[base + xtile_reg(k, S) + lane] : C64{0.f, 0.f};
        }
        for (int i = 0; i < nx; ++i) {
            const XTerm x = xts[S.x0 + i];
            const DTerm tm = terms[x.t];
            const double g = gout[b * nobs + tm.obs];
            const float wr = (float)(g * tm.wr), wi = (float)(g * tm.wi);
            const int h = x.pos < 6 ? x.pos : S.rb[x.pos - 6];
            // sign of the partner j ^ x: (-1)^{|j & z|} times (-1)^{z_h}
            const int s0 = (__popcll((uint64_t)base & tm.zmask) & 1) ^ (__popcll((uint64_t)lane & tm.zmask) & 1) ^
                           (int)((tm.zmask >> h) & 1);
            const int zr = xtile_zr(tm.zmask, S);
            if (x.pos < 6) {
                const int addr = (lane ^ (1 << x.pos)) << 2;
#pragma unroll
                for (int k = 0; k < 32; ++k) {
                    const C64 o = bperm_c64(v[k], addr);
                    const bool neg = (s0 ^ __popc(k & zr)) & 1;
                    const float dr = neg ? -wr : wr, di = neg ? -wi : wi;
                    l[k] = C64{l[k].x + (dr * o.x - di * o.y), l[k].y + (dr * o.y + di * o.x)};
                }
            } else {
#pragma unroll
                for (int r = 0; r < 5; ++r) {
                    if (x.pos != 6 + r) continue;
#pragma unroll
                    for (int k = 0; k < 32; ++k) {
                        const C64 o = v[k ^ (1 << r)];
                        const bool neg = (s0 ^ __popc(k & zr)) & 1;
                        const float dr = neg ? -wr : wr, di = neg ? -wi : wi;
                        l[k] = C64{l[k].x + (dr * o.x - di * o.y), l[k].y + (dr * o.y + di * o.x)};
                    }
                }
            }
        }
#pragma unroll
        for (int k = 0; k < 32; ++k) lam[base + xtile_reg(k, S) + lane] = l[k];
    }
}

// lambda_j = sum_k gout[b, obs_k] * coef_k i^{nY_k} (-1)^{|(j^x_k) & z_k|} psi_{j ^ x_k}
// (for the X-free group the terms collapse into one factor d(j) psi_j)
template <typename T>
__global__ __launch_bounds__(256) void k_lambda(const cx<T> *psi, cx<T> *lam, int n, int64_t total, const DGroup *groups,
                                                int g0, int ngroups, const DTerm *terms, const double *gout, int nobs, bool add) {
    const int64_t mask = (int64_t(1) << n) - 1;
    const cptr<DGroup> gp = to_const(groups);
    const cptr<DTerm> tp = to_const(terms);
    const cptr<double> go = to_const(gout);
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t b = i >> n, j = i & mask;
        const cx<T> *p = psi + (b << n);
        double ar = 0.0, ai = 0.0;
        for (int g = g0; g < ngroups; ++g) {
            const uint64_t x = gp[g].xmask;
            const int t0 = gp[g].t0, t1 = gp[g].t1;
            const int64_t jx = j ^ (int64_t)x;
            // d = sum_t w_t (-1)^{|jx & z_t|}, w_t = gout[b, obs_t] * coef_t i^{nY_t}
            double dr = 0.0, di = 0.0;
            for (int t = t0; t < t1; ++t) {
                const double w = go[b * nobs + tp[t].obs];
                const double wr = w * tp[t].wr, wi = w * tp[t].wi;
                const bool neg = __popcll((uint64_t)jx & tp[t].zmask) & 1;
                dr += neg ? -wr : wr;
                di += neg ? -wi : wi;
            }
            const cx<T> o = p[jx];
            const double ox = (double)o.x, oy = (double)o.y;
            ar += dr * ox - di * oy;
            ai += dr * oy + di * ox;
        }
        if (add) {
            ar += (double)lam[i].x;
            ai += (double)lam[i].y;
        }
        lam[i] = cx<T>{(T)ar, (T)ai};
    }
}

// Uneven batches: every circuit's adjoint seed in one launch; amplitude i of
// the concatenated circuits belongs to the entry whose [amp_begin, amp_begin
// + 2^n) holds it; weights at gout + out_off.  Every circuit holds a multiple
// of 64 amplitudes (n >= 6), so the 64 amplitudes of a wave belong to one
// circuit: the wave looks up its entry, terms and weights once, with scalar
// loads, instead of every lane searching the entries.
template <typename T>
__global__ __launch_bounds__(256) void k_lambda_multi(const cx<T> *st, char *ws, const MExp *ents, int nent,
                                                      int64_t total, const double *gout) {
    const cptr<MExp> ep = to_const(ents);
    const int lane = threadIdx.x & 63;
    const int64_t wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i0 = (int64_t)blockIdx.x * blockDim.x + 64 * wv; i0 < total; i0 += stride) {
        int lo = 0, hi = nent - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (ep[mid].amp_begin <= i0) lo = mid;
            else hi = mid - 1;
        }
        const int64_t i = i0 + lane;
        if (i >= total) continue;
        const int64_t j = i - ep[lo].amp_begin;
        const cx<T> *p = st + ep[lo].st_off;
        const cptr<DGroup> gp = to_const(ep[lo].groups);
        const cptr<DTerm> tp = to_const(ep[lo].terms);
        const cptr<double> go = to_const(gout + ep[lo].out_off);
        const int ng = ep[lo].ngroups;
        double ar = 0.0, ai = 0.0;
        for (int g = 0; g < ng; ++g) {
            const uint64_t x = gp[g].xmask;
            const int64_t jx = j ^ (int64_t)x;
            double dr = 0.0, di = 0.0;
            for (int t = gp[g].t0; t < gp[g].t1; ++t) {
                const double w = go[tp[t].obs];
                const double wr = tp[t].wr, wi = tp[t].wi;
                const bool neg = __popcll((uint64_t)jx & tp[t].zmask) & 1;
                dr += neg ? -w * wr : w * wr;
                di += neg ? -w * wi : w * wi;
            }
            const cx<T> o = p[jx];
            ar += dr * (double)o.x - di * (double)o.y;
            ai += dr * (double)o.y + di * (double)o.x;
        }
        ((cx<T> *)(ws + ep[lo].lam_off))[j] = cx<T>{(T)ar, (T)ai};
    }
}

// Uneven batches: every circuit's parameter gradients in one launch, one
// wave per output (unit u = packed parameter index): the wave's lanes take
// the per-wave partial sums w = lane, lane + 64, ... of each gradient slot of
// the parameter, weighted by its chain factor, then a fixed shuffle tree
// adds the lanes (deterministic).
__global__ __launch_bounds__(256) void k_grad_final_multi(const char *ws, const MGrad *ents, int nent, int64_t total,
                                                          double *out) {
    const int lane = threadIdx.x & 63;
    const int64_t u = blockIdx.x * (int64_t)(blockDim.x >> 6) + (threadIdx.x >> 6);
    if (u >= total) return;   // wave-uniform
    const int e = find_unit(ents, nent, u);
    const MGrad E = ents[e];
    const int64_t p = u - E.unit_begin;
    const double *part = (const double *)(ws + E.part_off);
    double s = 0.0;
    for (int64_t k = E.poff[p]; k < E.poff[p + 1]; ++k) {
        const int g = E.pg[k];
        double t = 0.0;
        for (int w = lane; w < E.wps; w += 64) t += part[(int64_t)w * E.ngrad + g];
        s += E.pf[k] * t;
    }
    s = wave_sum(s);
    if (lane == 0) out[E.par_off + p] = s;
}

}  // namespace

// ============================================================ launchers
// ============================================================ measurement
// Marginal probabilities.  Block (x, o, b) sums |psi_b[j]|^2 over chunk x of
// the basis states whose measured bits read o: j is the chunk index r with
// zeros inserted at the measured physical bits (ascending) and o's bits set
// there, so consecutive threads read consecutive amplitudes whenever the
// measured bits lie above the low ones.  One partial per block, summed in a
// fixed order by k_probs_final.
template <typename T>
__global__ __launch_bounds__(256) void k_probs_part(const cx<T> *psi, ProbArgs a, int64_t per_outcome,
                                                    double *partial, int64_t bpo) {
    __shared__ double red[4];
    const int64_t o = blockIdx.y, b = blockIdx.z;
    const int K = 1 << a.k;
    uint64_t set = 0;
    for (int i = 0; i < a.k; ++i)
        if ((o >> (a.k - 1 - i)) & 1) set |= 1ull << a.pb[i];
    const cx<T> *p = psi + (b << a.n);
    double acc = 0.0;
    const int64_t r0 = (int64_t)blockIdx.x * PROB_CHUNK + threadIdx.x;
#pragma unroll 4
    for (int t = 0; t < (int)(PROB_CHUNK / 256); ++t) {
        const int64_t r = r0 + t * 256;
        if (r < per_outcome) {
            int64_t j = r;
            for (int i = 0; i < a.k; ++i) j = insert_zero(j, a.asc[i]);
            const cx<T> v = p[(uint64_t)j | set];
            acc += (double)v.x * (double)v.x + (double)v.y * (double)v.y;
        }
    }
    acc = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) partial[(b * K + o) * bpo + blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

// out[row] = sum of the row's bpo partials (row = b * 2^k + o), fixed order
__global__ __launch_bounds__(256) void k_probs_final(const double *partial, int64_t bpo, double *out) {
    __shared__ double red[4];
    const int64_t row = blockIdx.x;
    double acc = 0.0;
    for (int64_t i = threadIdx.x; i < bpo; i += 256) acc += partial[row * bpo + i];
    acc = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) out[row] = (red[0] + red[1]) + (red[2] + red[3]);
}

// One shot per thread: the first outcome whose running sum exceeds u.
__global__ __launch_bounds__(256) void k_sample(const double *p, int64_t batch, int nout, const double *u, int shots,
                                                int64_t *out) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= batch * shots) return;
    const double *q = p + (i / shots) * nout;
    const double x = u[i];
    double c = 0.0;
    int64_t last = -1, res = -1;
    for (int m = 0; m < nout; ++m) {
        const double pm = q[m];
        if (pm > 0.0) last = m;
        c += pm;
        if (x < c) {
            res = m;
            break;
        }
    }
    out[i] = res >= 0 ? res : (last >= 0 ? last : 0);
}

#define DQ_LAUNCH_RET return hipGetLastError()

hipError_t launch_prepare(int dbl, const DGate *gates, const void *fixed, const DSlot *slots, int32_t nslots,
                          const double *params, int64_t pstride, const double *data, int64_t dstride, void *mats,
                          int64_t block, int64_t bm, hipStream_t s) {
    if (nslots <= 0) return hipSuccess;
    dim3 grid((nslots + 63) / 64, (unsigned)bm);
    if (dbl)
        hipLaunchKernelGGL(k_prepare<double>, grid, dim3(64), 0, s, gates, (const double2 *)fixed, slots, nslots,
                           params, pstride, data, dstride, (C128 *)mats, block);
    else
        hipLaunchKernelGGL(k_prepare<float>, grid, dim3(64), 0, s, gates, (const double2 *)fixed, slots, nslots,
                           params, pstride, data, dstride, (C64 *)mats, block);
    DQ_LAUNCH_RET;
}

hipError_t launch_prepare_blocks(int dbl, const DGate *gates, const void *fixed, const DBlock *blocks, int32_t nblocks,
                                 const int32_t *factors, const double *params, int64_t pstride, const double *data,
                                 int64_t dstride, void *mats, int64_t block, int64_t bm, hipStream_t s) {
    if (nblocks <= 0) return hipSuccess;
    dim3 grid((unsigned)nblocks, (unsigned)bm);
    if (dbl)
        hipLaunchKernelGGL(k_prepare_block<double>, grid, dim3(32), 0, s, gates, (const double2 *)fixed, blocks, factors,
                           params, pstride, data, dstride, (C128 *)mats, block);
    else
        hipLaunchKernelGGL(k_prepare_block<float>, grid, dim3(32), 0, s, gates, (const double2 *)fixed, blocks, factors,
                           params, pstride, data, dstride, (C64 *)mats, block);
    DQ_LAUNCH_RET;
}

hipError_t launch_init_zero(int dbl, void *st, int32_t n, int64_t batch, hipStream_t s) {
    const int64_t total = batch << n;
    if (dbl) hipLaunchKernelGGL(k_init_zero<double>, dim3(grid_for(total, 256)), dim3(256), 0, s, (C128 *)st, n, total);
    else hipLaunchKernelGGL(k_init_zero<float>, dim3(grid_for(total, 256)), dim3(256), 0, s, (C64 *)st, n, total);
    DQ_LAUNCH_RET;
}

hipError_t launch_init_copy(int dbl, void *st, const void *init, int32_t n, int64_t batch, hipStream_t s) {
    const int64_t total = batch << n;
    if (dbl)
        hipLaunchKernelGGL(k_init_copy<double>, dim3(grid_for(total, 256)), dim3(256), 0, s, (C128 *)st,
                           (const C128 *)init, n, total);
    else
        hipLaunchKernelGGL(k_init_copy<float>, dim3(grid_for(total, 256)), dim3(256), 0, s, (C64 *)st,
                           (const C64 *)init, n, total);
    DQ_LAUNCH_RET;
}

hipError_t launch_copy(int dbl, void *dst, const void *src, int64_t count, hipStream_t s) {
    if (dbl)
        hipLaunchKernelGGL(k_copy<double>, dim3(grid_for(count, 256)), dim3(256), 0, s, (C128 *)dst,
                           (const C128 *)src, count);
    else
        hipLaunchKernelGGL(k_copy<float>, dim3(grid_for(count, 256)), dim3(256), 0, s, (C64 *)dst,
                           (const C64 *)src, count);
    DQ_LAUNCH_RET;
}

template <typename T, typename M>
static void init_product(void *st, int32_t n, int64_t batch, const void *mats, int64_t mstride,
                         const int64_t *fold_off, hipStream_t s) {
    const int64_t N = int64_t(1) << n;
    if (n >= 16) {
        const int64_t nblk = N >> 16;
        dim3 grid((unsigned)(nblk < 4096 ? nblk : 4096), (unsigned)batch);
        hipLaunchKernelGGL((k_init_product_tab<T, M>), grid, dim3(256), 0, s, (cx<T> *)st, n, (const cx<M> *)mats,
                           mstride, fold_off);
        return;
    }
    dim3 grid(grid_for(N, 256, 8192), (unsigned)batch);
    hipLaunchKernelGGL((k_init_product<T, M>), grid, dim3(256), 0, s, (cx<T> *)st, n, (const cx<M> *)mats, mstride,
                       fold_off);
}

hipError_t launch_init_product(int dbl, int mdbl, void *st, int32_t n, int64_t batch, const void *mats,
                               int64_t mstride, const int64_t *fold_off, hipStream_t s) {
    if (dbl) init_product<double, double>(st, n, batch, mats, mstride, fold_off, s);
    else if (mdbl) init_product<float, double>(st, n, batch, mats, mstride, fold_off, s);
    else init_product<float, float>(st, n, batch, mats, mstride, fold_off, s);
    DQ_LAUNCH_RET;
}

hipError_t launch_gate1(int dbl, void *st, int32_t n, int64_t batch, int32_t bit, const void *mats, int64_t mstride,
                        int64_t off, hipStream_t s) {
    const int64_t total = batch << (n - 1);
    if (dbl)
        hipLaunchKernelGGL(k_gate1<double>, dim3(grid_for(total, 256)), dim3(256), 0, s, (C128 *)st, n, total, bit,
                           (const C128 *)mats, mstride, off);
    else
        hipLaunchKernelGGL(k_gate1<float>, dim3(grid_for(total, 256)), dim3(256), 0, s, (C64 *)st, n, total, bit,
                           (const C64 *)mats, mstride, off);
    DQ_LAUNCH_RET;
}

hipError_t launch_cnot(int dbl, void *st, int32_t n, int64_t batch, int32_t cbit, int32_t tbit, hipStream_t s) {
    const int64_t total = batch << (n - 2);
    if (dbl)
        hipLaunchKernelGGL(k_cnot<double>, dim3(grid_for(total, 256)), dim3(256), 0, s, (C128 *)st, n, total, cbit, tbit);
    else
        hipLaunchKernelGGL(k_cnot<float>, dim3(grid_for(total, 256)), dim3(256), 0, s, (C64 *)st, n, total, cbit, tbit);
    DQ_LAUNCH_RET;
}

hipError_t launch_cz(int dbl, void *st, int32_t n, int64_t batch, int32_t abit, int32_t bbit, hipStream_t s) {
    const int64_t total = batch << (n - 2);
    if (dbl)
        hipLaunchKernelGGL(k_cz<double>, dim3(grid_for(total, 256)), dim3(256), 0, s, (C128 *)st, n, total, abit, bbit);
    else
        hipLaunchKernelGGL(k_cz<float>, dim3(grid_for(total, 256)), dim3(256), 0, s, (C64 *)st, n, total, abit, bbit);
    DQ_LAUNCH_RET;
}

template <typename T>
static void gatek_t(cx<T> *st, int32_t n, int64_t batch, int32_t k, const KBits &kb, const cx<T> *mats,
                    int64_t mstride, int64_t off, hipStream_t s) {
    const int64_t total = batch << (n - k);
    dim3 g(grid_for(total, 256)), blk(256);
    switch (k) {
    case 1: hipLaunchKernelGGL((k_gatek<T, 1>), g, blk, 0, s, st, n, total, kb, mats, mstride, off); break;
    case 2: hipLaunchKernelGGL((k_gatek<T, 2>), g, blk, 0, s, st, n, total, kb, mats, mstride, off); break;
    case 3: hipLaunchKernelGGL((k_gatek<T, 3>), g, blk, 0, s, st, n, total, kb, mats, mstride, off); break;
    case 4: hipLaunchKernelGGL((k_gatek<T, 4>), g, blk, 0, s, st, n, total, kb, mats, mstride, off); break;
    default: hipLaunchKernelGGL((k_gatek<T, 5>), g, blk, 0, s, st, n, total, kb, mats, mstride, off); break;
    }
}

hipError_t launch_gatek(int dbl, void *st, int32_t n, int64_t batch, int32_t k, const int32_t *bits, const void *mats,
                        int64_t mstride, int64_t off, hipStream_t s) {
    KBits kb;
    for (int t = 0; t < 5; ++t) kb.bits[t] = kb.sorted[t] = t < k ? bits[t] : 0;
    for (int a = 0; a < k; ++a)   // insertion sort, ascending
        for (int b = a + 1; b < k; ++b)
            if (kb.sorted[b] < kb.sorted[a]) { int t = kb.sorted[a]; kb.sorted[a] = kb.sorted[b]; kb.sorted[b] = t; }
    if (dbl) gatek_t<double>((C128 *)st, n, batch, k, kb, (const C128 *)mats, mstride, off, s);
    else gatek_t<float>((C64 *)st, n, batch, k, kb, (const C64 *)mats, mstride, off, s);
    DQ_LAUNCH_RET;
}

hipError_t launch_dense(int dbl, void *st, int32_t n, int64_t batch, int32_t k, const int32_t *bits, const void *mats,
                        int64_t mstride, int64_t off, hipStream_t s) {
    DenseBits db;
    for (int t = 0; t < 5; ++t) db.bits[t] = db.sorted[t] = t < k ? bits[t] : 0;
    for (int a = 0; a < k; ++a)
        for (int b = a + 1; b < k; ++b)
            if (db.sorted[b] < db.sorted[a]) { int t = db.sorted[a]; db.sorted[a] = db.sorted[b]; db.sorted[b] = t; }
    const int colbits = dbl ? 4 : 5;
    if (k < 4 || k > 5 || n < k + colbits) return hipErrorInvalidValue;
    const int64_t groups = batch << (n - k - colbits);
    const unsigned grid = grid_for(groups * 64, 256, 4096);
    if (dbl) {
        if (k == 4) hipLaunchKernelGGL(k_dense_f64<4>, dim3(grid), dim3(256), 0, s, (C128 *)st, n, groups, db, (const C128 *)mats, mstride, off);
        else hipLaunchKernelGGL(k_dense_f64<5>, dim3(grid), dim3(256), 0, s, (C128 *)st, n, groups, db, (const C128 *)mats, mstride, off);
    } else {
        // through LDS with 16-byte coalesced accesses (16-byte aligned states):
        // a block inside the low K + 5 bits (each group one contiguous run),
        // or a 5-qubit block that leaves physical bit 0 to the columns
        // (adjacent pairs; 4-qubit blocks there ran 3 % faster directly)
        const bool aligned = ((uintptr_t)st & 15) == 0;
        const bool contiguous = aligned && db.sorted[k - 1] < k + 5;
        const bool pairs = aligned && !contiguous && db.sorted[0] > 0 && k == 5;
        const unsigned lgrid = (unsigned)(groups < 16384 ? groups : 16384);
        const C64 *m = (const C64 *)mats;
        if (contiguous && k == 4) hipLaunchKernelGGL((k_dense_f32_lds<4, true>), dim3(lgrid), dim3(64), 0, s, (C64 *)st, n, groups, db, m, mstride, off);
        else if (contiguous) hipLaunchKernelGGL((k_dense_f32_lds<5, true>), dim3(lgrid), dim3(64), 0, s, (C64 *)st, n, groups, db, m, mstride, off);
        else if (pairs) hipLaunchKernelGGL((k_dense_f32_lds<5, false>), dim3(lgrid), dim3(64), 0, s, (C64 *)st, n, groups, db, m, mstride, off);
        else if (k == 4) hipLaunchKernelGGL(k_dense_f32<4>, dim3(grid), dim3(256), 0, s, (C64 *)st, n, groups, db, m, mstride, off);
        else hipLaunchKernelGGL(k_dense_f32<5>, dim3(grid), dim3(256), 0, s, (C64 *)st, n, groups, db, m, mstride, off);
    }
    DQ_LAUNCH_RET;
}

hipError_t launch_tile_fwd(int dbl, const TileArgs &a, hipStream_t s) {
    return dbl ? tile_fwd_f64(a, s) : tile_fwd_f32(a, s);
}

hipError_t launch_tile_adj(int dbl, const TileArgs &a, hipStream_t s) {
    if (a.nlslots > MAX_LSLOTS) return hipErrorInvalidValue;
    return dbl ? tile_adj_f64(a, s) : tile_adj_f32(a, s);
}

int tile_adj_capacity(int dbl, int R) { return dbl ? tile_adj_capacity_f64(R) : tile_adj_capacity_f32(R); }

hipError_t launch_tile_fwd_multi(int dbl, int R, void *st, const void *ws, const MultiEntry *ents, int32_t nent,
                                 int64_t units, hipStream_t s) {
    if (units <= 0) return hipSuccess;
    return dbl ? tile_fwd_multi_f64(R, st, ws, ents, nent, units, s) : tile_fwd_multi_f32(R, st, ws, ents, nent, units, s);
}

hipError_t launch_tile_adj_multi(int dbl, int R, void *st, void *ws, const MultiEntry *ents, int32_t nent,
                                 int64_t units, int32_t max_nls, hipStream_t s) {
    if (units <= 0) return hipSuccess;
    if (max_nls > MAX_LSLOTS || units > 0x7fffffff) return hipErrorInvalidValue;
    const size_t lds = sizeof(double) * 64 * (max_nls > 0 ? max_nls : 1);
    return dbl ? tile_adj_multi_f64(R, st, ws, ents, nent, units, lds, s)
               : tile_adj_multi_f32(R, st, ws, ents, nent, units, lds, s);
}

hipError_t launch_grad_gate(int dbl, const void *psi, const void *lam, int32_t n, int64_t batch, int32_t gen,
                            int32_t bit0, int32_t bit1, double *partial, int32_t wps, int32_t ngrad, int32_t gslot,
                            hipStream_t s) {
    dim3 g((unsigned)wps, (unsigned)batch);
    if (dbl)
        hipLaunchKernelGGL(k_grad_gate<double>, g, dim3(256), 0, s, (const C128 *)psi, (const C128 *)lam, n, gen,
                           bit0, bit1, partial, wps, ngrad, gslot);
    else
        hipLaunchKernelGGL(k_grad_gate<float>, g, dim3(256), 0, s, (const C64 *)psi, (const C64 *)lam, n, gen,
                           bit0, bit1, partial, wps, ngrad, gslot);
    DQ_LAUNCH_RET;
}

hipError_t launch_grad_final(const double *partial, int64_t batch, int32_t wps, int32_t ngrad, const int64_t *csr_off,
                             const int32_t *csr_g, const double *csr_f, int64_t nout, int32_t per_sample, double *out,
                             hipStream_t s) {
    const int64_t total = per_sample ? batch * nout : nout;
    if (total <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_grad_final, dim3((unsigned)((total + 127) / 128)), dim3(128), 0, s, partial, batch, wps, ngrad,
                       csr_off, csr_g, csr_f, nout, per_sample, out);
    DQ_LAUNCH_RET;
}

hipError_t launch_prepare_multi(int dbl, const MPrep *ents, int32_t nent, int32_t max_slots, const double *params,
                                void *ws, hipStream_t s) {
    if (nent <= 0 || max_slots <= 0) return hipSuccess;
    dim3 grid((unsigned)((max_slots + 63) / 64), (unsigned)nent);
    if (dbl) hipLaunchKernelGGL(k_prepare_multi<double>, grid, dim3(64), 0, s, ents, params, (char *)ws);
    else hipLaunchKernelGGL(k_prepare_multi<float>, grid, dim3(64), 0, s, ents, params, (char *)ws);
    DQ_LAUNCH_RET;
}

hipError_t launch_init_multi(int dbl, void *st, const void *ws, const MInit *ents, int32_t nent, int32_t max_n,
                             hipStream_t s) {
    if (nent <= 0) return hipSuccess;
    const int64_t N = int64_t(1) << max_n;
    dim3 grid(grid_for(N, 256, 4096), (unsigned)nent);
    if (dbl) hipLaunchKernelGGL(k_init_multi<double>, grid, dim3(256), 0, s, (C128 *)st, (const char *)ws, ents);
    else hipLaunchKernelGGL(k_init_multi<float>, grid, dim3(256), 0, s, (C64 *)st, (const char *)ws, ents);
    DQ_LAUNCH_RET;
}

hipError_t launch_expval_multi(int dbl, const void *st, void *ws, const MExp *ents, int32_t nent, int64_t units,
                               int32_t max_group, double *out, hipStream_t s) {
    if (nent <= 0) return hipSuccess;
    const bool narrow = max_group <= 4;
    if (dbl && narrow)
        hipLaunchKernelGGL((k_expval_multi<double, 4>), dim3((unsigned)units), dim3(256), 0, s, (const C128 *)st,
                           (char *)ws, ents, nent);
    else if (dbl)
        hipLaunchKernelGGL((k_expval_multi<double, EXP_TM>), dim3((unsigned)units), dim3(256), 0, s, (const C128 *)st,
                           (char *)ws, ents, nent);
    else if (narrow)
        hipLaunchKernelGGL((k_expval_multi<float, 4>), dim3((unsigned)units), dim3(256), 0, s, (const C64 *)st,
                           (char *)ws, ents, nent);
    else
        hipLaunchKernelGGL((k_expval_multi<float, EXP_TM>), dim3((unsigned)units), dim3(256), 0, s, (const C64 *)st,
                           (char *)ws, ents, nent);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_expval_final_multi, dim3((unsigned)nent), dim3(64), 0, s, (const char *)ws, ents, out);
    DQ_LAUNCH_RET;
}

hipError_t launch_lambda_multi(int dbl, const void *st, void *ws, const MExp *ents, int32_t nent, int64_t total,
                               const double *gout, hipStream_t s) {
    if (nent <= 0) return hipSuccess;
    if (dbl)
        hipLaunchKernelGGL(k_lambda_multi<double>, dim3(grid_for(total, 256)), dim3(256), 0, s, (const C128 *)st,
                           (char *)ws, ents, nent, total, gout);
    else
        hipLaunchKernelGGL(k_lambda_multi<float>, dim3(grid_for(total, 256)), dim3(256), 0, s, (const C64 *)st,
                           (char *)ws, ents, nent, total, gout);
    DQ_LAUNCH_RET;
}

hipError_t launch_grad_final_multi(const void *ws, const MGrad *ents, int32_t nent, int64_t total, double *out,
                                   hipStream_t s) {
    if (nent <= 0 || total <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_grad_final_multi, dim3((unsigned)((total + 3) / 4)), dim3(256), 0, s, (const char *)ws, ents,
                       nent, total, out);
    DQ_LAUNCH_RET;
}

hipError_t launch_hess_rows(const double *params, const int32_t *occ_param, const double *occ_scale, int64_t K,
                            int64_t c0, int64_t mc, double *rows, hipStream_t s) {
    const int64_t total = 2 * mc * K;
    if (total <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_hess_rows, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, params, occ_param,
                       occ_scale, K, c0, mc, rows);
    DQ_LAUNCH_RET;
}

hipError_t launch_bcast_rows(const double *w, int32_t nobs, int64_t rows, double *out, hipStream_t s) {
    const int64_t total = rows * nobs;
    if (total <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_bcast_rows, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, w, nobs, rows, out);
    DQ_LAUNCH_RET;
}

hipError_t launch_hess_accum(const double *G, int64_t K, int64_t c0, int64_t mc, const int64_t *poff,
                             const int32_t *pocc, const double *occ_scale, int64_t P, double *H, hipStream_t s) {
    const int64_t total = P * P;
    if (total <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_hess_accum, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, G, K, c0, mc, poff,
                       pocc, occ_scale, P, H);
    DQ_LAUNCH_RET;
}

hipError_t launch_probs(int dbl, const void *st, int64_t batch, const ProbArgs &a, double *partial, int64_t bpo,
                        double *out, hipStream_t s) {
    const int64_t per_outcome = int64_t(1) << (a.n - a.k);
    dim3 g((unsigned)bpo, (unsigned)(1u << a.k), (unsigned)batch);
    if (dbl)
        hipLaunchKernelGGL(k_probs_part<double>, g, dim3(256), 0, s, (const C128 *)st, a, per_outcome, partial, bpo);
    else
        hipLaunchKernelGGL(k_probs_part<float>, g, dim3(256), 0, s, (const C64 *)st, a, per_outcome, partial, bpo);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_probs_final, dim3((unsigned)(batch << a.k)), dim3(256), 0, s, (const double *)partial, bpo,
                       out);
    DQ_LAUNCH_RET;
}

hipError_t launch_sample(const double *p, int64_t batch, int32_t nout, const double *u, int32_t shots, int64_t *out,
                         hipStream_t s) {
    const int64_t total = batch * shots;
    hipLaunchKernelGGL(k_sample, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, p, batch, nout, u, shots,
                       out);
    DQ_LAUNCH_RET;
}

hipError_t launch_expval(int dbl, const void *st, int32_t n, int64_t batch, const DGroup *groups, int32_t ngroups,
                         const DTerm *terms, int32_t nterms, int32_t nobs, double *partial, int32_t eb, double *out,
                         int32_t dt0, int32_t dt1, double *dpart, const XSet *xs, int32_t nxs, const XTerm *xt,
                         hipStream_t s) {
    if (nxs > 0 && (dbl || n < 11)) return hipErrorInvalidValue;
    for (int k = 0; k < nxs; ++k)
        hipLaunchKernelGGL(k_xtile_expval, dim3((unsigned)eb, (unsigned)batch), dim3(256), 0, s, (const C64 *)st, n, xs[k],
                           xt, terms, nterms, partial, eb);
    // the X-free group (terms dt0..dt1, group 0) by k_zdiag when dt0 < dt1
    const bool zd = dt0 < dt1;
    const int deb = zd ? zdiag_blocks(n) : 0;
    if (zd) {
        dim3 g((unsigned)deb, (unsigned)batch);
        if (dbl)
            hipLaunchKernelGGL((k_zdiag<double, false>), g, dim3(256), 0, s, (const C128 *)st, (C128 *)nullptr, n, terms,
                               dt0, dt1, (const double *)nullptr, nobs, dpart);
        else
            hipLaunchKernelGGL((k_zdiag<float, false>), g, dim3(256), 0, s, (const C64 *)st, (C64 *)nullptr, n, terms,
                               dt0, dt1, (const double *)nullptr, nobs, dpart);
    }
    const int g0 = zd ? 1 : 0;
    if (ngroups > g0) {
        dim3 g((unsigned)eb, (unsigned)batch);
        if (dbl)
            hipLaunchKernelGGL(k_expval_part<double>, g, dim3(256), 0, s, (const C128 *)st, n, groups, g0, ngroups, terms,
                               nterms, partial, eb);
        else
            hipLaunchKernelGGL(k_expval_part<float>, g, dim3(256), 0, s, (const C64 *)st, n, groups, g0, ngroups, terms,
                               nterms, partial, eb);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t total = batch * nobs;
    hipLaunchKernelGGL(k_expval_final, dim3((unsigned)((total + 127) / 128)), dim3(128), 0, s, partial, batch, eb,
                       terms, nterms, nobs, out, zd ? dt0 : 0, zd ? dt1 : 0, zd ? (const double *)dpart : nullptr, deb);
    DQ_LAUNCH_RET;
}

hipError_t launch_lambda(int dbl, const void *psi, void *lam, int32_t n, int64_t batch, const DGroup *groups,
                         int32_t ngroups, const DTerm *terms, const double *grad_out, int32_t nobs, int32_t dt0, int32_t dt1,
                         const XSet *xs, int32_t nxs, const XTerm *xt, hipStream_t s) {
    if (nxs > 0 && (dbl || n < 11)) return hipErrorInvalidValue;
    const int64_t total = batch << n;
    const bool zd = dt0 < dt1;   // the X-free group (terms dt0..dt1, group 0) by k_zdiag
    const int g0 = zd ? 1 : 0;
    // the one-bit-X tile sets after the pair groups, each adding to lambda
    auto tiles = [&](bool add) {
        const int64_t waves = batch << (n - 11);
        const unsigned g = (unsigned)((waves + 3) / 4 < 4096 ? (waves + 3) / 4 : 4096);
        for (int k = 0; k < nxs; ++k)
            hipLaunchKernelGGL(k_xtile_lambda, dim3(g), dim3(256), 0, s, (const C64 *)psi, (C64 *)lam, n, batch, xs[k], xt,
                               terms, grad_out, nobs, add || k > 0);
    };
    if (zd) {
        const int64_t q = (int64_t(1) << (n - 11)) / 4;
        dim3 g((unsigned)(q < 1 ? 1 : (q < 4096 ? q : 4096)), (unsigned)batch);
        if (dbl)
            hipLaunchKernelGGL((k_zdiag<double, true>), g, dim3(256), 0, s, (const C128 *)psi, (C128 *)lam, n, terms,
                               dt0, dt1, grad_out, nobs, (double *)nullptr);
        else
            hipLaunchKernelGGL((k_zdiag<float, true>), g, dim3(256), 0, s, (const C64 *)psi, (C64 *)lam, n, terms,
                               dt0, dt1, grad_out, nobs, (double *)nullptr);
        if (ngroups <= 1) {
            tiles(true);
            DQ_LAUNCH_RET;
        }
    }
    if (ngroups > g0 || (!zd && nxs == 0)) {
        if (dbl)
            hipLaunchKernelGGL(k_lambda<double>, dim3(grid_for(total, 256)), dim3(256), 0, s, (const C128 *)psi,
                               (C128 *)lam, n, total, groups, g0, ngroups, terms, grad_out, nobs, zd);
        else
            hipLaunchKernelGGL(k_lambda<float>, dim3(grid_for(total, 256)), dim3(256), 0, s, (const C64 *)psi,
                               (C64 *)lam, n, total, groups, g0, ngroups, terms, grad_out, nobs, zd);
    }
    tiles(zd || ngroups > g0);
    DQ_LAUNCH_RET;
}

}  // namespace dq
